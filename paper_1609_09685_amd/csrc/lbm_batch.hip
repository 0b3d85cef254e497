// Batches of independent domains behind the lbm_batch_* entry points of
// include/lbm.h.
//
// One kernel launch per time step covers every running sample.  The launch is
// described by tables in the caller's batch work buffer:
//   args    StepArgs<T> [2 n]     arguments of sample d at its current parity
//                                 (entry 2d) and at the other one (2d + 1)
//   owner   int2 [cap]            block b of the launch -> (sample, block of the
//                                 sample's own grid), or (-1, 0)
//   reduce  two sets of per-sample pointers, partial counts and chunk tables,
//           one for the flux of the step kernel (one partial per bitmap word)
//           and one for the flux pass (one partial per 256 slots)
//   q       double [n]            reduced flux of every sample
// Each sample's stretch of the owner table starts at a multiple of 8 and
// lists its blocks in hardware order, so the XCD that runs a block is the one
// the sample's own launch would use: the tile orders (banded, remapped) carry
// over unchanged, and so does every bit of the arithmetic.
//
// Retiring a sample rewrites the owner table without its blocks (the tail is
// filled with (-1, 0) up to the size of the captured graph's launch); the
// window graph reads the table from device memory, so it is recaptured only
// when the launch can shrink by half.
#include <string.h>

#include <new>
#include <vector>

#include "context.h"
#include "step_launch.h"

using namespace lbm;
using namespace lbm::host;

struct lbm_batch {
  int n;
  std::vector<lbm_ctx*> ctx;
  int lattice, precision, linear_eq, K;
  bool off32, periodic, trt;
  hipStream_t stream;
  size_t arg_size;
  // device tables
  uint8_t* args;
  int2* owner;
  int owner_cap;
  BatchReduce fused, pass;
  int fused_chunks, pass_chunks;   // blocks of the chunk launch of each reduction
  double* q;
  // host mirror of the sample layout
  std::vector<int> grid;           // blocks of each sample's own launch
  std::vector<int2> owner_h;
  // host staging of the uploads (kept until the stream has been synchronised)
  std::vector<uint8_t> h_args;
  std::vector<int> h_pass;
  std::vector<int2> h_owner;
  // graphs of one check window, by the parity flip of its first step
  int use_graph;
  hipStream_t capture;
  hipGraphExec_t exec[2];
  int exec_grid[2];
};

namespace {

struct BatchLayout {
  size_t arg_size, off_args, off_owner, off_ptr, off_int, off_q, bytes;
  int owner_cap, chunk_cap_fused, chunk_cap_pass;
};

size_t arg_bytes(int precision) {
  return precision == LBM_FP64 ? sizeof(StepArgs<double>) : sizeof(StepArgs<float>);
}

template <class T>
int sample_grid(const lbm_ctx* c) {
  const StepArgs<T> a = step_args<T>(c);
  return step_grid(c, a);
}

int sample_grid_any(const lbm_ctx* c) {
  return c->g.precision == LBM_FP64 ? sample_grid<double>(c) : sample_grid<float>(c);
}

int fused_parts(const lbm_ctx* c) { return (int)(c->L.rows * c->L.nw); }

lbm_status validate_ctxs(int32_t n, lbm_ctx* const* ctxs) {
  if (n < 1) return fail(LBM_EINVAL, "a batch needs n >= 1 samples, got %d", n);
  if (!ctxs) return fail(LBM_EINVAL, "ctxs is NULL");
  for (int d = 0; d < n; ++d) {
    const lbm_ctx* c = ctxs[d];
    if (!c) return fail(LBM_EINVAL, "ctxs[%d] is NULL", d);
    for (int e = 0; e < d; ++e)
      if (ctxs[e] == c) return fail(LBM_EINVAL, "ctxs[%d] and ctxs[%d] are the same context", e, d);
    const lbm_ctx* c0 = ctxs[0];
    if (c->g.lattice != c0->g.lattice || c->g.precision != c0->g.precision)
      return fail(LBM_EINVAL, "sample %d: lattice and precision must match sample 0", d);
    if (c->g.check_every != c0->g.check_every)
      return fail(LBM_EINVAL, "sample %d: check_every must match sample 0", d);
    if (c->linear_eq != c0->linear_eq)
      return fail(LBM_EINVAL, "sample %d: the linear-equilibrium option must match sample 0", d);
    if (c->g.boundary != c0->g.boundary)
      return fail(LBM_EINVAL, "sample %d: boundary case must match sample 0", d);
    if ((c->trt_magic > 0.0) != (c0->trt_magic > 0.0))
      return fail(LBM_EINVAL, "sample %d: collision model (BGK / TRT) must match sample 0", d);
    if (off32_ok(c) != off32_ok(c0))
      return fail(LBM_EINVAL, "sample %d: sizes too different to share one step kernel", d);
  }
  return LBM_OK;
}

lbm_status batch_layout(int32_t n, lbm_ctx* const* ctxs, BatchLayout* B) {
  lbm_status s = validate_ctxs(n, ctxs);
  if (s != LBM_OK) return s;
  // the kernel indexes the table as a StepArgs<T> array: the stride is sizeof
  B->arg_size = arg_bytes(ctxs[0]->g.precision);
  uint64_t cap = 0, cf = 0, cp = 0;
  for (int d = 0; d < n; ++d) {
    cap += align_up((size_t)sample_grid_any(ctxs[d]), 8);
    cf += (fused_parts(ctxs[d]) + kChunk - 1) / kChunk;
    cp += ctxs[d]->L.chunks;
  }
  if (cap >= (1ull << 31) || cf >= (1ull << 31) || cp >= (1ull << 31))
    return fail(LBM_EINVAL, "batch too large for one launch");
  B->owner_cap = (int)cap;
  B->chunk_cap_fused = (int)cf;
  B->chunk_cap_pass = (int)cp;
  size_t off = 0;
  B->off_args = off;
  off = align_up(off + 2 * (size_t)n * B->arg_size, 256);
  B->off_owner = off;
  off = align_up(off + cap * sizeof(int2), 256);
  B->off_ptr = off;   // part[n], chunk[n] (shared by both reductions)
  off = align_up(off + 2 * (size_t)n * sizeof(void*), 256);
  B->off_int = off;   // per reduction: nparts[n], chunk_start[n + 1], chunk_owner[cap]
  off = align_up(off + ((4 * (size_t)n + 2) + cf + cp) * sizeof(int), 256);
  B->off_q = off;     // scale[n], q[n]
  off = align_up(off + 2 * (size_t)n * sizeof(double), 256);
  B->bytes = off;
  return LBM_OK;
}

// Copies host memory to the device and waits, so the host copy may change.
lbm_status h2d(hipStream_t st, void* dst, const void* src, size_t bytes) {
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return LBM_OK;
}

// Host image of one reduction's integer tables: nparts, chunk_start, owner.
void reduce_tables(const std::vector<int>& nparts, std::vector<int>* out, int* nchunks) {
  const int n = (int)nparts.size();
  out->assign(2 * (size_t)n + 1, 0);
  std::vector<int> owners;
  int c = 0;
  for (int d = 0; d < n; ++d) {
    (*out)[d] = nparts[d];
    (*out)[n + d] = c;
    const int k = (nparts[d] + kChunk - 1) / kChunk;
    for (int i = 0; i < k; ++i) owners.push_back(d);
    c += k;
  }
  (*out)[2 * n] = c;
  out->insert(out->end(), owners.begin(), owners.end());
  *nchunks = c;
}

// Uploads one reduction's tables to dst (ints) and points r at them.
lbm_status upload_reduce(lbm_batch* b, const std::vector<int>& nparts, int* dst, BatchReduce* r,
                         int* nchunks) {
  std::vector<int> t;
  reduce_tables(nparts, &t, nchunks);
  lbm_status s = h2d(b->stream, dst, t.data(), t.size() * sizeof(int));
  if (s != LBM_OK) return s;
  r->nparts = dst;
  r->chunk_start = dst + b->n;
  r->chunk_owner = dst + 2 * b->n + 1;
  return LBM_OK;
}

// Owner table of the samples flagged in run[]; the stretch of sample d lists
// blocks 0 .. grid[d] - 1 and is padded to a multiple of 8.
void build_owner(lbm_batch* b, const std::vector<char>& run) {
  b->owner_h.clear();
  for (int d = 0; d < b->n; ++d) {
    if (!run[d]) continue;
    for (int i = 0; i < b->grid[d]; ++i) b->owner_h.push_back(make_int2(d, i));
    while (b->owner_h.size() % 8) b->owner_h.push_back(make_int2(-1, 0));
  }
}

// Writes the owner table, padded with (-1, 0) to `size` entries.
lbm_status upload_owner(lbm_batch* b, int size) {
  b->h_owner = b->owner_h;
  b->h_owner.resize(size, make_int2(-1, 0));
  if (size == 0) return LBM_OK;
  return h2d(b->stream, b->owner, b->h_owner.data(), (size_t)size * sizeof(int2));
}

// Step arguments of every sample at its current parity and the other one,
// and the launch grid of each (the contexts' options may have changed).
template <class T>
lbm_status upload_args(lbm_batch* b) {
  if (b->arg_size != sizeof(StepArgs<T>)) return fail(LBM_ESTATE, "internal: argument stride");
  std::vector<uint8_t>& h = b->h_args;
  h.assign(2 * (size_t)b->n * b->arg_size, 0);
  for (int d = 0; d < b->n; ++d) {
    lbm_ctx* c = b->ctx[d];
    if (c->linear_eq != b->linear_eq)
      return fail(LBM_ESTATE, "sample %d: the linear-equilibrium option changed", d);
    if ((c->trt_magic > 0.0) != b->trt)
      return fail(LBM_ESTATE, "sample %d: the collision model changed", d);
    if (off32_ok(c) != b->off32)
      return fail(LBM_ESTATE, "sample %d: the offset width changed", d);
    const int p = c->parity;
    for (int j = 0; j < 2; ++j) {
      c->parity = p ^ j;
      const StepArgs<T> a = step_args<T>(c);
      memcpy(h.data() + (2 * (size_t)d + j) * b->arg_size, &a, sizeof a);
      if (j == 0) b->grid[d] = step_grid(c, a);
    }
    c->parity = p;
  }
  size_t need = 0;
  for (int d = 0; d < b->n; ++d) need += align_up((size_t)b->grid[d], 8);
  if (need > (size_t)b->owner_cap)
    return fail(LBM_ESTATE, "the samples' tile-order options changed since the batch was created");
  return h2d(b->stream, b->args, h.data(), h.size());
}

lbm_status refresh_args(lbm_batch* b) {
  return b->precision == LBM_FP64 ? upload_args<double>(b) : upload_args<float>(b);
}

void launch_step(const lbm_batch* b, int grid, int flip, bool flux, hipStream_t st) {
  if (grid <= 0) return;
  const StepVariant v{flux, b->linear_eq != 0, b->off32, b->periodic, b->trt};
  if (b->lattice == LBM_D2Q9) {
    if (b->precision == LBM_FP64)
      launch_batch_step_kernel<D2Q9, double>((const StepArgs<double>*)b->args, b->owner, flip,
                                             grid, st, v);
    else
      launch_batch_step_kernel<D2Q9, float>((const StepArgs<float>*)b->args, b->owner, flip,
                                            grid, st, v);
  } else {
    if (b->precision == LBM_FP64)
      launch_batch_step_kernel<D3Q19, double>((const StepArgs<double>*)b->args, b->owner, flip,
                                              grid, st, v);
    else
      launch_batch_step_kernel<D3Q19, float>((const StepArgs<float>*)b->args, b->owner, flip,
                                             grid, st, v);
  }
}

void launch_reduce(const lbm_batch* b, const BatchReduce& r, int nchunks, hipStream_t st) {
  k_reduce_chunks_batch<<<nchunks, 1024, 0, st>>>(r);
  k_reduce_final_batch<<<b->n, 1024, 0, st>>>(r);
}

// One check window: K steps from parity flip `flip0`, the flux fused into the
// last, and the batched reduction into q.
void launch_window(const lbm_batch* b, int grid, int flip0, hipStream_t st) {
  for (int s = 0; s < b->K; ++s) launch_step(b, grid, (flip0 + s) & 1, s == b->K - 1, st);
  launch_reduce(b, b->fused, b->fused_chunks, st);
}

void drop_graphs(lbm_batch* b) {
  for (int i = 0; i < 2; ++i) {
    if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
    b->exec[i] = nullptr;
    b->exec_grid[i] = 0;
  }
}

// Window graph for a launch of `grid` blocks starting at parity flip `flip0`.
// Captured on the batch's private stream (capture records, it does not run).
lbm_status window_graph(lbm_batch* b, int grid, int flip0, hipGraphExec_t* out) {
  if (b->exec[flip0] && b->exec_grid[flip0] == grid) {
    *out = b->exec[flip0];
    return LBM_OK;
  }
  if (b->exec[flip0]) {
    HIP_TRY(hipGraphExecDestroy(b->exec[flip0]));
    b->exec[flip0] = nullptr;
  }
  if (!b->capture) HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
  launch_window(b, grid, flip0, b->capture);
  hipGraph_t g = nullptr;
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipStreamEndCapture(b->capture, &g);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(LBM_EHIP, "window capture: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  hipGraphExec_t x = nullptr;
  const hipError_t e3 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) return fail(LBM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e3));
  b->exec[flip0] = x;
  b->exec_grid[flip0] = grid;
  *out = x;
  return LBM_OK;
}

// Flux pass of every sample and the batched reduction into q (no sync).
lbm_status pass_flux(lbm_batch* b) {
  std::vector<int> np(b->n);
  for (int d = 0; d < b->n; ++d) {
    lbm_status s = flux_pass(b->ctx[d], &np[d]);
    if (s != LBM_OK) return s;
  }
  if (np != b->h_pass) {   // the tables change only with the slot counts
    lbm_status s = upload_reduce(b, np, (int*)b->pass.nparts, &b->pass, &b->pass_chunks);
    if (s != LBM_OK) return s;
    b->h_pass = np;
  }
  launch_reduce(b, b->pass, b->pass_chunks, b->stream);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

// Pass-flux results of every sample, lowered by its force offset (see
// flux_pass_offset): the same arithmetic as the single-domain flux.
lbm_status read_pass_q(lbm_batch* b, double* h);

lbm_status read_q(lbm_batch* b, double* h) {
  HIP_TRY(hipMemcpyAsync(h, b->q, (size_t)b->n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

lbm_status read_pass_q(lbm_batch* b, double* h) {
  lbm_status s = read_q(b, h);
  if (s != LBM_OK) return s;
  for (int d = 0; d < b->n; ++d) h[d] -= flux_pass_offset(b->ctx[d]);
  return LBM_OK;
}

// Advances the host state of sample d by k steps.
void advance(lbm_ctx* c, int64_t k) {
  c->parity ^= (int)(k & 1);
  c->steps += k;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_query_sizes(int32_t n, lbm_ctx* const* ctxs, size_t* work_bytes) {
  BatchLayout B;
  lbm_status s = batch_layout(n, ctxs, &B);
  if (s != LBM_OK) return s;
  if (work_bytes) *work_bytes = B.bytes;
  return ok();
}

lbm_status lbm_batch_create(lbm_batch** out, int32_t n, lbm_ctx* const* ctxs, void* work,
                            void* stream) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  BatchLayout B;
  lbm_status s = batch_layout(n, ctxs, &B);
  if (s != LBM_OK) return s;
  if (!work) return fail(LBM_EINVAL, "work is NULL");
  if ((uintptr_t)work & 255) return fail(LBM_EINVAL, "work must be 256-byte aligned");
  for (int d = 0; d < n; ++d)
    if (ctxs[d]->stream != (hipStream_t)stream)
      return fail(LBM_EINVAL, "sample %d enqueues on another stream than the batch", d);
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return fail(LBM_ENOMEM, "out of host memory");
  b->n = n;
  b->ctx.assign(ctxs, ctxs + n);
  b->lattice = ctxs[0]->g.lattice;
  b->precision = ctxs[0]->g.precision;
  b->linear_eq = ctxs[0]->linear_eq;
  b->K = ctxs[0]->g.check_every;
  b->off32 = off32_ok(ctxs[0]);
  b->periodic = ctxs[0]->g.boundary == LBM_BC_PERIODIC;
  b->trt = ctxs[0]->trt_magic > 0.0;
  b->stream = (hipStream_t)stream;
  b->arg_size = B.arg_size;
  uint8_t* w = (uint8_t*)work;
  b->args = w + B.off_args;
  b->owner = (int2*)(w + B.off_owner);
  b->owner_cap = B.owner_cap;
  b->grid.assign(n, 0);
  b->use_graph = 1;
  b->capture = nullptr;
  b->exec[0] = b->exec[1] = nullptr;
  b->exec_grid[0] = b->exec_grid[1] = 0;
  double** ptr = (double**)(w + B.off_ptr);
  int* ints = (int*)(w + B.off_int);
  double* dbl = (double*)(w + B.off_q);
  b->q = dbl + n;
  // pointer and scale tables (fixed for the batch's life)
  std::vector<double*> hp(2 * (size_t)n);
  std::vector<double> hs(n);
  std::vector<int> fp(n);
  for (int d = 0; d < n; ++d) {
    hp[d] = ctxs[d]->partial();
    hp[n + d] = ctxs[d]->partial() + ctxs[d]->L.partials;
    hs[d] = 1.0 / ctxs[d]->g.nx;
    fp[d] = fused_parts(ctxs[d]);
  }
  auto fail_free = [&](lbm_status st) { delete b; return st; };
  s = h2d(b->stream, ptr, hp.data(), hp.size() * sizeof(double*));
  if (s == LBM_OK) s = h2d(b->stream, dbl, hs.data(), hs.size() * sizeof(double));
  if (s != LBM_OK) return fail_free(s);
  for (BatchReduce* r : {&b->fused, &b->pass}) {
    r->part = ptr;
    r->chunk = ptr + n;
    r->scale = dbl;
    r->out = b->q;
  }
  s = upload_reduce(b, fp, ints, &b->fused, &b->fused_chunks);
  if (s != LBM_OK) return fail_free(s);
  // the pass tables follow the fused ones; their contents come with each pass
  int* pass_ints = ints + 2 * n + 1 + B.chunk_cap_fused;
  b->pass.nparts = pass_ints;
  b->pass.chunk_start = pass_ints + n;
  b->pass.chunk_owner = pass_ints + 2 * n + 1;
  b->pass_chunks = 0;
  s = refresh_args(b);
  if (s != LBM_OK) return fail_free(s);
  *out = b;
  return ok();
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return ok();
  lbm_status s = refresh_args(b);
  if (s != LBM_OK) return s;
  build_owner(b, std::vector<char>(b->n, 1));
  const int grid = (int)b->owner_h.size();
  s = upload_owner(b, grid);
  if (s != LBM_OK) return s;
  for (int64_t i = 0; i < nsteps; ++i) launch_step(b, grid, (int)(i & 1), false, b->stream);
  HIP_TRY(hipGetLastError());
  for (lbm_ctx* c : b->ctx) advance(c, nsteps);
  // the args table now holds the arguments of the starting parities
  return ok();
}

lbm_status lbm_batch_run_to_steady(lbm_batch* b, double tol, int64_t max_steps,
                                   int64_t* steps_out, double* resid_out, int32_t* status_out,
                                   double* q_log, int64_t log_windows) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (!(tol >= 0.0) || max_steps < 0) return fail(LBM_EINVAL, "need tol >= 0 and max_steps >= 0");
  if (log_windows < 0 || (log_windows > 0 && !q_log))
    return fail(LBM_EINVAL, "q_log must hold log_windows >= 0 rows");
  for (int64_t i = 0; i < log_windows * b->n; ++i) q_log[i] = NAN;
  const int n = b->n, K = b->K;
  lbm_status s = refresh_args(b);
  if (s != LBM_OK) return s;
  // flux of the starting states
  s = pass_flux(b);
  if (s != LBM_OK) return s;
  std::vector<double> prev(n), q(n), resid(n, INFINITY);
  s = read_pass_q(b, prev.data());
  if (s != LBM_OK) return s;
  std::vector<char> run(n);
  std::vector<int64_t> done(n, 0);   // steps taken in this call
  std::vector<lbm_status> st(n, LBM_ENOTCONV);
  int running = 0;
  for (int d = 0; d < n; ++d) {
    run[d] = b->ctx[d]->steps + K <= max_steps;
    running += run[d];
  }
  bool changed = true;
  int launch = 0;   // blocks of the current launch (table size)
  int64_t t = 0;    // steps taken by the running samples in this call
  lbm_status err = LBM_OK;
  while (running > 0) {
    if (changed) {
      build_owner(b, run);
      const int live = (int)b->owner_h.size();
      // keep the launch size of the captured graph unless it can halve
      if (!b->use_graph || launch == 0 || 2 * live < launch) launch = live;
      err = upload_owner(b, launch);
      if (err != LBM_OK) break;
      changed = false;
    }
    const int flip0 = (int)(t & 1);
    if (b->use_graph) {
      hipGraphExec_t x = nullptr;
      err = window_graph(b, launch, flip0, &x);
      if (err != LBM_OK) break;
      const hipError_t e = hipGraphLaunch(x, b->stream);
      if (e != hipSuccess) {
        err = fail(LBM_EHIP, "hipGraphLaunch: %s", hipGetErrorString(e));
        break;
      }
    } else {
      launch_window(b, launch, flip0, b->stream);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) {
        err = fail(LBM_EHIP, "window launch: %s", hipGetErrorString(e));
        break;
      }
    }
    const int64_t window = t / K;   // index of this window in the call
    t += K;
    err = read_q(b, q.data());
    if (err != LBM_OK) break;
    for (int d = 0; d < n; ++d) {
      if (!run[d]) continue;
      done[d] += K;
      if (window < log_windows) q_log[window * n + d] = q[d];
      if (!isfinite(q[d])) {
        st[d] = LBM_ENONFINITE;
        resid[d] = NAN;
        run[d] = 0;
      } else {
        resid[d] = fabs(q[d] - prev[d]) / fabs(q[d]);
        prev[d] = q[d];
        if (resid[d] < tol) {
          st[d] = LBM_OK;
          run[d] = 0;
        } else if (b->ctx[d]->steps + done[d] + K > max_steps) {
          run[d] = 0;
        }
      }
      if (!run[d]) {
        --running;
        changed = true;
      }
    }
  }
  for (int d = 0; d < n; ++d) advance(b->ctx[d], done[d]);
  if (err != LBM_OK) return err;
  lbm_status first = LBM_OK;
  int first_d = -1;
  for (int d = 0; d < n; ++d) {
    if (steps_out) steps_out[d] = b->ctx[d]->steps;
    if (resid_out) resid_out[d] = resid[d];
    if (status_out) status_out[d] = st[d];
    if (st[d] != LBM_OK && first == LBM_OK) {
      first = st[d];
      first_d = d;
    }
  }
  if (first != LBM_OK)
    return fail(first, "sample %d %s", first_d,
                first == LBM_ENONFINITE ? "has a non-finite flux" : "did not converge");
  return ok();
}

lbm_status lbm_batch_flux(lbm_batch* b, double* q_out) {
  if (!b || !q_out) return fail(LBM_EINVAL, "NULL argument");
  lbm_status s = pass_flux(b);
  if (s != LBM_OK) return s;
  s = read_pass_q(b, q_out);
  if (s != LBM_OK) return s;
  for (int d = 0; d < b->n; ++d)
    if (!isfinite(q_out[d])) return fail(LBM_ENONFINITE, "sample %d: flux is not finite", d);
  return ok();
}

lbm_status lbm_batch_permeability(lbm_batch* b, double* k_out, int32_t* status_out) {
  if (!b || !k_out) return fail(LBM_EINVAL, "NULL argument");
  for (int d = 0; d < b->n; ++d) {
    const lbm_ctx* c = b->ctx[d];
    if (c->g.boundary == LBM_BC_PRESSURE && c->rho_in == c->rho_out)
      return fail(LBM_ESTATE, "sample %d: rho_in == rho_out: no pressure drop", d);
    if (c->g.boundary == LBM_BC_PERIODIC && c->g.body_force == 0.0)
      return fail(LBM_ESTATE, "sample %d: periodic case without a body force", d);
  }
  lbm_status s = pass_flux(b);
  if (s != LBM_OK) return s;
  std::vector<double> q(b->n);
  s = read_pass_q(b, q.data());
  if (s != LBM_OK) return s;
  lbm_status first = LBM_OK;
  int first_d = -1;
  for (int d = 0; d < b->n; ++d) {
    lbm_status sd = LBM_OK;
    if (!isfinite(q[d])) {
      k_out[d] = q[d];
      sd = LBM_ENONFINITE;
    } else if (q[d] == 0.0) {
      k_out[d] = 0.0;
      sd = LBM_ENOFLOW;
    } else {
      k_out[d] = perm_from_flux(b->ctx[d], q[d]);
    }
    if (status_out) status_out[d] = sd;
    if (sd != LBM_OK && first == LBM_OK) {
      first = sd;
      first_d = d;
    }
  }
  if (first != LBM_OK)
    return fail(first, "sample %d: %s", first_d,
                first == LBM_ENOFLOW ? "zero mass flow rate" : "flux is not finite");
  return ok();
}

lbm_status lbm_batch_set_option(lbm_batch* b, int32_t option, int64_t value) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  switch (option) {
    case LBM_BATCH_OPT_GRAPH:
      if (value != 0 && value != 1) return fail(LBM_EINVAL, "graph option is 0 or 1");
      b->use_graph = (int)value;
      return ok();
    default:
      return fail(LBM_EINVAL, "unknown batch option %d", option);
  }
}

lbm_status lbm_batch_destroy(lbm_batch* b) {
  if (!b) return ok();
  drop_graphs(b);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
  return ok();
}

}  // extern "C"
