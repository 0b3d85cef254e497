// Host side of the C ABI declared in include/lbm.h.
//
// A context holds host metadata only: the geometry, the physical parameters,
// the caller's buffers and stream, the ping-pong parity and the step count.
// Device memory is the caller's; the work buffer is carved here into
//   bits     uint64 [nz][ny][nw + 2]     fluid bitmap with guard words
//   pfx      uint32 [nz][ny][nw]         compact index of each word's first fluid node
//   desc     WordDesc [nz][ny][nw]       per-word records read by the D2Q9 step kernels
//   count    uint32 [nz][ny][nw]         fluid nodes per word (set-up only)
//   scan     uint32 [scan blocks]        block totals of the prefix scan (set-up only)
//   bplane   T [2 parities][2 sides][D+1][nz][ny]   edge-node moments
//   partial  double [...]                flux partials
//   scalars  double [8]                  reduced flux, fluid count
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

#include "context.h"
#include "step_launch.h"

using namespace lbm;

namespace lbm {
namespace host {

namespace {
thread_local char g_err[512] = "";
}  // namespace

lbm_status fail(lbm_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

lbm_status ok() {
  g_err[0] = 0;
  return LBM_OK;
}

}  // namespace host
}  // namespace lbm

namespace {

using namespace lbm::host;

lbm_status validate_geom(const lbm_geom* g) {
  if (!g) return fail(LBM_EINVAL, "geom is NULL");
  if (g->lattice != LBM_D2Q9 && g->lattice != LBM_D3Q19)
    return fail(LBM_EINVAL, "lattice must be 9 (D2Q9) or 19 (D3Q19), got %d", g->lattice);
  if (g->precision != LBM_FP64 && g->precision != LBM_FP32)
    return fail(LBM_EINVAL, "precision must be LBM_FP64 or LBM_FP32, got %d", g->precision);
  if (g->nx < 2 || g->ny < 1 || g->nz < 1)
    return fail(LBM_EINVAL, "need nx >= 2, ny >= 1, nz >= 1 (got %d x %d x %d)", g->nx, g->ny, g->nz);
  if (g->lattice == LBM_D2Q9 && g->nz != 1) return fail(LBM_EINVAL, "D2Q9 needs nz == 1");
  if (g->check_every < 1) return fail(LBM_EINVAL, "check_every must be >= 1");
  if (!(g->rho0 > 0.0) || !isfinite(g->rho0)) return fail(LBM_EINVAL, "rho0 must be > 0");
  if (g->boundary != LBM_BC_PRESSURE && g->boundary != LBM_BC_PERIODIC)
    return fail(LBM_EINVAL, "boundary must be LBM_BC_PRESSURE or LBM_BC_PERIODIC");
  if (!isfinite(g->body_force)) return fail(LBM_EINVAL, "body_force must be finite");
  if (g->boundary == LBM_BC_PRESSURE && g->body_force != 0.0)
    return fail(LBM_EINVAL, "a body force needs LBM_BC_PERIODIC");
  const uint64_t N = (uint64_t)g->nx * g->ny * g->nz;
  if (g->n_fluid < 0 || (uint64_t)g->n_fluid > N)
    return fail(LBM_EINVAL, "n_fluid must be in [0, nx*ny*nz], got %lld", (long long)g->n_fluid);
  return LBM_OK;
}

lbm_status make_layout(const lbm_geom* g, Layout* L) {
  lbm_status s = validate_geom(g);
  if (s != LBM_OK) return s;
  L->Q = g->lattice;
  L->D = g->lattice == LBM_D2Q9 ? 2 : 3;
  L->esize = g->precision == LBM_FP64 ? 8 : 4;
  L->nw = (g->nx + kWave - 1) / kWave;
  L->S = L->nw >= 4 ? 4 : (L->nw >= 2 ? 2 : 1);
  L->segs_per_row = (L->nw + L->S - 1) / L->S;
  L->align = (uint32_t)(128 / L->esize);
  L->rows = (uint64_t)g->ny * g->nz;
  L->nsegs = L->rows * L->segs_per_row;
  L->n_fluid = (uint64_t)g->n_fluid;
  // every segment may need up to align - 1 padding slots
  L->ps = align_up(L->n_fluid + (uint64_t)(L->align - 1) * L->nsegs, 64);
  if (L->ps == 0) L->ps = 64;
  if (L->ps >= (1ull << 32) || (uint64_t)g->nx * g->ny * g->nz >= (1ull << 40))
    return fail(LBM_EINVAL, "domain too large: more than 2^32 population slots");
  L->f_bytes = (size_t)L->Q * L->ps * L->esize;
  {
    const int rows_per_tile = kRows / L->S;
    const uint64_t b = (uint64_t)L->segs_per_row * ((g->ny + rows_per_tile - 1) / rows_per_tile) * g->nz;
    if (b * 8 >= (1ull << 31)) return fail(LBM_EINVAL, "too many blocks");
  }
  const uint64_t nwords = L->rows * L->nw;
  if (L->rows * (uint64_t)(L->nw + 2) >= (1ull << 31))
    return fail(LBM_EINVAL, "too many bitmap words");
  L->scan_blocks = (int)((nwords + kScanBlock - 1) / kScanBlock);
  L->seg_scan_blocks = (int)((L->nsegs + kScanBlock - 1) / kScanBlock);
  // one flux partial per bitmap word (step) or per 256 slots (flux pass)
  const uint64_t flux_blocks = (L->ps + 255) / 256;
  const uint64_t parts = nwords > flux_blocks ? nwords : flux_blocks;
  L->partials = (int)(parts < 1 ? 1 : parts);
  L->chunks = (L->partials + kChunk - 1) / kChunk;
  L->bplane_one = (size_t)2 * (L->D + 1) * g->nz * g->ny;
  size_t off = 0;
  L->off_bits = off;
  off = align_up(off + L->rows * (L->nw + 2) * 8, 256);
  L->off_pfx = off;
  off = align_up(off + nwords * 4, 256);
  L->off_desc = off;
  if (g->lattice == LBM_D2Q9) off = align_up(off + nwords * sizeof(WordDesc), 256);
  L->off_count = off;
  off = align_up(off + nwords * 4, 256);
  L->off_scan = off;
  off = align_up(off + (size_t)L->scan_blocks * 4, 256);
  L->off_seg = off;
  off = align_up(off + (size_t)L->nsegs * 4, 256);
  L->off_seg_scan = off;
  off = align_up(off + (size_t)L->seg_scan_blocks * 4, 256);
  L->off_bplane = off;
  off = align_up(off + 2 * L->bplane_one * L->esize, 256);
  L->off_partial = off;
  off = align_up(off + (size_t)(L->partials + L->chunks) * 8, 256);
  L->off_scalar = off;
  off = align_up(off + 64, 256);
  L->work_bytes = off;
  return LBM_OK;
}

template <class Lat, class T>
lbm_status launch_steps(lbm_ctx* c, int64_t n, bool flux_last) {
  StepVariant v{false, c->linear_eq != 0, off32_ok(c), c->g.boundary == LBM_BC_PERIODIC,
                c->trt_magic > 0.0};
  for (int64_t s = 0; s < n; ++s) {
    StepArgs<T> a = step_args<T>(c);
    v.flux = flux_last && s == n - 1;
    launch_step_kernel<Lat, T>(a, step_grid(c, a), c->stream, v);
    c->parity ^= 1;
    c->steps += 1;
  }
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

template <class Lat, class T>
lbm_status launch_bplane(lbm_ctx* c) {
  const uint64_t n = 2ull * c->g.nz * c->g.ny;
  k_bplane<Lat, T><<<grid_1d(n), 256, 0, c->stream>>>(
      (const T*)c->f[c->parity], c->fmap(), (T*)c->bplane(c->parity), c->L.ps, (T)c->g.rho0);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

template <class Lat, class T>
lbm_status launch_reset(lbm_ctx* c, int mode) {
  k_init_rest<Lat, T><<<grid_1d(n_nodes(c)), 256, 0, c->stream>>>(
      (T*)c->f[c->parity], (T*)c->f[c->parity ^ 1], c->fmap(), c->L.ps, mode, c->rho_in,
      c->rho_out, c->g.rho0);
  HIP_TRY(hipGetLastError());
  return launch_bplane<Lat, T>(c);
}

template <class Lat, class T>
lbm_status launch_fields(lbm_ctx* c, const float* rho, const float* u) {
  auto kern = c->linear_eq ? k_init_fields<Lat, T, true> : k_init_fields<Lat, T, false>;
  kern<<<grid_1d(n_nodes(c)), 256, 0, c->stream>>>((T*)c->f[c->parity], c->fmap(), rho, u, c->L.ps,
                                                   c->g.rho0, 0.5 * (double)force_density<T>(c));
  HIP_TRY(hipGetLastError());
  return launch_bplane<Lat, T>(c);
}

template <class Lat, class T>
lbm_status launch_flux(lbm_ctx* c, double* partial, int* nparts) {
  const unsigned nb = flux_partials(c);
  k_flux<Lat, T><<<nb, 256, 0, c->stream>>>((const T*)c->f[c->parity], c->n_slots, c->L.ps,
                                              partial);
  HIP_TRY(hipGetLastError());
  *nparts = (int)nb;
  return LBM_OK;
}

template <class Lat, class T>
lbm_status launch_macro(lbm_ctx* c, void* rho, void* u, int dtype) {
  const unsigned nb = grid_1d(n_nodes(c));
  const T fhalf = T(0.5) * force_density<T>(c);
  if (dtype == 0)
    k_macro<Lat, T, float><<<nb, 256, 0, c->stream>>>((const T*)c->f[c->parity], c->fmap(),
                                                       (float*)rho, (float*)u, c->L.ps,
                                                       (T)c->g.rho0, fhalf);
  else
    k_macro<Lat, T, double><<<nb, 256, 0, c->stream>>>((const T*)c->f[c->parity], c->fmap(),
                                                        (double*)rho, (double*)u, c->L.ps,
                                                        (T)c->g.rho0, fhalf);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

template <template <class, class> class F, class... A>
lbm_status dispatch(lbm_ctx* c, A... args) {
  if (c->g.lattice == LBM_D2Q9)
    return c->g.precision == LBM_FP64 ? F<D2Q9, double>::run(c, args...)
                                      : F<D2Q9, float>::run(c, args...);
  return c->g.precision == LBM_FP64 ? F<D3Q19, double>::run(c, args...)
                                    : F<D3Q19, float>::run(c, args...);
}

template <class Lat, class T> struct Steps {
  static lbm_status run(lbm_ctx* c, int64_t n, bool fl) { return launch_steps<Lat, T>(c, n, fl); }
};
template <class Lat, class T> struct Reset {
  static lbm_status run(lbm_ctx* c, int mode) { return launch_reset<Lat, T>(c, mode); }
};
template <class Lat, class T> struct Fields {
  static lbm_status run(lbm_ctx* c, const float* r, const float* u) {
    return launch_fields<Lat, T>(c, r, u);
  }
};
template <class Lat, class T> struct Flux {
  static lbm_status run(lbm_ctx* c, double* p, int* np) { return launch_flux<Lat, T>(c, p, np); }
};
template <class Lat, class T> struct Macro {
  static lbm_status run(lbm_ctx* c, void* r, void* u, int d) { return launch_macro<Lat, T>(c, r, u, d); }
};
template <class Lat, class T> struct Bplane {
  static lbm_status run(lbm_ctx* c) { return launch_bplane<Lat, T>(c); }
};
// n times: one step, then the current state becomes the mean of the states
// before and after that step (both ping-pong buffers), with fresh edge moments.
template <class Lat, class T> struct Smooth {
  static lbm_status run(lbm_ctx* c, int32_t n) {
    const uint64_t count = (uint64_t)c->L.Q * c->L.ps;
    for (int32_t i = 0; i < n; ++i) {
      lbm_status s = launch_steps<Lat, T>(c, 1, false);
      if (s != LBM_OK) return s;
      k_mean_states<T><<<grid_1d(count), 256, 0, c->stream>>>((T*)c->f[c->parity],
                                                               (const T*)c->f[c->parity ^ 1], count);
      HIP_TRY(hipGetLastError());
      s = launch_bplane<Lat, T>(c);
      if (s != LBM_OK) return s;
    }
    return LBM_OK;
  }
};

// Scans n counts in place (exclusive) with the three-pass scan; returns the
// total through *total (device) - block totals go to tmp.
lbm_status scan_in_place(lbm_ctx* c, uint32_t* data, uint64_t n, uint32_t* tmp, int nblocks,
                         uint64_t* total) {
  k_scan_local<<<nblocks, kScanBlock, 0, c->stream>>>(data, data, tmp, n);
  HIP_TRY(hipGetLastError());
  k_scan_totals<<<1, kScanBlock, 0, c->stream>>>(tmp, nblocks, total);
  HIP_TRY(hipGetLastError());
  k_scan_add<<<nblocks, kScanBlock, 0, c->stream>>>(data, tmp, n);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

// Bitmap, segment-aligned slots of every word, and the fluid count check.
lbm_status build_fluid_map(lbm_ctx* c) {
  const Layout& L = c->L;
  const uint64_t nwords = L.rows * L.nw;
  k_pack_bits<<<(unsigned)((nwords * 64 + 255) / 256), 256, 0, c->stream>>>(
      c->mask, c->bits(), c->count(), c->g.nx, c->g.ny, c->g.nz, L.nw);
  HIP_TRY(hipGetLastError());
  // fluid count: scan a copy of the per-word counts
  HIP_TRY(hipMemcpyAsync(c->pfx(), c->count(), nwords * 4, hipMemcpyDeviceToDevice, c->stream));
  uint64_t* totals = (uint64_t*)(c->scalar() + 1);   // [0] fluid nodes, [1] slots
  lbm_status s = scan_in_place(c, c->pfx(), nwords, c->scan(), L.scan_blocks, totals);
  if (s != LBM_OK) return s;
  // padded segment sizes -> first slot of every segment -> slot of every word
  k_seg_sizes<<<grid_1d(L.nsegs), 256, 0, c->stream>>>(c->count(), c->seg(), L.nsegs, L.nw, L.S,
                                                         L.segs_per_row, L.align);
  HIP_TRY(hipGetLastError());
  s = scan_in_place(c, c->seg(), L.nsegs, c->seg_scan(), L.seg_scan_blocks, totals + 1);
  if (s != LBM_OK) return s;
  k_word_pfx<<<grid_1d(nwords), 256, 0, c->stream>>>(c->count(), c->seg(), c->pfx(), nwords, L.nw,
                                                      L.S, L.segs_per_row);
  HIP_TRY(hipGetLastError());
  if (c->g.lattice == LBM_D2Q9) {
    k_word_desc<<<grid_1d(nwords), 256, 0, c->stream>>>(c->fmap(), c->desc(), nwords);
    HIP_TRY(hipGetLastError());
  }
  uint64_t h[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(h, totals, sizeof h, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (h[0] != L.n_fluid)
    return fail(LBM_EINVAL, "the mask has %llu fluid nodes but geom.n_fluid is %llu",
                (unsigned long long)h[0], (unsigned long long)L.n_fluid);
  if (h[1] > L.ps)
    return fail(LBM_EINVAL, "internal: %llu slots exceed the capacity %llu",
                (unsigned long long)h[1], (unsigned long long)L.ps);
  c->n_slots = h[1];
  return LBM_OK;
}

}  // namespace

namespace lbm {
namespace host {

lbm_status flux_pass(lbm_ctx* c, int* nparts) { return dispatch<Flux>(c, c->partial(), nparts); }

// Reduces n partials at `partial` (chunk sums to `chunk`, the result to *dev)
// and reads the result back.
lbm_status reduce_partials(lbm_ctx* c, const double* partial, double* chunk, double* dev, int n,
                           double* q) {
  const int nch = (n + kChunk - 1) / kChunk;
  k_reduce_chunks<<<nch, 1024, 0, c->stream>>>(partial, n, chunk);
  HIP_TRY(hipGetLastError());
  k_reduce_final<<<1, 1024, 0, c->stream>>>(chunk, nch, 1.0 / c->g.nx, dev);
  HIP_TRY(hipGetLastError());
  double h = 0.0;
  HIP_TRY(hipMemcpyAsync(&h, dev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *q = h;
  return LBM_OK;
}

// Reduces n partials of the last flux pass into scalar[0] and reads it back.
lbm_status reduce_flux(lbm_ctx* c, int n, double* q) {
  return reduce_partials(c, c->partial(), c->partial() + c->L.partials, c->scalar(), n, q);
}

lbm_status current_flux(lbm_ctx* c, double* q) {
  int n = 0;
  lbm_status s = flux_pass(c, &n);
  if (s != LBM_OK) return s;
  s = reduce_flux(c, n, q);
  if (s == LBM_OK) *q -= flux_pass_offset(c);
  return s;
}

double perm_from_flux(const lbm_ctx* c, double q) {
  const double nu = (c->tau - 0.5) / 3.0;
  if (c->g.boundary == LBM_BC_PERIODIC)   // Eq. 2: nu <u> / g, <u> = nx q / (rho0 N)
    return nu * q / (c->g.rho0 * c->g.body_force * (double)c->g.ny * c->g.nz);
  const double L = c->g.nx + 1.0, A = (double)c->g.ny * c->g.nz;
  return nu * q * L / (A * (1.0 / 3.0) * (c->rho_in - c->rho_out));
}

}  // namespace host
}  // namespace lbm

namespace {

using namespace lbm::host;

// Scratch of lbm_flux_noalloc: the flux pass's per-block partials, their chunk
// sums and the result, in a file-scope device array (one copy per GPU, held
// until the process ends) instead of the context's work buffer.
constexpr int kNoallocPartials = 1 << 18;                  // flux blocks: up to 2^26 slots
constexpr int kNoallocChunks = kNoallocPartials / kChunk;
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kNoallocPartials + kNoallocChunks + 32];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the device of the context's stream, looked
// up once per device with that device current.  In host code the array's name
// is only a stand-in: this address is what the kernels get.
lbm_status scratch_on(hipStream_t stream, double** out) {
  int dev = 0, cur = 0;
  HIP_TRY(hipStreamGetDevice(stream, &dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    HIP_TRY(hipGetDevice(&cur));
    if (cur != dev) HIP_TRY(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) HIP_TRY(hipSetDevice(cur));
    if (e != hipSuccess || !p)
      return fail(LBM_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_query_sizes(const lbm_geom* geom, size_t* f_bytes, size_t* work_bytes) {
  Layout L;
  lbm_status s = make_layout(geom, &L);
  if (s != LBM_OK) return s;
  if (f_bytes) *f_bytes = L.f_bytes;
  if (work_bytes) *work_bytes = L.work_bytes;
  return ok();
}

lbm_status lbm_init(lbm_ctx** out, const lbm_geom* geom, const lbm_buffers* bufs, double tau,
                    double rho_in, double rho_out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  Layout L;
  lbm_status s = make_layout(geom, &L);
  if (s != LBM_OK) return s;
  if (!bufs) return fail(LBM_EINVAL, "bufs is NULL");
  if (!bufs->f[0] || !bufs->f[1] || !bufs->mask || !bufs->work)
    return fail(LBM_EINVAL, "a device buffer is NULL");
  if (bufs->f[0] == bufs->f[1]) return fail(LBM_EINVAL, "f[0] and f[1] must differ");
  if (!(tau > 0.5) || !isfinite(tau))
    return fail(LBM_EINVAL, "tau must be > 1/2 (positive viscosity), got %g", tau);
  if (!(rho_in > 0.0) || !(rho_out > 0.0) || !isfinite(rho_in) || !isfinite(rho_out))
    return fail(LBM_EINVAL, "rho_in and rho_out must be positive and finite");
  if (geom->boundary == LBM_BC_PERIODIC && rho_in != rho_out)
    return fail(LBM_EINVAL, "periodic case: rho_in must equal rho_out (the starting density)");
  if (((uintptr_t)bufs->f[0] | (uintptr_t)bufs->f[1] | (uintptr_t)bufs->work) & 255)
    return fail(LBM_EINVAL, "f[0], f[1] and work must be 256-byte aligned");
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_ENOMEM, "out of host memory");
  c->g = *geom;
  c->L = L;
  c->f[0] = bufs->f[0];
  c->f[1] = bufs->f[1];
  c->mask = (const uint8_t*)bufs->mask;
  c->work = (uint8_t*)bufs->work;
  c->stream = (hipStream_t)bufs->stream;
  c->tau = tau;
  c->rho_in = rho_in;
  c->rho_out = rho_out;
  c->parity = 0;
  c->steps = 0;
  c->linear_eq = 0;
  c->xcd_remap = 1;
  c->n_slots = 0;
  c->band = 16;
  c->trt_magic = 0.0;
  c->wide_offsets = 0;

  auto fail_free = [&](lbm_status st) { delete c; return st; };
  s = build_fluid_map(c);
  if (s != LBM_OK) return fail_free(s);
  hipError_t e = hipMemsetAsync(c->f[0], 0, L.f_bytes, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->f[1], 0, L.f_bytes, c->stream);
  if (e != hipSuccess) return fail_free(fail(LBM_EHIP, "hipMemsetAsync: %s", hipGetErrorString(e)));
  s = dispatch<Reset>(c, (int)LBM_START_UNIFORM);
  if (s != LBM_OK) return fail_free(s);
  *out = c;
  return ok();
}

lbm_status lbm_reset(lbm_ctx* c, int32_t start) {
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  if (start != LBM_START_UNIFORM && start != LBM_START_LINEAR)
    return fail(LBM_EINVAL, "start must be LBM_START_UNIFORM or LBM_START_LINEAR");
  if (start == LBM_START_LINEAR && c->g.boundary == LBM_BC_PERIODIC)
    return fail(LBM_EINVAL, "the linear-density start needs the pressure case");
  c->parity = 0;
  c->steps = 0;
  lbm_status s = dispatch<Reset>(c, (int)start);
  return s == LBM_OK ? ok() : s;
}

lbm_status lbm_set_macro(lbm_ctx* c, const float* rho, const float* u) {
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  if (!rho || !u) return fail(LBM_EINVAL, "rho and u must be device pointers");
  c->parity = 0;
  c->steps = 0;
  lbm_status s = dispatch<Fields>(c, rho, u);
  return s == LBM_OK ? ok() : s;
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  lbm_status s = dispatch<Steps>(c, n, false);
  return s == LBM_OK ? ok() : s;
}

lbm_status lbm_flux(lbm_ctx* c, double* q_out) {
  if (!c || !q_out) return fail(LBM_EINVAL, "NULL argument");
  double q;
  lbm_status s = current_flux(c, &q);
  if (s != LBM_OK) return s;
  *q_out = q;
  if (!isfinite(q)) return fail(LBM_ENONFINITE, "flux is not finite");
  return ok();
}

lbm_status lbm_flux_noalloc(lbm_ctx* c, double* q_out) {
  if (!c || !q_out) return fail(LBM_EINVAL, "NULL argument");
  const unsigned np = flux_partials(c);
  if (np > (unsigned)kNoallocPartials)
    return fail(LBM_EINVAL, "lbm_flux_noalloc: %llu slots exceed its scratch (at most %llu)",
                (unsigned long long)c->n_slots, 256ull * kNoallocPartials);
  double* sp = nullptr;
  lbm_status s = scratch_on(c->stream, &sp);
  if (s != LBM_OK) return s;
  // every partial, chunk sum and the result are written before they are read:
  // nothing in the scratch needs clearing
  int n = 0;
  s = dispatch<Flux>(c, sp, &n);
  if (s != LBM_OK) return s;
  double q;
  s = reduce_partials(c, sp, sp + kNoallocPartials, sp + kNoallocPartials + kNoallocChunks, n, &q);
  if (s != LBM_OK) return s;
  q -= flux_pass_offset(c);
  *q_out = q;
  if (!isfinite(q)) return fail(LBM_ENONFINITE, "flux is not finite");
  return ok();
}

lbm_status lbm_permeability(lbm_ctx* c, double* k_out) {
  if (!c || !k_out) return fail(LBM_EINVAL, "NULL argument");
  if (c->g.boundary == LBM_BC_PRESSURE && c->rho_in == c->rho_out)
    return fail(LBM_ESTATE, "rho_in == rho_out: no pressure drop");
  if (c->g.boundary == LBM_BC_PERIODIC && c->g.body_force == 0.0)
    return fail(LBM_ESTATE, "periodic case without a body force: no driving");
  double q;
  lbm_status s = current_flux(c, &q);
  if (s != LBM_OK) return s;
  if (!isfinite(q)) {
    *k_out = q;
    return fail(LBM_ENONFINITE, "flux is not finite");
  }
  if (q == 0.0) {
    *k_out = 0.0;
    return fail(LBM_ENOFLOW, "zero mass flow rate");
  }
  *k_out = perm_from_flux(c, q);
  return ok();
}

lbm_status lbm_run_to_steady(lbm_ctx* c, double tol, int64_t max_steps, int64_t* steps_out,
                             double* resid_out) {
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  if (!(tol >= 0.0) || max_steps < 0) return fail(LBM_EINVAL, "need tol >= 0 and max_steps >= 0");
  const int K = c->g.check_every;
  double prev;
  lbm_status s = current_flux(c, &prev);
  if (s != LBM_OK) return s;
  double r = INFINITY;
  bool conv = false;
  while (c->steps + K <= max_steps) {
    s = dispatch<Steps>(c, (int64_t)K, true);
    if (s != LBM_OK) return s;
    double q;
    s = reduce_flux(c, (int)(c->L.rows * c->L.nw), &q);
    if (s != LBM_OK) return s;
    if (!isfinite(q)) {
      if (steps_out) *steps_out = c->steps;
      if (resid_out) *resid_out = NAN;
      return fail(LBM_ENONFINITE, "flux became non-finite after %lld steps", (long long)c->steps);
    }
    r = fabs(q - prev) / fabs(q);
    prev = q;
    if (r < tol) {
      conv = true;
      break;
    }
  }
  if (steps_out) *steps_out = c->steps;
  if (resid_out) *resid_out = r;
  if (!conv)
    return fail(LBM_ENOTCONV, "residual %g above %g after %lld steps", r, tol, (long long)c->steps);
  return ok();
}

lbm_status lbm_get_macro(lbm_ctx* c, void* rho, void* u, int32_t dtype) {
  if (!c || !rho || !u) return fail(LBM_EINVAL, "NULL argument");
  if (dtype != 0 && dtype != 1) return fail(LBM_EINVAL, "dtype must be 0 (float32) or 1 (float64)");
  lbm_status s = dispatch<Macro>(c, rho, u, (int)dtype);
  return s == LBM_OK ? ok() : s;
}

lbm_status lbm_get_populations(lbm_ctx* c, void* dst) {
  if (!c || !dst) return fail(LBM_EINVAL, "NULL argument");
  HIP_TRY(hipMemcpyAsync(dst, c->f[c->parity], c->L.f_bytes, hipMemcpyDeviceToDevice, c->stream));
  return ok();
}

lbm_status lbm_set_populations(lbm_ctx* c, const void* src) {
  if (!c || !src) return fail(LBM_EINVAL, "NULL argument");
  HIP_TRY(hipMemcpyAsync(c->f[c->parity], src, c->L.f_bytes, hipMemcpyDeviceToDevice, c->stream));
  lbm_status s = dispatch<Bplane>(c);
  return s == LBM_OK ? ok() : s;
}

lbm_status lbm_smooth(lbm_ctx* c, int32_t n) {
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  lbm_status s = dispatch<Smooth>(c, n);
  return s == LBM_OK ? ok() : s;
}

lbm_status lbm_set_option(lbm_ctx* c, int32_t option, int64_t value) {
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  switch (option) {
    case LBM_OPT_XCD_REMAP:
      if (value < 0 || value > 64) return fail(LBM_EINVAL, "tile order mode is 0..64");
      c->xcd_remap = (int)value;
      return ok();
    case LBM_OPT_BAND:
      if (value < 0 || value > 65536) return fail(LBM_EINVAL, "band is 0 (off) or 1..65536 tile rows");
      c->band = (int)value;
      return ok();
    case LBM_OPT_LINEAR_EQ:
      if (value != 0 && value != 1) return fail(LBM_EINVAL, "linear equilibrium is 0 or 1");
      c->linear_eq = (int)value;
      return ok();
    case LBM_OPT_WIDE_OFFSETS:
      if (value != 0 && value != 1) return fail(LBM_EINVAL, "wide offsets is 0 or 1");
      c->wide_offsets = (int)value;
      return ok();
    default:
      return fail(LBM_EINVAL, "unknown option %d", option);
  }
}

lbm_status lbm_set_trt(lbm_ctx* c, double magic) {
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  if (!(magic >= 0.0) || !isfinite(magic))
    return fail(LBM_EINVAL, "the TRT magic parameter must be >= 0 and finite, got %g", magic);
  c->trt_magic = magic;
  return ok();
}

lbm_status lbm_get_slot_map(lbm_ctx* c, int32_t* map) {
  if (!c || !map) return fail(LBM_EINVAL, "NULL argument");
  k_slot_map<<<grid_1d((uint64_t)c->g.nx * c->g.ny * c->g.nz), 256, 0, c->stream>>>(c->fmap(), map);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status lbm_lattice(int32_t lattice, int32_t* cv, double* w) {
  if (!cv || !w) return fail(LBM_EINVAL, "NULL argument");
  if (lattice == LBM_D2Q9) {
    for (int i = 0; i < D2Q9::Q; ++i) {
      cv[3 * i] = D2Q9::cx[i]; cv[3 * i + 1] = D2Q9::cy[i]; cv[3 * i + 2] = D2Q9::cz[i];
      w[i] = D2Q9::w[i];
    }
  } else if (lattice == LBM_D3Q19) {
    for (int i = 0; i < D3Q19::Q; ++i) {
      cv[3 * i] = D3Q19::cx[i]; cv[3 * i + 1] = D3Q19::cy[i]; cv[3 * i + 2] = D3Q19::cz[i];
      w[i] = D3Q19::w[i];
    }
  } else {
    return fail(LBM_EINVAL, "lattice must be 9 or 19");
  }
  return ok();
}

lbm_status lbm_steps(const lbm_ctx* c, int64_t* steps_out) {
  if (!c || !steps_out) return fail(LBM_EINVAL, "NULL argument");
  *steps_out = c->steps;
  return ok();
}

double lbm_knudsen(double tau, int32_t nx) { return sqrt(M_PI / 6.0) * (tau - 0.5) / (double)nx; }

lbm_status lbm_destroy(lbm_ctx* c) {
  delete c;
  return ok();
}

const char* lbm_last_error(void) { return lbm::host::g_err; }

const char* lbm_version(void) { return "1.0.0"; }

}  // extern "C"
