// Host side of the warm-start network ABI declared in include/wsn.h: layer
// launches with their argument checks, and the U-Net's forward and backward
// passes as sequences of those layers over caller-provided buffers.
#include <math.h>
#include <string.h>

#include <vector>

#include "context.h"
#include "wsn.h"
#include "wsn_kernels.h"

using lbm::host::fail;
using lbm::host::ok;
using namespace wsn;

namespace {

unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
size_t align256(size_t v) { return (v + 255) / 256 * 256; }

lbm_status check_image(int32_t batch, int32_t height, int32_t width, int32_t c, const char* what) {
  if (batch < 1 || height < 1 || width < 1 || c < 1)
    return fail(LBM_EINVAL, "%s: batch, height, width and channels must be >= 1", what);
  if ((int64_t)batch * height * width * c >= (1ll << 40))
    return fail(LBM_EINVAL, "%s: image too large", what);
  return LBM_OK;
}

lbm_status check_conv(int32_t batch, int32_t height, int32_t width, int32_t cin, int32_t cout,
                      int32_t ks, const char* what) {
  lbm_status s = check_image(batch, height, width, cin > cout ? cin : cout, what);
  if (s != LBM_OK) return s;
  if (ks != 1 && ks != 3) return fail(LBM_EINVAL, "%s: ks must be 1 or 3", what);
  if (width % 16) return fail(LBM_EINVAL, "%s: width must be a multiple of 16, got %d", what, width);
  if ((int64_t)batch * height * width >= (1ll << 31))
    return fail(LBM_EINVAL, "%s: more than 2^31 pixels", what);
  return LBM_OK;
}

// ----------------------------------------------------------------- conv launch

template <int KS, int NT>
void launch_fwd_t(const ConvArgs& a, int batch, hipStream_t st) {
  const dim3 grid((unsigned)(batch * a.tiles_h * a.tiles_w), (unsigned)((a.cout + NT - 1) / NT));
  const bool v4 = a.cin % 4 == 0 && a.cout % 4 == 0 && ((uintptr_t)a.x & 15u) == 0 &&
                  ((uintptr_t)a.w & 15u) == 0;
  if (v4) k_conv_fwd<KS, NT, true><<<grid, kBlock, 0, st>>>(a);
  else k_conv_fwd<KS, NT, false><<<grid, kBlock, 0, st>>>(a);
}

void conv_fwd(const float* x, const float* w, const float* bias, float* y, int batch, int H, int W,
              int cin, int cout, int ks, int relu, hipStream_t st) {
  ConvArgs a;
  a.x = x;
  a.w = w;
  a.bias = bias;
  a.y = y;
  a.H = H;
  a.W = W;
  a.cin = cin;
  a.cout = cout;
  const int tw = W % 64 == 0 ? 64 : (W % 32 == 0 ? 32 : 16);
  a.tw_log2 = tw == 64 ? 6 : (tw == 32 ? 5 : 4);
  a.th = kTile / tw;
  a.tiles_w = W / tw;
  a.tiles_h = (H + a.th - 1) / a.th;
  a.relu = relu;
  const int nt = cout > 32 ? 64 : (cout > 16 ? 32 : 16);
  if (ks == 3) {
    if (nt == 64) launch_fwd_t<3, 64>(a, batch, st);
    else if (nt == 32) launch_fwd_t<3, 32>(a, batch, st);
    else launch_fwd_t<3, 16>(a, batch, st);
  } else {
    if (nt == 64) launch_fwd_t<1, 64>(a, batch, st);
    else if (nt == 32) launch_fwd_t<1, 32>(a, batch, st);
    else launch_fwd_t<1, 16>(a, batch, st);
  }
}

// Split of a weight-gradient reduction: enough blocks to fill the GPU, pixel
// ranges of a multiple of 16.
struct WgradPlan {
  int tm, nt, mtiles, ntiles, nsplit, sp, colsplit, colsp;
  size_t part_floats, bias_floats;
};

WgradPlan wgrad_plan(int batch, int H, int W, int cin, int cout, int ks) {
  WgradPlan p;
  if (ks == 3) {
    // all nine taps per block (k_conv_wgrad3): 32 x 32 channel tiles, or 16
    // where the layer is that narrow
    p.tm = cin > 16 ? 32 : 16;
    p.nt = cout > 16 ? 32 : 16;
  } else {
    // input-channel tile: 64 unless a 32-wide tile divides cin and a 64-wide
    // one would leave a partly empty last tile (96 = 3 x 32, not 2 x 64)
    p.tm = cin > 32 ? (cin % 64 != 0 && cin % 32 == 0 ? 32 : 64) : (cin > 16 ? 32 : 16);
    p.nt = cout > 32 ? 64 : (cout > 16 ? 32 : 16);
  }
  p.mtiles = (cin + p.tm - 1) / p.tm;
  p.ntiles = (cout + p.nt - 1) / p.nt;
  const long npix = (long)batch * H * W;
  const long per_split = (long)p.mtiles * p.ntiles;   // blocks per pixel split (taps: one block for 3x3, ks = 1 has one tap)
  long want = ((ks == 3 ? 1024 : 2048) + per_split - 1) / per_split;   // blocks to fill the GPU
  const long chunks = (npix + 15) / 16;
  if (want > chunks) want = chunks;
  if (want < 1) want = 1;
  p.sp = (int)(((chunks + want - 1) / want) * 16);
  p.nsplit = (int)((npix + p.sp - 1) / p.sp);
  p.part_floats = (size_t)p.nsplit * ks * ks * cin * cout;
  // bias: 4096 pixels per partial sum
  p.colsp = 4096;
  p.colsplit = (int)((npix + p.colsp - 1) / p.colsp);
  p.bias_floats = (size_t)p.colsplit * cout;
  return p;
}

size_t wgrad_bytes(const WgradPlan& p) {
  return align256(p.part_floats * 4) + align256(p.bias_floats * 4);
}

template <int KS, int TM, int NT>
void launch_wgrad_t(const WgradArgs& a, const WgradPlan& p, hipStream_t st) {
  if constexpr (KS == 3) {
    if constexpr (TM <= 32 && NT <= 32) {
      const dim3 grid((unsigned)p.nsplit, (unsigned)(p.mtiles * p.ntiles));
      const bool v4 = a.cin % 4 == 0 && a.cout % 4 == 0 && ((uintptr_t)a.x & 15u) == 0 &&
                      ((uintptr_t)a.dy & 15u) == 0;
      if (v4) k_conv_wgrad3<TM, NT, true><<<grid, kBlock, 0, st>>>(a);
      else k_conv_wgrad3<TM, NT, false><<<grid, kBlock, 0, st>>>(a);
    }
  } else {
    const dim3 grid((unsigned)p.nsplit, (unsigned)(KS * KS * p.mtiles * p.ntiles));
    k_conv_wgrad<KS, TM, NT><<<grid, kBlock, 0, st>>>(a);
  }
}

template <int KS, int TM>
void launch_wgrad_m(const WgradArgs& a, const WgradPlan& p, hipStream_t st) {
  if (p.nt == 64) launch_wgrad_t<KS, TM, 64>(a, p, st);
  else if (p.nt == 32) launch_wgrad_t<KS, TM, 32>(a, p, st);
  else launch_wgrad_t<KS, TM, 16>(a, p, st);
}

template <int KS>
void launch_wgrad_k(const WgradArgs& a, const WgradPlan& p, hipStream_t st) {
  if (p.tm == 64) launch_wgrad_m<KS, 64>(a, p, st);
  else if (p.tm == 32) launch_wgrad_m<KS, 32>(a, p, st);
  else launch_wgrad_m<KS, 16>(a, p, st);
}

void conv_wgrad(const float* x, const float* dy, float* dw, float* db, int batch, int H, int W,
                int cin, int cout, int ks, void* work, hipStream_t st) {
  const WgradPlan p = wgrad_plan(batch, H, W, cin, cout, ks);
  float* part = (float*)work;
  float* bpart = (float*)((char*)work + align256(p.part_floats * 4));
  WgradArgs a;
  a.x = x;
  a.dy = dy;
  a.part = part;
  a.H = H;
  a.W = W;
  a.cin = cin;
  a.cout = cout;
  a.npix = batch * H * W;
  a.sp = p.sp;
  a.mtiles = p.mtiles;
  if (ks == 3) launch_wgrad_k<3>(a, p, st);
  else launch_wgrad_k<1>(a, p, st);
  const size_t n = (size_t)ks * ks * cin * cout;
  k_sum_splits<<<blocks_for(n), kBlock, 0, st>>>(part, p.nsplit, n, dw);
  if (db) {
    const dim3 g((unsigned)p.colsplit, (unsigned)((cout + kBlock - 1) / kBlock));
    k_colsum_part<<<g, kBlock, 0, st>>>(dy, a.npix, cout, p.colsp, bpart);
    k_sum_splits<<<blocks_for(cout), kBlock, 0, st>>>(bpart, p.colsplit, cout, db);
  }
}

void conv_dgrad(const float* dy, const float* w, float* dx, float* wflip, int batch, int H, int W,
                int cin, int cout, int ks, hipStream_t st) {
  const size_t n = (size_t)ks * ks * cin * cout;
  k_flip_weights<<<blocks_for(n), kBlock, 0, st>>>(w, ks * ks, cin, cout, wflip);
  conv_fwd(dy, wflip, nullptr, dx, batch, H, W, cout, cin, ks, 0, st);
}

// ----------------------------------------------------------------- network plan

struct Layer {
  int ks, cin, cout;
  size_t w_off, b_off;   // floats into the parameter vector
};

struct Plan {
  int L, B, H, W;
  std::vector<int> ch;          // channels per level
  std::vector<Layer> layers;    // enc0a, enc0b, ..., dec{L-2}a, ..., head
  int64_t n_params;
  // activation offsets (floats): pool_l (l >= 1), a_l, e_l; cat_l, da_l, db_l (l <= L-2)
  std::vector<size_t> pool, a, e, cat, da, db;
  size_t act_floats;
  // work offsets (floats): gradients of each activation, flipped weights, wgrad scratch
  std::vector<size_t> gpool, ga, ge, gcat, gda, gdb, gskip;
  size_t wflip, wgrad, work_bytes;
  int Hl(int l) const { return H >> l; }
  int Wl(int l) const { return W >> l; }
  size_t px(int l) const { return (size_t)B * Hl(l) * Wl(l); }
  const Layer& enc(int l, int k) const { return layers[2 * l + k]; }
  const Layer& dec(int l, int k) const { return layers[2 * L + 2 * (L - 2 - l) + k]; }
  const Layer& head() const { return layers.back(); }
};

lbm_status make_plan(const wsn_config* c, int32_t batch, Plan* P) {
  if (!c) return fail(LBM_EINVAL, "config is NULL");
  if (c->levels < 1 || c->levels > 8) return fail(LBM_EINVAL, "levels must be 1..8");
  if (c->base < 1 || c->in_ch < 1 || c->out_ch < 1)
    return fail(LBM_EINVAL, "base, in_ch and out_ch must be >= 1");
  if ((int64_t)c->base << (c->levels - 1) > 4096) return fail(LBM_EINVAL, "too many channels");
  const int div = 1 << (c->levels - 1);
  if (c->height < div || c->height % div)
    return fail(LBM_EINVAL, "height must be a multiple of 2^(levels-1) = %d", div);
  if (c->width % (16 * div))
    return fail(LBM_EINVAL, "width must be a multiple of 16 * 2^(levels-1) = %d", 16 * div);
  if (batch < 1) return fail(LBM_EINVAL, "batch must be >= 1");
  if ((int64_t)batch * c->height * c->width >= (1ll << 31))
    return fail(LBM_EINVAL, "more than 2^31 pixels");
  P->L = c->levels;
  P->B = batch;
  P->H = c->height;
  P->W = c->width;
  P->ch.clear();
  for (int l = 0; l < P->L; ++l) P->ch.push_back(c->base << l);
  P->layers.clear();
  size_t o = 0;
  auto add = [&](int ks, int ci, int co) {
    Layer y;
    y.ks = ks;
    y.cin = ci;
    y.cout = co;
    y.w_off = o;
    o += (size_t)ks * ks * ci * co;
    y.b_off = o;
    o += co;
    P->layers.push_back(y);
  };
  int cin = c->in_ch;
  for (int l = 0; l < P->L; ++l) {
    add(3, cin, P->ch[l]);
    add(3, P->ch[l], P->ch[l]);
    cin = P->ch[l];
  }
  for (int l = P->L - 2; l >= 0; --l) {
    add(3, P->ch[l + 1] + P->ch[l], P->ch[l]);
    add(3, P->ch[l], P->ch[l]);
  }
  add(1, P->ch[0], c->out_ch);
  P->n_params = (int64_t)o;

  const int L = P->L;
  P->pool.assign(L, 0);
  P->a.assign(L, 0);
  P->e.assign(L, 0);
  P->cat.assign(L, 0);
  P->da.assign(L, 0);
  P->db.assign(L, 0);
  size_t f = 0;
  auto take = [&](size_t n) {
    const size_t at = f;
    f += (n + 63) / 64 * 64;   // 256-byte aligned offsets
    return at;
  };
  for (int l = 0; l < L; ++l) {
    if (l > 0) P->pool[l] = take(P->px(l) * P->ch[l - 1]);
    P->a[l] = take(P->px(l) * P->ch[l]);
    P->e[l] = take(P->px(l) * P->ch[l]);
  }
  for (int l = L - 2; l >= 0; --l) {
    P->cat[l] = take(P->px(l) * (P->ch[l + 1] + P->ch[l]));
    P->da[l] = take(P->px(l) * P->ch[l]);
    P->db[l] = take(P->px(l) * P->ch[l]);
  }
  P->act_floats = f;

  P->gpool.assign(L, 0);
  P->ga.assign(L, 0);
  P->ge.assign(L, 0);
  P->gcat.assign(L, 0);
  P->gda.assign(L, 0);
  P->gdb.assign(L, 0);
  P->gskip.assign(L, 0);
  f = 0;
  for (int l = 0; l < L; ++l) {
    if (l > 0) P->gpool[l] = take(P->px(l) * P->ch[l - 1]);
    P->ga[l] = take(P->px(l) * P->ch[l]);
    P->ge[l] = take(P->px(l) * P->ch[l]);
  }
  for (int l = L - 2; l >= 0; --l) {
    P->gcat[l] = take(P->px(l) * (P->ch[l + 1] + P->ch[l]));
    P->gda[l] = take(P->px(l) * P->ch[l]);
    P->gdb[l] = take(P->px(l) * P->ch[l]);
    P->gskip[l] = take(P->px(l) * P->ch[l]);
  }
  size_t wmax = 0, gmax = 0;
  auto consider = [&](const Layer& y, int l) {
    const size_t n = (size_t)y.ks * y.ks * y.cin * y.cout;
    if (n > wmax) wmax = n;
    const size_t g = wgrad_bytes(wgrad_plan(P->B, P->Hl(l), P->Wl(l), y.cin, y.cout, y.ks));
    if (g > gmax) gmax = g;
  };
  for (int l = 0; l < L; ++l) {
    consider(P->enc(l, 0), l);
    consider(P->enc(l, 1), l);
  }
  for (int l = L - 2; l >= 0; --l) {
    consider(P->dec(l, 0), l);
    consider(P->dec(l, 1), l);
  }
  consider(P->head(), 0);
  P->wflip = take(wmax);
  P->wgrad = take(gmax / 4 + 64);
  P->work_bytes = f * 4;
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status wsn_conv_forward(const float* x, const float* w, const float* bias, float* y,
                            int32_t batch, int32_t height, int32_t width, int32_t cin,
                            int32_t cout, int32_t ks, int32_t relu, void* stream) {
  lbm_status s = check_conv(batch, height, width, cin, cout, ks, "wsn_conv_forward");
  if (s != LBM_OK) return s;
  if (!x || !w || !y) return fail(LBM_EINVAL, "wsn_conv_forward: NULL buffer");
  conv_fwd(x, w, bias, y, batch, height, width, cin, cout, ks, relu ? 1 : 0, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_conv_backward_data(const float* dy, const float* w, float* dx, float* wflip,
                                  int32_t batch, int32_t height, int32_t width, int32_t cin,
                                  int32_t cout, int32_t ks, void* stream) {
  lbm_status s = check_conv(batch, height, width, cin, cout, ks, "wsn_conv_backward_data");
  if (s != LBM_OK) return s;
  if (!dy || !w || !dx || !wflip) return fail(LBM_EINVAL, "wsn_conv_backward_data: NULL buffer");
  conv_dgrad(dy, w, dx, wflip, batch, height, width, cin, cout, ks, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_conv_wgrad_work(int32_t batch, int32_t height, int32_t width, int32_t cin,
                               int32_t cout, int32_t ks, size_t* work_bytes) {
  lbm_status s = check_conv(batch, height, width, cin, cout, ks, "wsn_conv_wgrad_work");
  if (s != LBM_OK) return s;
  if (!work_bytes) return fail(LBM_EINVAL, "work_bytes is NULL");
  *work_bytes = wgrad_bytes(wgrad_plan(batch, height, width, cin, cout, ks));
  return ok();
}

lbm_status wsn_conv_backward_weight(const float* x, const float* dy, float* dw, float* db,
                                    int32_t batch, int32_t height, int32_t width, int32_t cin,
                                    int32_t cout, int32_t ks, void* work, size_t work_bytes,
                                    void* stream) {
  lbm_status s = check_conv(batch, height, width, cin, cout, ks, "wsn_conv_backward_weight");
  if (s != LBM_OK) return s;
  if (!x || !dy || !dw || !work) return fail(LBM_EINVAL, "wsn_conv_backward_weight: NULL buffer");
  const size_t need = wgrad_bytes(wgrad_plan(batch, height, width, cin, cout, ks));
  if (work_bytes < need)
    return fail(LBM_ENOMEM, "wsn_conv_backward_weight: work needs %zu bytes, got %zu", need,
                work_bytes);
  conv_wgrad(x, dy, dw, db, batch, height, width, cin, cout, ks, work, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_relu_backward(const float* y, float* g, int64_t n, void* stream) {
  if (!y || !g || n < 0) return fail(LBM_EINVAL, "wsn_relu_backward: bad argument");
  if (n == 0) return ok();
  k_relu_bwd<<<blocks_for((size_t)n), kBlock, 0, (hipStream_t)stream>>>(y, g, (size_t)n);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_pool_forward(const float* x, float* y, int32_t batch, int32_t height, int32_t width,
                            int32_t c, void* stream) {
  lbm_status s = check_image(batch, height, width, c, "wsn_pool_forward");
  if (s != LBM_OK) return s;
  if (height % 2 || width % 2) return fail(LBM_EINVAL, "wsn_pool_forward: odd height or width");
  if (!x || !y) return fail(LBM_EINVAL, "wsn_pool_forward: NULL buffer");
  const size_t n = (size_t)batch * (height / 2) * (width / 2) * c;
  k_pool_fwd<<<blocks_for(n), kBlock, 0, (hipStream_t)stream>>>(x, y, height / 2, width / 2, c, n);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_pool_backward(const float* x, const float* gy, const float* add, float* gx,
                             int32_t batch, int32_t height, int32_t width, int32_t c, void* stream) {
  lbm_status s = check_image(batch, height, width, c, "wsn_pool_backward");
  if (s != LBM_OK) return s;
  if (height % 2 || width % 2) return fail(LBM_EINVAL, "wsn_pool_backward: odd height or width");
  if (!x || !gy || !gx) return fail(LBM_EINVAL, "wsn_pool_backward: NULL buffer");
  const size_t n = (size_t)batch * (height / 2) * (width / 2) * c;
  k_pool_bwd<<<blocks_for(n), kBlock, 0, (hipStream_t)stream>>>(x, gy, add, gx, height / 2,
                                                                  width / 2, c, n);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_upcat_forward(const float* deep, const float* skip, float* cat, int32_t batch,
                             int32_t height, int32_t width, int32_t c1, int32_t c2, void* stream) {
  lbm_status s = check_image(batch, height, width, c1 + c2, "wsn_upcat_forward");
  if (s != LBM_OK) return s;
  if (c1 < 1 || c2 < 1 || height % 2 || width % 2)
    return fail(LBM_EINVAL, "wsn_upcat_forward: bad channels or odd size");
  if (!deep || !skip || !cat) return fail(LBM_EINVAL, "wsn_upcat_forward: NULL buffer");
  const size_t n = (size_t)batch * height * width * (c1 + c2);
  k_upcat_fwd<<<blocks_for(n), kBlock, 0, (hipStream_t)stream>>>(deep, skip, cat, height, width,
                                                                   c1, c2, n);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_upcat_backward(const float* gcat, float* gdeep, float* gskip, int32_t batch,
                              int32_t height, int32_t width, int32_t c1, int32_t c2, void* stream) {
  lbm_status s = check_image(batch, height, width, c1 + c2, "wsn_upcat_backward");
  if (s != LBM_OK) return s;
  if (c1 < 1 || c2 < 1 || height % 2 || width % 2)
    return fail(LBM_EINVAL, "wsn_upcat_backward: bad channels or odd size");
  if (!gcat || !gdeep || !gskip) return fail(LBM_EINVAL, "wsn_upcat_backward: NULL buffer");
  const size_t n1 = (size_t)batch * (height / 2) * (width / 2) * c1;
  const size_t n2 = (size_t)batch * height * width * c2;
  k_upcat_bwd<<<blocks_for(n1 + n2), kBlock, 0, (hipStream_t)stream>>>(gcat, gdeep, gskip, height,
                                                                         width, c1, c2, n1, n2);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_mse_work(int64_t npix, size_t* work_bytes) {
  if (npix < 1 || npix >= (1ll << 31) || !work_bytes) return fail(LBM_EINVAL, "wsn_mse_work: bad argument");
  *work_bytes = align256((size_t)blocks_for((size_t)npix) * 2 * sizeof(double)) + 256;
  return ok();
}

lbm_status wsn_masked_mse(const float* pred, const float* target, const uint8_t* solid,
                          int64_t npix, int32_t channels, double* loss, float* grad, void* work,
                          size_t work_bytes, void* stream) {
  size_t need = 0;
  lbm_status s = wsn_mse_work(npix, &need);
  if (s != LBM_OK) return s;
  if (channels < 1) return fail(LBM_EINVAL, "wsn_masked_mse: channels must be >= 1");
  if (!pred || !target || !solid || !loss || !grad || !work)
    return fail(LBM_EINVAL, "wsn_masked_mse: NULL buffer");
  if (work_bytes < need) return fail(LBM_ENOMEM, "wsn_masked_mse: work needs %zu bytes", need);
  hipStream_t st = (hipStream_t)stream;
  const int nb = (int)blocks_for((size_t)npix);
  double* part = (double*)work;
  double* fin = (double*)((char*)work + align256((size_t)nb * 2 * sizeof(double)));
  k_mse_part<<<nb, kBlock, 0, st>>>(pred, target, solid, (int)npix, channels, part);
  k_mse_final<<<1, kBlock, 0, st>>>(part, nb, channels, fin);
  k_mse_grad<<<blocks_for((size_t)npix * channels), kBlock, 0, st>>>(pred, target, solid, fin,
                                                                      (int)npix, channels, grad);
  HIP_TRY(hipMemcpyAsync(loss, fin, sizeof(double), hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_adam(float* p, const float* g, float* m, float* v, int64_t n, double lr, double b1,
                    double b2, double eps, int64_t t, void* stream) {
  if (!p || !g || !m || !v || n < 0) return fail(LBM_EINVAL, "wsn_adam: bad buffer or size");
  if (t < 1) return fail(LBM_EINVAL, "wsn_adam: step number t must be >= 1");
  if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(LBM_EINVAL, "wsn_adam: need lr > 0, 0 <= b1, b2 < 1, eps > 0");
  if (n == 0) return ok();
  const double bc1 = 1.0 - pow(b1, (double)t), bc2 = 1.0 - pow(b2, (double)t);
  k_adam<<<blocks_for((size_t)n), kBlock, 0, (hipStream_t)stream>>>(
      p, g, m, v, (size_t)n, (float)lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2),
      (float)eps, (float)bc1, (float)bc2);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_query_sizes(const wsn_config* cfg, int32_t batch, int64_t* n_params,
                           size_t* act_bytes, size_t* work_bytes) {
  Plan P;
  lbm_status s = make_plan(cfg, batch, &P);
  if (s != LBM_OK) return s;
  if (n_params) *n_params = P.n_params;
  if (act_bytes) *act_bytes = P.act_floats * 4;
  if (work_bytes) *work_bytes = P.work_bytes;
  return ok();
}

lbm_status wsn_forward(const wsn_config* cfg, int32_t batch, const float* params, const float* x,
                       float* y, void* act, void* stream) {
  Plan P;
  lbm_status s = make_plan(cfg, batch, &P);
  if (s != LBM_OK) return s;
  if (!params || !x || !y || !act) return fail(LBM_EINVAL, "wsn_forward: NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  float* A = (float*)act;
  const int L = P.L, B = P.B;
  auto conv = [&](const Layer& y_, const float* in, float* out, int l, int relu) {
    conv_fwd(in, params + y_.w_off, params + y_.b_off, out, B, P.Hl(l), P.Wl(l), y_.cin, y_.cout,
             y_.ks, relu, st);
  };
  const float* in = x;
  for (int l = 0; l < L; ++l) {
    if (l > 0) {
      const size_t n = P.px(l) * P.ch[l - 1];
      k_pool_fwd<<<blocks_for(n), kBlock, 0, st>>>(A + P.e[l - 1], A + P.pool[l], P.Hl(l), P.Wl(l),
                                                   P.ch[l - 1], n);
      in = A + P.pool[l];
    }
    conv(P.enc(l, 0), in, A + P.a[l], l, 1);
    conv(P.enc(l, 1), A + P.a[l], A + P.e[l], l, 1);
  }
  const float* deep = A + P.e[L - 1];
  for (int l = L - 2; l >= 0; --l) {
    const size_t n = P.px(l) * (P.ch[l + 1] + P.ch[l]);
    k_upcat_fwd<<<blocks_for(n), kBlock, 0, st>>>(deep, A + P.e[l], A + P.cat[l], P.Hl(l), P.Wl(l),
                                                  P.ch[l + 1], P.ch[l], n);
    conv(P.dec(l, 0), A + P.cat[l], A + P.da[l], l, 1);
    conv(P.dec(l, 1), A + P.da[l], A + P.db[l], l, 1);
    deep = A + P.db[l];
  }
  conv(P.head(), deep, y, 0, 0);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_backward(const wsn_config* cfg, int32_t batch, const float* params, const float* x,
                        const float* dy, float* grad, const void* act, void* work, void* stream) {
  Plan P;
  lbm_status s = make_plan(cfg, batch, &P);
  if (s != LBM_OK) return s;
  if (!params || !x || !dy || !grad || !act || !work)
    return fail(LBM_EINVAL, "wsn_backward: NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  const float* A = (const float*)act;
  float* Wk = (float*)work;
  float* wflip = Wk + P.wflip;
  float* scratch = Wk + P.wgrad;
  const int L = P.L, B = P.B;
  // gradient of layer y_ whose input is `in` and output gradient `g` (already
  // through the ReLU); the input gradient goes to gin (nullptr: not needed)
  auto layer_bwd = [&](const Layer& y_, const float* in, const float* g, float* gin, int l) {
    conv_wgrad(in, g, grad + y_.w_off, grad + y_.b_off, B, P.Hl(l), P.Wl(l), y_.cin, y_.cout,
               y_.ks, scratch, st);
    if (gin)
      conv_dgrad(g, params + y_.w_off, gin, wflip, B, P.Hl(l), P.Wl(l), y_.cin, y_.cout, y_.ks, st);
  };
  auto relu_bwd = [&](const float* yv, float* g, size_t n) {
    k_relu_bwd<<<blocks_for(n), kBlock, 0, st>>>(yv, g, n);
  };
  // head (no ReLU): its input is the output of the last decoder (or of level 0)
  const float* head_in = L >= 2 ? A + P.db[0] : A + P.e[0];
  float* g_top = L >= 2 ? Wk + P.gdb[0] : Wk + P.ge[0];
  layer_bwd(P.head(), head_in, dy, g_top, 0);
  for (int l = 0; l <= L - 2; ++l) {
    const size_t n = P.px(l) * P.ch[l];
    relu_bwd(A + P.db[l], Wk + P.gdb[l], n);
    layer_bwd(P.dec(l, 1), A + P.da[l], Wk + P.gdb[l], Wk + P.gda[l], l);
    relu_bwd(A + P.da[l], Wk + P.gda[l], n);
    layer_bwd(P.dec(l, 0), A + P.cat[l], Wk + P.gda[l], Wk + P.gcat[l], l);
    // the decoder's input came from the level below: its decoder output, or the bottom encoder
    float* gdeep = l + 1 <= L - 2 ? Wk + P.gdb[l + 1] : Wk + P.ge[L - 1];
    const size_t n1 = P.px(l + 1) * P.ch[l + 1], n2 = P.px(l) * P.ch[l];
    k_upcat_bwd<<<blocks_for(n1 + n2), kBlock, 0, st>>>(Wk + P.gcat[l], gdeep, Wk + P.gskip[l],
                                                        P.Hl(l), P.Wl(l), P.ch[l + 1], P.ch[l], n1,
                                                        n2);
  }
  for (int l = L - 1; l >= 0; --l) {
    const size_t n = P.px(l) * P.ch[l];
    // ge[l] holds the gradient of the level's output: written above for the
    // bottom level (and for a single level by the head), else by pool backward
    relu_bwd(A + P.e[l], Wk + P.ge[l], n);
    layer_bwd(P.enc(l, 1), A + P.a[l], Wk + P.ge[l], Wk + P.ga[l], l);
    relu_bwd(A + P.a[l], Wk + P.ga[l], n);
    const float* in = l > 0 ? A + P.pool[l] : x;
    layer_bwd(P.enc(l, 0), in, Wk + P.ga[l], l > 0 ? Wk + P.gpool[l] : nullptr, l);
    if (l > 0) {
      // gradient of level l - 1's output: through the pooling, plus its skip
      const size_t np = P.px(l) * P.ch[l - 1];
      k_pool_bwd<<<blocks_for(np), kBlock, 0, st>>>(A + P.e[l - 1], Wk + P.gpool[l],
                                                    Wk + P.gskip[l - 1], Wk + P.ge[l - 1],
                                                    P.Hl(l), P.Wl(l), P.ch[l - 1], np);
    }
  }
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_pack_input(const uint8_t* solid, const float* feat, int32_t batch, int32_t height,
                          int32_t width, float* x, void* stream) {
  lbm_status s = check_image(batch, height, width, 2, "wsn_pack_input");
  if (s != LBM_OK) return s;
  if (!solid || !feat || !x) return fail(LBM_EINVAL, "wsn_pack_input: NULL buffer");
  const size_t n = (size_t)batch * height * width;
  k_pack_input<<<blocks_for(n), kBlock, 0, (hipStream_t)stream>>>(solid, feat, height * width, n, x);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_column_profile(const uint8_t* solid, int32_t batch, int32_t height, int32_t width,
                              float* profile, void* stream) {
  lbm_status s = check_image(batch, height, width, 1, "wsn_column_profile");
  if (s != LBM_OK) return s;
  if (!solid || !profile) return fail(LBM_EINVAL, "wsn_column_profile: NULL buffer");
  if (width > 16384) return fail(LBM_EINVAL, "wsn_column_profile: width above 16384");
  k_column_profile<<<(unsigned)batch, kBlock, (size_t)width * sizeof(float), (hipStream_t)stream>>>(
      solid, height, width, profile);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_pack_input_profile(const uint8_t* solid, const float* feat, const float* profile,
                                  float scale, int32_t batch, int32_t height, int32_t width,
                                  float* x, void* stream) {
  lbm_status s = check_image(batch, height, width, 3, "wsn_pack_input_profile");
  if (s != LBM_OK) return s;
  if (!solid || !feat || !profile || !x) return fail(LBM_EINVAL, "wsn_pack_input_profile: NULL buffer");
  if (!isfinite(scale)) return fail(LBM_EINVAL, "wsn_pack_input_profile: scale not finite");
  const size_t n = (size_t)batch * height * width;
  k_pack_input_profile<<<blocks_for(n), kBlock, 0, (hipStream_t)stream>>>(solid, feat, profile, scale,
                                                                           height * width, width, n, x);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_fields_to_nhwc(const float* rho, const float* u, const float* shift,
                              const float* slope, const float* scale, int32_t batch,
                              int32_t height, int32_t width, float* y, void* stream) {
  lbm_status s = check_image(batch, height, width, 3, "wsn_fields_to_nhwc");
  if (s != LBM_OK) return s;
  if (!rho || !u || !shift || !scale || !y) return fail(LBM_EINVAL, "wsn_fields_to_nhwc: NULL buffer");
  const size_t n = (size_t)batch * height * width;
  k_fields_to_nhwc<<<blocks_for(n), kBlock, 0, (hipStream_t)stream>>>(rho, u, shift, slope, scale,
                                                                       height * width, width, n, y);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_nhwc_to_fields(const float* y, const float* shift, const float* slope,
                              const float* scale, const uint8_t* keep_u, int32_t batch,
                              int32_t height, int32_t width, float* rho, float* u, int32_t* bad,
                              void* stream) {
  lbm_status s = check_image(batch, height, width, 3, "wsn_nhwc_to_fields");
  if (s != LBM_OK) return s;
  if (!y || !shift || !scale || !rho || !u || !bad)
    return fail(LBM_EINVAL, "wsn_nhwc_to_fields: NULL buffer");
  const size_t n = (size_t)batch * height * width;
  HIP_TRY(hipMemsetAsync(bad, 0, (size_t)batch * sizeof(int32_t), (hipStream_t)stream));
  k_nhwc_to_fields<<<blocks_for(n), kBlock, 0, (hipStream_t)stream>>>(
      y, shift, slope, scale, keep_u, height * width, width, n, rho, u, bad);
  HIP_TRY(hipGetLastError());
  return ok();
}

lbm_status wsn_mirror(const void* in, int32_t elem_bytes, int32_t batch, int32_t height,
                      int32_t width, int32_t channels, int32_t flip_h, int32_t flip_w,
                      const float* scale, int32_t accumulate, void* out, void* stream) {
  lbm_status s = check_image(batch, height, width, channels, "wsn_mirror");
  if (s != LBM_OK) return s;
  if (!in || !out) return fail(LBM_EINVAL, "wsn_mirror: NULL buffer");
  if (in == out) return fail(LBM_EINVAL, "wsn_mirror: in and out must not overlap");
  if (elem_bytes != 1 && elem_bytes != 4)
    return fail(LBM_EINVAL, "wsn_mirror: elem_bytes must be 1 or 4, got %d", elem_bytes);
  if ((flip_h != 0 && flip_h != 1) || (flip_w != 0 && flip_w != 1) ||
      (accumulate != 0 && accumulate != 1))
    return fail(LBM_EINVAL, "wsn_mirror: flip_h, flip_w and accumulate must be 0 or 1");
  if ((scale || accumulate) && elem_bytes != 4)
    return fail(LBM_EINVAL, "wsn_mirror: scale and accumulate need float elements");
  if (scale && channels > kMirrorC)
    return fail(LBM_EINVAL, "wsn_mirror: scale covers at most %d channels", kMirrorC);
  if ((int64_t)batch * height * width >= (1ll << 31))
    return fail(LBM_EINVAL, "wsn_mirror: more than 2^31 pixels");
  MirrorScale sc{};
  if (scale)
    for (int k = 0; k < channels; ++k) sc.s[k] = scale[k];
  const size_t n = (size_t)batch * height * width;
  const unsigned g = blocks_for(n);
  hipStream_t st = (hipStream_t)stream;
  const float* fi = (const float*)in;
  float* fo = (float*)out;
  if (elem_bytes == 1)
    k_mirror<uint8_t, false, false><<<g, kBlock, 0, st>>>((const uint8_t*)in, height, width,
                                                          channels, flip_h, flip_w, sc, n,
                                                          (uint8_t*)out);
  else if (scale && accumulate)
    k_mirror<float, true, true><<<g, kBlock, 0, st>>>(fi, height, width, channels, flip_h, flip_w,
                                                      sc, n, fo);
  else if (scale)
    k_mirror<float, true, false><<<g, kBlock, 0, st>>>(fi, height, width, channels, flip_h,
                                                       flip_w, sc, n, fo);
  else if (accumulate)
    k_mirror<float, false, true><<<g, kBlock, 0, st>>>(fi, height, width, channels, flip_h,
                                                       flip_w, sc, n, fo);
  else
    k_mirror<float, false, false><<<g, kBlock, 0, st>>>(fi, height, width, channels, flip_h,
                                                        flip_w, sc, n, fo);
  HIP_TRY(hipGetLastError());
  return ok();
}


}  // extern "C"
