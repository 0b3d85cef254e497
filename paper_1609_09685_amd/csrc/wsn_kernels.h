// Device kernels of the warm-start network (a small U-Net, FP32).
//
// Images are NHWC float32, [B][H][W][C].  A convolution has ks x ks taps
// (ks = 3 with zero padding 1, or ks = 1) in row-major order over (dy, dx),
// weights w[t][ci][co] and a bias b[co]:
//     y[b, h, x, co] = b[co] + sum_t sum_ci x[b, h + dy_t, x + dx_t, ci] w[t, ci, co].
//
// Convolutions are implicit GEMMs on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32: D[16x16] += A[16x4] B[4x16]; lane l holds
// A[l % 16][l / 16], B[l / 16][l % 16] and D[4 (l / 16) + r][l % 16], r < 4):
//   forward      M = pixels of a 64-pixel tile, N = output channels, K = (tap, ci);
//                the block stages the tile's input patch (tile plus halo) for a
//                chunk of 8 input channels and the matching weights in LDS, and
//                every tap reads its shifted window out of the one patch;
//   data grad    the forward kernel on the output gradient with the weights
//                flipped in space and transposed (w'[t][co][ci] = w[T-1-t][ci][co]);
//   weight grad  M = ci, N = co, K = pixels, split over pixel ranges into
//                partial sums that a second kernel adds in a fixed order
//                (deterministic, no atomics); for 3x3 convolutions one block
//                serves all nine taps from one staged input patch.
// LDS row strides are 16 (mod 32) words, so the two halves of a wavefront's
// operand reads fall on disjoint banks.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace wsn {

constexpr int kBlock = 256;
constexpr int kCK = 8;        // input channels per K chunk of the forward kernel
constexpr int kTile = 64;     // pixels per forward tile

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Waves of a block over an (SM x 16) x (SN x 16) output tile: WM x WN waves,
// each FM x FN MFMA tiles; fewer than 4 waves compute when the tile is small.
template <int SM, int SN>
struct WaveGrid {
  static constexpr int WN0 = SN < 2 ? SN : 2;
  static constexpr int WM = SM < 4 / WN0 ? SM : 4 / WN0;
  static constexpr int WN = WM * WN0 < 4 ? (SN < 4 / WM ? SN : 4 / WM) : WN0;
  static constexpr int FM = SM / WM;
  static constexpr int FN = SN / WN;
  static_assert(WM * FM == SM && WN * FN == SN && WM * WN <= 4, "wave grid");
};

// Row stride (words) >= n with stride = 16 (mod 32).
constexpr int lds_stride(int n) { return (n + 15) / 32 * 32 + 16; }

struct ConvArgs {
  const float* __restrict__ x;      // [B][H][W][cin]
  const float* __restrict__ w;      // [T][cin][cout]
  const float* __restrict__ bias;   // [cout] or nullptr
  float* __restrict__ y;            // [B][H][W][cout]
  int H, W, cin, cout;
  int tw_log2, th;                  // tile: th rows x (1 << tw_log2) columns, th * tw = 64
  int tiles_w, tiles_h;             // W / tw, ceil(H / th)
  int relu;
};

// V4: cin and cout are multiples of 4 and x, w are 16-byte aligned, so the
// staging moves four channels per load (the channel runs are contiguous).
template <int KS, int NT, bool V4>
__global__ __launch_bounds__(kBlock) void k_conv_fwd(const ConvArgs a) {
  constexpr int R = KS / 2, T = KS * KS;
  using G = WaveGrid<kTile / 16, NT / 16>;
  // patch pixels for the widest tile (64 x 1 plus halo); narrower tiles need fewer
  constexpr int PMAX = (1 + 2 * R) * (kTile + 2 * R) > (4 + 2 * R) * (16 + 2 * R)
                           ? (1 + 2 * R) * (kTile + 2 * R)
                           : (4 + 2 * R) * (16 + 2 * R);
  constexpr int PS = lds_stride(PMAX), NS = lds_stride(NT);
  __shared__ float xs[kCK][PS];
  __shared__ __attribute__((aligned(16))) float ws[T][kCK][NS];

  const int tw = 1 << a.tw_log2;
  const int tile = blockIdx.x;
  const int twi = tile % a.tiles_w;
  const int rest = tile / a.tiles_w;
  const int thi = rest % a.tiles_h;
  const int b = rest / a.tiles_h;
  const int h0 = thi * a.th, w0 = twi * tw;
  const int n0 = blockIdx.y * NT;
  const int PC = tw + 2 * R, NP = (a.th + 2 * R) * PC;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave % G::WM, wn = wave / G::WM;
  const bool active = wave < G::WM * G::WN;
  const size_t img = (size_t)b * a.H;

  v4f acc[G::FM][G::FN];
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  // patch offset of each of this lane's A rows (pixel m of the tile)
  int poff[G::FM];
#pragma unroll
  for (int i = 0; i < G::FM; ++i) {
    const int m = (wm * G::FM + i) * 16 + (lane & 15);
    poff[i] = (m >> a.tw_log2) * PC + (m & (tw - 1));
  }
  const int kq = lane >> 4;

  // The input patch of one chunk of kCK channels in registers: the next
  // chunk's patch loads are issued right after this chunk is in LDS, so they
  // are in flight during its matrix-core work.  The weights, read by every
  // block and mostly found in the L2, are staged directly.
  constexpr int XR = V4 ? (PMAX * (kCK / 4) + kBlock - 1) / kBlock : (PMAX * kCK + kBlock - 1) / kBlock;
  v4f xr[V4 ? XR : 1];
  float xs1[V4 ? 1 : XR];
  auto fetch = [&](int c0) {
    if constexpr (V4) {
#pragma unroll
      for (int k = 0; k < XR; ++k) {
        const int e = threadIdx.x + k * kBlock;   // (pixel, group of 4 channels)
        const int cq = e % (kCK / 4), p = e / (kCK / 4);
        const int pr = p / PC, pc = p - pr * PC;
        const int h = h0 - R + pr, w = w0 - R + pc, ci = c0 + 4 * cq;
        v4f v = v4f{0.f, 0.f, 0.f, 0.f};
        if (e < NP * (kCK / 4) && h >= 0 && h < a.H && w >= 0 && w < a.W && ci < a.cin)
          v = *(const v4f*)(a.x + ((img + h) * a.W + w) * a.cin + ci);
        xr[k] = v;
      }
    } else {
#pragma unroll
      for (int k = 0; k < XR; ++k) {
        const int e = threadIdx.x + k * kBlock;
        const int c = e % kCK, p = e / kCK;
        const int pr = p / PC, pc = p - pr * PC;
        const int h = h0 - R + pr, w = w0 - R + pc, ci = c0 + c;
        float v = 0.f;
        if (e < NP * kCK && h >= 0 && h < a.H && w >= 0 && w < a.W && ci < a.cin)
          v = a.x[((img + h) * a.W + w) * a.cin + ci];
        xs1[k] = v;
      }
    }
  };
  fetch(0);
  for (int c0 = 0; c0 < a.cin; c0 += kCK) {
    __syncthreads();   // the previous chunk's reads of xs / ws are done
    if constexpr (V4) {
#pragma unroll
      for (int k = 0; k < XR; ++k) {
        const int e = threadIdx.x + k * kBlock;
        if (e < NP * (kCK / 4)) {
          const int cq = e % (kCK / 4), p = e / (kCK / 4);
          xs[4 * cq + 0][p] = xr[k].x;
          xs[4 * cq + 1][p] = xr[k].y;
          xs[4 * cq + 2][p] = xr[k].z;
          xs[4 * cq + 3][p] = xr[k].w;
        }
      }
      for (int e = threadIdx.x; e < T * kCK * (NT / 4); e += kBlock) {
        const int n4 = e % (NT / 4), c = (e / (NT / 4)) % kCK, t = e / ((NT / 4) * kCK);
        const int ci = c0 + c, co = n0 + 4 * n4;
        v4f v = v4f{0.f, 0.f, 0.f, 0.f};
        if (ci < a.cin && co < a.cout) v = *(const v4f*)(a.w + ((size_t)t * a.cin + ci) * a.cout + co);
        *(v4f*)&ws[t][c][4 * n4] = v;
      }
    } else {
#pragma unroll
      for (int k = 0; k < XR; ++k) {
        const int e = threadIdx.x + k * kBlock;
        if (e < NP * kCK) xs[e % kCK][e / kCK] = xs1[k];
      }
      for (int e = threadIdx.x; e < T * kCK * NT; e += kBlock) {
        const int n = e % NT, c = (e / NT) % kCK, t = e / (NT * kCK);
        const int ci = c0 + c, co = n0 + n;
        float v = 0.f;
        if (ci < a.cin && co < a.cout) v = a.w[((size_t)t * a.cin + ci) * a.cout + co];
        ws[t][c][n] = v;
      }
    }
    __syncthreads();
    if (c0 + kCK < a.cin) fetch(c0 + kCK);   // uniform
    if (active) {
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int toff = (t / KS) * PC + (t % KS);
#pragma unroll
        for (int kk = 0; kk < kCK; kk += 4) {
          float av[G::FM], bv[G::FN];
#pragma unroll
          for (int i = 0; i < G::FM; ++i) av[i] = xs[kk + kq][poff[i] + toff];
#pragma unroll
          for (int j = 0; j < G::FN; ++j) bv[j] = ws[t][kk + kq][(wn * G::FN + j) * 16 + (lane & 15)];
#pragma unroll
          for (int i = 0; i < G::FM; ++i)
#pragma unroll
            for (int j = 0; j < G::FN; ++j) acc[i][j] = mfma4(av[i], bv[j], acc[i][j]);
        }
      }
    }
  }
  if (!active) return;
#pragma unroll
  for (int j = 0; j < G::FN; ++j) {
    const int co = n0 + (wn * G::FN + j) * 16 + (lane & 15);
    if (co >= a.cout) continue;
    const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = (wm * G::FM + i) * 16 + 4 * kq + r;
        const int h = h0 + (m >> a.tw_log2), w = w0 + (m & (tw - 1));
        if (h >= a.H) continue;
        float v = acc[i][j][r] + bias;
        if (a.relu) v = v > 0.f ? v : 0.f;
        a.y[((img + h) * a.W + w) * a.cout + co] = v;
      }
  }
}

struct WgradArgs {
  const float* __restrict__ x;     // layer input [B][H][W][cin]
  const float* __restrict__ dy;    // output gradient [B][H][W][cout]
  float* __restrict__ part;        // [nsplit][T][cin][cout]
  int H, W, cin, cout;
  int npix;                        // B * H * W
  int sp;                          // pixels per split, a multiple of 16
  int mtiles;                      // ceil(cin / TM)
};

// dW[t][ci][co] over the pixels of split blockIdx.x, tap and channel tiles from
// blockIdx.y.  16-pixel chunks never straddle a row (W % 16 == 0).
template <int KS, int TM, int NT>
__global__ __launch_bounds__(kBlock) void k_conv_wgrad(const WgradArgs a) {
  constexpr int R = KS / 2, T = KS * KS;
  using G = WaveGrid<TM / 16, NT / 16>;
  constexpr int XS = lds_stride(TM), GS = lds_stride(NT);
  __shared__ float xs[16][XS];
  __shared__ float gs[16][GS];

  const int t = blockIdx.y % T;
  const int mt = (blockIdx.y / T) % a.mtiles;
  const int nt = blockIdx.y / (T * a.mtiles);
  const int m0 = mt * TM, n0 = nt * NT;
  const int dyo = t / KS - R, dxo = t % KS - R;
  const int p_begin = blockIdx.x * a.sp;
  const int p_end = min(p_begin + a.sp, a.npix);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave % G::WM, wn = wave / G::WM;
  const bool active = wave < G::WM * G::WN;
  const int kq = lane >> 4;

  v4f acc[G::FM][G::FN];
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  for (int p0 = p_begin; p0 < p_end; p0 += 16) {
    // the chunk's row: image b, row h, columns w0 .. w0 + 15
    const int w0 = p0 % a.W;
    const int bh = p0 / a.W;
    const int h = bh % a.H;
    const int hs = h + dyo;
    const bool row_ok = hs >= 0 && hs < a.H;
    const size_t xrow = ((size_t)(bh + dyo)) * a.W;   // same image when row_ok
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * TM; e += kBlock) {
      const int m = e % TM, j = e / TM;
      const int ws = w0 + j + dxo, ci = m0 + m;
      float v = 0.f;
      if (row_ok && p0 + j < p_end && ws >= 0 && ws < a.W && ci < a.cin)
        v = a.x[(xrow + ws) * a.cin + ci];
      xs[j][m] = v;
    }
    for (int e = threadIdx.x; e < 16 * NT; e += kBlock) {
      const int n = e % NT, j = e / NT;
      const int co = n0 + n;
      float v = 0.f;
      if (p0 + j < p_end && co < a.cout) v = a.dy[((size_t)p0 + j) * a.cout + co];
      gs[j][n] = v;
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        float av[G::FM], bv[G::FN];
#pragma unroll
        for (int i = 0; i < G::FM; ++i) av[i] = xs[kk + kq][(wm * G::FM + i) * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < G::FN; ++j) bv[j] = gs[kk + kq][(wn * G::FN + j) * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < G::FM; ++i)
#pragma unroll
          for (int j = 0; j < G::FN; ++j) acc[i][j] = mfma4(av[i], bv[j], acc[i][j]);
      }
    }
  }
  if (!active) return;
  float* out = a.part + ((size_t)blockIdx.x * T + t) * a.cin * a.cout;
#pragma unroll
  for (int j = 0; j < G::FN; ++j) {
    const int co = n0 + (wn * G::FN + j) * 16 + (lane & 15);
    if (co >= a.cout) continue;
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ci = m0 + (wm * G::FM + i) * 16 + 4 * kq + r;
        if (ci < a.cin) out[(size_t)ci * a.cout + co] = acc[i][j][r];
      }
  }
}

// Weight gradient of a 3x3 convolution with all nine taps in one block:
// dW[t][ci][co] = sum_p x[p + d_t][ci] dy[p][co] over the pixels p of split
// blockIdx.x, channel tiles from blockIdx.y.  For every 16-pixel chunk of a row
// the block stages the output gradient once and the input patch of rows
// h - 1 .. h + 1, columns w0 - 1 .. w0 + 16 (zero outside the image); each tap
// reads its shifted window of that one patch, so both operands are read once
// per chunk instead of once per tap.  The staging is double-buffered: the
// loads of the next chunk are issued before the matrix-core work on this one
// and written to the other LDS buffer after it, one barrier per chunk.
// Partial sums go to part[split][t][ci][co] (added in a fixed order by
// k_sum_splits).
// V4: cin and cout are multiples of 4 and x, dy are 16-byte aligned, so the
// staging moves four channels per load.
template <int TM, int NT, bool V4>
__global__ __launch_bounds__(kBlock) void k_conv_wgrad3(const WgradArgs a) {
  using G = WaveGrid<TM / 16, NT / 16>;
  constexpr int XS = lds_stride(TM), GS = lds_stride(NT);
  constexpr int VW = V4 ? 4 : 1;                      // channels per staged value
  constexpr int XN = 3 * 18 * TM / VW, GN = 16 * NT / VW;   // staged values per chunk
  constexpr int XR = (XN + kBlock - 1) / kBlock, GR = (GN + kBlock - 1) / kBlock;
  using SV = typename std::conditional<V4, v4f, float>::type;
  __shared__ __attribute__((aligned(16))) float xs[2][3][18][XS];
  __shared__ __attribute__((aligned(16))) float gs[2][16][GS];

  const int mt = blockIdx.y % a.mtiles;
  const int nt = blockIdx.y / a.mtiles;
  const int m0 = mt * TM, n0 = nt * NT;
  const int p_begin = blockIdx.x * a.sp;
  const int p_end = min(p_begin + a.sp, a.npix);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave % G::WM, wn = wave / G::WM;
  const bool active = wave < G::WM * G::WN;
  const int kq = lane >> 4;

  // a chunk's values in registers: input patch, then output gradient (VW
  // channels per value)
  constexpr int TMV = TM / VW, NTV = NT / VW;
  SV xr[XR], gr[GR];
  auto fetch = [&](int p0) {
    const int w0 = p0 % a.W;   // the chunk's row: image b, row h, columns w0 .. w0 + 15
    const int bh = p0 / a.W;
    const int h = bh % a.H;
#pragma unroll
    for (int k = 0; k < XR; ++k) {
      const int e = threadIdx.x + k * kBlock;
      const int m = e % TMV, pc = (e / TMV) % 18, pr = e / (18 * TMV);
      const int hs = h + pr - 1, ws = w0 + pc - 1, ci = m0 + VW * m;
      SV v = SV{};
      if (e < XN && hs >= 0 && hs < a.H && ws >= 0 && ws < a.W && ci < a.cin)
        v = *(const SV*)(a.x + ((size_t)(bh + pr - 1) * a.W + ws) * a.cin + ci);
      xr[k] = v;
    }
#pragma unroll
    for (int k = 0; k < GR; ++k) {
      const int e = threadIdx.x + k * kBlock;
      const int n = e % NTV, j = e / NTV;
      const int co = n0 + VW * n;
      SV v = SV{};
      if (e < GN && p0 + j < p_end && co < a.cout) v = *(const SV*)(a.dy + ((size_t)p0 + j) * a.cout + co);
      gr[k] = v;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int k = 0; k < XR; ++k) {
      const int e = threadIdx.x + k * kBlock;
      if (e < XN) *(SV*)&xs[b][e / (18 * TMV)][(e / TMV) % 18][VW * (e % TMV)] = xr[k];
    }
#pragma unroll
    for (int k = 0; k < GR; ++k) {
      const int e = threadIdx.x + k * kBlock;
      if (e < GN) *(SV*)&gs[b][e / NTV][VW * (e % NTV)] = gr[k];
    }
  };

  v4f acc[9][G::FM][G::FN];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int j = 0; j < G::FN; ++j) acc[t][i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  if (p_begin < p_end) {
    fetch(p_begin);
    stash(0);
  }
  __syncthreads();
  int buf = 0;
  for (int p0 = p_begin; p0 < p_end; p0 += 16) {
    const bool more = p0 + 16 < p_end;   // uniform
    if (more) fetch(p0 + 16);
    if (active) {
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        float bv[G::FN];
#pragma unroll
        for (int j = 0; j < G::FN; ++j)
          bv[j] = gs[buf][kk + kq][(wn * G::FN + j) * 16 + (lane & 15)];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          float av[G::FM];
#pragma unroll
          for (int i = 0; i < G::FM; ++i)
            av[i] = xs[buf][t / 3][kk + kq + t % 3][(wm * G::FM + i) * 16 + (lane & 15)];
#pragma unroll
          for (int i = 0; i < G::FM; ++i)
#pragma unroll
            for (int j = 0; j < G::FN; ++j) acc[t][i][j] = mfma4(av[i], bv[j], acc[t][i][j]);
        }
      }
    }
    // the other buffer was last read before the previous barrier
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (!active) return;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    float* out = a.part + ((size_t)blockIdx.x * 9 + t) * a.cin * a.cout;
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int co = n0 + (wn * G::FN + j) * 16 + (lane & 15);
      if (co >= a.cout) continue;
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ci = m0 + (wm * G::FM + i) * 16 + 4 * kq + r;
          if (ci < a.cin) out[(size_t)ci * a.cout + co] = acc[t][i][j][r];
        }
    }
  }
}

// out[e] = sum over s < nsplit of part[s * n + e], s ascending.
__global__ __launch_bounds__(kBlock) void k_sum_splits(const float* __restrict__ part, int nsplit,
                                                       size_t n, float* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  // four accumulators (split k into k % 4), so that the loads overlap;
  // added in a fixed order, the result does not depend on the schedule
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  int k = 0;
  for (; k + 3 < nsplit; k += 4) {
    s0 += part[(size_t)k * n + e];
    s1 += part[(size_t)(k + 1) * n + e];
    s2 += part[(size_t)(k + 2) * n + e];
    s3 += part[(size_t)(k + 3) * n + e];
  }
  if (k < nsplit) s0 += part[(size_t)k * n + e];
  if (k + 1 < nsplit) s1 += part[(size_t)(k + 1) * n + e];
  if (k + 2 < nsplit) s2 += part[(size_t)(k + 2) * n + e];
  out[e] = (s0 + s1) + (s2 + s3);
}

// Column sums of g [npix][c] over pixel ranges of `sp` pixels into partial
// [split][c]; blockIdx.y selects 256 channels.  With cc < 256 channels in the
// block, thread t adds pixels t / cc, t / cc + groups, ... of channel t % cc,
// and the groups are then added in ascending order.
__global__ __launch_bounds__(kBlock) void k_colsum_part(const float* __restrict__ g, int npix, int c,
                                                        int sp, float* __restrict__ part) {
  __shared__ float s[kBlock];
  const int c0 = blockIdx.y * kBlock;
  const int cc = min(c - c0, kBlock);
  const int groups = kBlock / cc;
  const int t = threadIdx.x;
  const int grp = t / cc, ch = t % cc;
  const int p_begin = blockIdx.x * sp, p_end = min(p_begin + sp, npix);
  // eight accumulators (pixel step i into i % 8), so that the loads overlap;
  // added in a fixed order
  float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (grp < groups) {
    int p = p_begin + grp;
    for (; p + 7 * groups < p_end; p += 8 * groups) {
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] += g[(size_t)(p + u * groups) * c + c0 + ch];
    }
#pragma unroll
    for (int u = 0; u < 7; ++u)
      if (p + u * groups < p_end) v[u] += g[(size_t)(p + u * groups) * c + c0 + ch];
  }
  s[t] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  __syncthreads();
  if (t < cc) {
    float tot = 0.f;
    for (int k = 0; k < groups; ++k) tot += s[k * cc + t];
    part[(size_t)blockIdx.x * c + c0 + t] = tot;
  }
}

// w'[t][co][ci] = w[T - 1 - t][ci][co]: weights of the data-gradient convolution.
__global__ __launch_bounds__(kBlock) void k_flip_weights(const float* __restrict__ w, int T, int cin,
                                                         int cout, float* __restrict__ wt) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const size_t n = (size_t)T * cin * cout;
  if (e >= n) return;
  const int ci = (int)(e % cin);
  const int co = (int)((e / cin) % cout);
  const int t = (int)(e / ((size_t)cin * cout));
  wt[e] = w[((size_t)(T - 1 - t) * cin + ci) * cout + co];
}

// g = (y > 0) ? g : 0, in place.
__global__ __launch_bounds__(kBlock) void k_relu_bwd(const float* __restrict__ y, float* __restrict__ g,
                                                     size_t n) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n && !(y[e] > 0.f)) g[e] = 0.f;
}

// 2 x 2 max pooling: y[b][h][w][c] = max of x[b][2h + i][2w + j][c].
__global__ __launch_bounds__(kBlock) void k_pool_fwd(const float* __restrict__ x, float* __restrict__ y,
                                                     int Ho, int Wo, int C, size_t n) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e % C);
  const size_t pix = e / C;
  const int w = (int)(pix % Wo);
  const size_t bh = pix / Wo;   // b * Ho + h
  const size_t row0 = (bh * 2) * (size_t)(2 * Wo);
  const size_t i00 = (row0 + 2 * w) * C + c, i10 = i00 + (size_t)2 * Wo * C;
  float m = x[i00];
  const float v01 = x[i00 + C], v10 = x[i10], v11 = x[i10 + C];
  if (v01 > m) m = v01;
  if (v10 > m) m = v10;
  if (v11 > m) m = v11;
  y[e] = m;
}

// Gradient of 2 x 2 max pooling (to the first maximal element of each window in
// row-major order) plus an optional addend of the input's shape.
__global__ __launch_bounds__(kBlock) void k_pool_bwd(const float* __restrict__ x,
                                                     const float* __restrict__ gy,
                                                     const float* __restrict__ add,
                                                     float* __restrict__ gx, int Ho, int Wo, int C,
                                                     size_t n) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e % C);
  const size_t pix = e / C;
  const int w = (int)(pix % Wo);
  const size_t bh = pix / Wo;
  const size_t row0 = (bh * 2) * (size_t)(2 * Wo);
  const size_t idx[4] = {(row0 + 2 * w) * C + c, (row0 + 2 * w + 1) * C + c,
                         (row0 + 2 * Wo + 2 * w) * C + c, (row0 + 2 * Wo + 2 * w + 1) * C + c};
  float m = x[idx[0]];
  int arg = 0;
  for (int k = 1; k < 4; ++k) {
    const float v = x[idx[k]];
    if (v > m) {
      m = v;
      arg = k;
    }
  }
  const float g = gy[e];
  for (int k = 0; k < 4; ++k) {
    float v = k == arg ? g : 0.f;
    if (add) v += add[idx[k]];
    gx[idx[k]] = v;
  }
}

// cat[b][h][w][c] = c < C1 ? deep[b][h/2][w/2][c] : skip[b][h][w][c - C1]
__global__ __launch_bounds__(kBlock) void k_upcat_fwd(const float* __restrict__ deep,
                                                      const float* __restrict__ skip,
                                                      float* __restrict__ cat, int H, int W, int C1,
                                                      int C2, size_t n) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const int C = C1 + C2;
  const int c = (int)(e % C);
  const size_t pix = e / C;
  if (c >= C1) {
    cat[e] = skip[pix * C2 + (c - C1)];
    return;
  }
  const int w = (int)(pix % W);
  const size_t bh = pix / W;
  const int h = (int)(bh % H);
  const size_t b = bh / H;
  cat[e] = deep[((b * (H / 2) + h / 2) * (size_t)(W / 2) + w / 2) * C1 + c];
}

// Gradients of upsample-and-concatenate: gdeep (sum over each 2 x 2 block of the
// first C1 channels, in row-major order) for n1 elements, then gskip.
__global__ __launch_bounds__(kBlock) void k_upcat_bwd(const float* __restrict__ gcat,
                                                      float* __restrict__ gdeep,
                                                      float* __restrict__ gskip, int H, int W,
                                                      int C1, int C2, size_t n1, size_t n2) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const int C = C1 + C2;
  if (e < n1) {
    const int c = (int)(e % C1);
    const size_t pix = e / C1;   // pixel of the half-resolution image
    const int w = (int)(pix % (W / 2));
    const size_t bh = pix / (W / 2);   // b * (H / 2) + h
    const size_t r0 = bh * 2 * (size_t)W;
    const size_t i00 = (r0 + 2 * w) * C + c;
    const size_t i10 = i00 + (size_t)W * C;
    gdeep[e] = ((gcat[i00] + gcat[i00 + C]) + gcat[i10]) + gcat[i10 + C];
  } else if (e < n1 + n2) {
    const size_t k = e - n1;
    const int c = (int)(k % C2);
    const size_t pix = k / C2;
    gskip[k] = gcat[pix * C + C1 + c];
  }
}

// Masked squared error, pass 1: per block, the sum of (pred - target)^2 over the
// fluid pixels (solid[p] == 0) and all channels, and the number of fluid pixels.
__global__ __launch_bounds__(kBlock) void k_mse_part(const float* __restrict__ pred,
                                                     const float* __restrict__ tgt,
                                                     const uint8_t* __restrict__ solid, int npix,
                                                     int C, double* __restrict__ part) {
  __shared__ double s[kBlock], cnt[kBlock];
  const int p = blockIdx.x * kBlock + threadIdx.x;
  double v = 0.0, k = 0.0;
  if (p < npix && solid[p] == 0) {
    for (int c = 0; c < C; ++c) {
      const double d = (double)pred[(size_t)p * C + c] - (double)tgt[(size_t)p * C + c];
      v += d * d;
    }
    k = 1.0;
  }
  s[threadIdx.x] = v;
  cnt[threadIdx.x] = k;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s[threadIdx.x] += s[threadIdx.x + o];
      cnt[threadIdx.x] += cnt[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s[0];
    part[2 * blockIdx.x + 1] = cnt[0];
  }
}

// Pass 2 (one block): loss = sum / (C * count) -> out[0] (double), and
// scale = 2 / (C * count) -> out[1].
__global__ __launch_bounds__(kBlock) void k_mse_final(const double* __restrict__ part, int nb, int C,
                                                      double* __restrict__ out) {
  __shared__ double s[kBlock], cnt[kBlock];
  double v = 0.0, k = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    v += part[2 * i];
    k += part[2 * i + 1];
  }
  s[threadIdx.x] = v;
  cnt[threadIdx.x] = k;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s[threadIdx.x] += s[threadIdx.x + o];
      cnt[threadIdx.x] += cnt[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n = cnt[0] * C;
    out[0] = n > 0 ? s[0] / n : 0.0;
    out[1] = n > 0 ? 2.0 / n : 0.0;
  }
}

// Pass 3: grad = scale (pred - target) on fluid pixels, 0 on solid ones.
__global__ __launch_bounds__(kBlock) void k_mse_grad(const float* __restrict__ pred,
                                                     const float* __restrict__ tgt,
                                                     const uint8_t* __restrict__ solid,
                                                     const double* __restrict__ scale, int npix,
                                                     int C, float* __restrict__ grad) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (size_t)npix * C) return;
  const size_t p = e / C;
  grad[e] = solid[p] == 0 ? (float)(scale[1] * ((double)pred[e] - (double)tgt[e])) : 0.f;
}

// Adam (Kingma & Ba 2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m / bc1) / (sqrt(v / bc2) + eps), bc_k = 1 - b_k^t.  The factors
// 1 - b_k come from the host (rounding b2 = 0.999 to FP32 first and then
// subtracting would be off by 1.3e-5).
__global__ __launch_bounds__(kBlock) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                                 float* __restrict__ m, float* __restrict__ v, size_t n,
                                                 float lr, float b1, float b2, float omb1, float omb2,
                                                 float eps, float bc1, float bc2) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + omb1 * gg;
  const float vv = b2 * v[e] + omb2 * gg * gg;
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

// Network input from a batch of solid masks: x[b][p][0] = solid[b][p],
// x[b][p][1] = feat[b] (the sample's scaled Knudsen number).
__global__ __launch_bounds__(kBlock) void k_pack_input(const uint8_t* __restrict__ solid,
                                                       const float* __restrict__ feat, int hw,
                                                       size_t npix, float* __restrict__ x) {
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= npix) return;
  x[2 * p] = (float)solid[p];
  x[2 * p + 1] = feat[p / hw];
}

// Network input with a third channel: x[p][2] = scale * profile[b][column].
__global__ __launch_bounds__(kBlock) void k_pack_input_profile(const uint8_t* __restrict__ solid,
                                                               const float* __restrict__ feat,
                                                               const float* __restrict__ profile,
                                                               float scale, int hw, int width,
                                                               size_t npix, float* __restrict__ x) {
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= npix) return;
  const size_t b = p / hw;
  const int col = (int)(p % hw) % width;
  x[3 * p] = (float)solid[p];
  x[3 * p + 1] = feat[b];
  x[3 * p + 2] = scale * profile[b * width + col];
}

// Resistance profile along x of each sample's mask (one block per sample,
// `width` floats of dynamic LDS): the fluid fraction phi(x) of column x
// (at least 1/H), a Kozeny-Carman resistance R(x) = (1 - phi + 1/H)^2 / phi^3,
// its normalised running sum C(x) = sum_{x' <= x} R / sum R (summed in x
// order), and profile[b][x] = (x + 1)/(W + 1) - C(x): where a density drop
// concentrated in the resistive columns departs from the linear drop between
// the ghost planes, in units of the drop.
__global__ __launch_bounds__(kBlock) void k_column_profile(const uint8_t* __restrict__ solid,
                                                           int height, int width,
                                                           float* __restrict__ profile) {
  extern __shared__ float run[];
  const size_t b = blockIdx.x;
  const uint8_t* s = solid + b * (size_t)height * width;
  const float hmin = 1.0f / (float)height;
  for (int x = threadIdx.x; x < width; x += kBlock) {
    int fluid = 0;
    for (int h = 0; h < height; ++h) fluid += s[(size_t)h * width + x] == 0;
    const float phi = fmaxf((float)fluid * hmin, hmin);
    const float a = 1.0f - phi + hmin;
    run[x] = a * a / (phi * phi * phi);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float acc = 0.f;
    for (int x = 0; x < width; ++x) {
      acc += run[x];
      run[x] = acc;
    }
  }
  __syncthreads();
  const float total = run[width - 1];
  for (int x = threadIdx.x; x < width; x += kBlock)
    profile[b * width + x] = (float)(x + 1) / (float)(width + 1) - run[x] / total;
}

// Solver fields (rho [b][p], u [b][2][p]) -> NHWC [b][p][3]:
// y_k = (f_k - shift[3b + k] - slope[3b + k] (x + 1)) * scale[3b + k], with x
// the pixel's column (slope may be null: 0).  A slope along x lets the
// network see the density without its linear drop between the ghost planes,
// which no translation-invariant map could produce.
__global__ __launch_bounds__(kBlock) void k_fields_to_nhwc(const float* __restrict__ rho,
                                                           const float* __restrict__ u,
                                                           const float* __restrict__ shift,
                                                           const float* __restrict__ slope,
                                                           const float* __restrict__ scale, int hw,
                                                           int width, size_t npix,
                                                           float* __restrict__ y) {
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= npix) return;
  const size_t b = p / hw, q = p % hw;
  const float xp = (float)(q % width + 1);
  const float f[3] = {rho[p], u[(2 * b) * hw + q], u[(2 * b + 1) * hw + q]};
  for (int k = 0; k < 3; ++k) {
    const float base = shift[3 * b + k] + (slope ? slope[3 * b + k] * xp : 0.f);
    y[3 * p + k] = (f[k] - base) * scale[3 * b + k];
  }
}

// NHWC [b][p][3] -> solver fields: f_k = y_k * scale[3b + k] + shift[3b + k]
// + slope[3b + k] (x + 1); the velocity is zero where keep_u[p] == 0 (when
// keep_u is given).  A non-finite value anywhere in a sample's prediction is
// reported in bad[b].
__global__ __launch_bounds__(kBlock) void k_nhwc_to_fields(const float* __restrict__ y,
                                                           const float* __restrict__ shift,
                                                           const float* __restrict__ slope,
                                                           const float* __restrict__ scale,
                                                           const uint8_t* __restrict__ keep_u,
                                                           int hw, int width, size_t npix,
                                                           float* __restrict__ rho,
                                                           float* __restrict__ u,
                                                           int* __restrict__ bad) {
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= npix) return;
  const size_t b = p / hw, q = p % hw;
  const float xp = (float)(q % width + 1);
  float f[3];
  bool finite = true;
  for (int k = 0; k < 3; ++k) {
    const float base = shift[3 * b + k] + (slope ? slope[3 * b + k] * xp : 0.f);
    f[k] = y[3 * p + k] * scale[3 * b + k] + base;
    finite = finite && isfinite(f[k]);
  }
  if (keep_u && !keep_u[p]) f[1] = f[2] = 0.f;
  rho[p] = f[0];
  u[(2 * b) * hw + q] = f[1];
  u[(2 * b + 1) * hw + q] = f[2];
  if (!finite) bad[b] = 1;   // plain store of a flag; every writer stores the same value
}

// Per-channel factors of a mirror image (up to kMirrorC channels).
constexpr int kMirrorC = 8;
struct MirrorScale {
  float s[kMirrorC];
};

// Mirror image of NHWC images [b][h][w][c]: out pixel (b, h, w) is in pixel
// (b, fh ? H - 1 - h : h, fw ? W - 1 - w : w); with SCALE, channel k is
// multiplied by sc.s[k]; with ACC, the result is added to out.
template <class E, bool SCALE, bool ACC>
__global__ __launch_bounds__(kBlock) void k_mirror(const E* __restrict__ in, int height, int width,
                                                   int c, int fh, int fw, MirrorScale sc,
                                                   size_t npix, E* __restrict__ out) {
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= npix) return;
  const size_t hw = (size_t)height * width;
  const size_t b = p / hw;
  const int q = (int)(p - b * hw);
  const int h = q / width, w = q - h * width;
  const int hs = fh ? height - 1 - h : h, ws = fw ? width - 1 - w : w;
  const E* src = in + (b * hw + (size_t)hs * width + ws) * c;
  E* dst = out + p * c;
  for (int k = 0; k < c; ++k) {
    E v = src[k];
    if constexpr (SCALE) v = v * sc.s[k < kMirrorC ? k : 0];
    if constexpr (ACC) v = dst[k] + v;
    dst[k] = v;
  }
}

}  // namespace wsn
