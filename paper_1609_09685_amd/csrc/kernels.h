// Device kernels of the lattice Boltzmann permeability solver (gfx950).
//
// One fused, pull-scheme kernel does a whole time step: for every fluid node it
// gathers the Q populations that arrive from its neighbours (applying the
// boundary rules), forms density and momentum, relaxes towards the
// equilibrium (BGK with the normalised relaxation time tau), and writes the Q
// post-collision populations to the other buffer.  The step is bound by HBM
// bandwidth (about 1.3 flop per byte for D3Q19 in FP32): the design goal is to
// move each fluid population once in and once out per step, and nothing else.
//
// Compact fluid-only storage.  Porous media at the voxel scale mix solid and
// fluid inside almost every 128-byte line, so a dense array would drag the
// solid slots through HBM with the fluid ones.  Populations are therefore kept
// for fluid nodes only, numbered in x-fastest (x, y, z) order:
//     g[i][k],  i = direction, k = compact fluid index,
// as deviations from the rest state, g_i = f_i - w_i rho0.  Each direction's
// array is padded to 64 entries.
//
// The pull source of a node is found from a bitmap of the mask: for every
// (y, z) row, 64-bit words with bit x%64 set for fluid nodes (one guard word
// of zeros before and after each row) and, per word, the compact index of its
// first fluid node.  The compact index of a fluid node x in a row is then
// pfx[word] + popcount(bits[word] below x).  A wavefront covers 64 aligned x of
// one row, so every bitmap word it needs is uniform across its lanes (scalar
// loads, ~16 MB for 512^3, cache resident), and the stores of its fluid lanes
// go to one contiguous range of each direction's array.
//
// Boundary rules, in the order they apply to the source x - c_i of direction i
// at a fluid node x:
//   1. symmetric planes: a source row outside [0, ny) (or [0, nz)) is the
//      node's own row, and the direction read is the mirrored one (my / mz);
//   2. solid source: halfway bounce-back, g*_opp(i)(x);
//   3. source on a ghost plane (x - c_x = -1 or nx): the value at the edge
//      node b = (x, y_s, z_s) in the (mirrored) direction k plus the
//      non-equilibrium-extrapolation term w_i (rho_set - rho_b) P_k(u_b),
//      where P_k(u) = 1 + 3 c_k.u + 9/2 (c_k.u)^2 - 3/2 u.u and rho_b, u_b are
//      the edge node's moments of its stored populations of the previous step
//      (kept in a double-buffered boundary-plane array); a ghost copies the
//      solidity of b;
//   4. otherwise plain streaming, g*_i(x - c_i).
// Collision in deviation form: drho = sum g, j = sum c g, rho = rho0 + drho,
// u = j / rho, g_eq_i = w_i [drho + rho (3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u)],
// g* = g - (g - g_eq)/tau.  The linear ("Stokes") equilibrium drops the two
// quadratic terms (the paper's remedy for inertia in its 3D case).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lattice.h"

namespace lbm {

constexpr int kWave = 64;    // lanes per wavefront = x per bitmap word
constexpr int kRows = 4;     // (y) rows per block: 256 threads
constexpr int kThreads = kWave * kRows;

template <int I, int N, class F>
__device__ __forceinline__ void unroll(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    unroll<I + 1, N>(f);
  }
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Bitmap of the fluid nodes.  bits: [nz][ny][nw + 2] words, word w + 1 holds
// x in [64 w, 64 w + 64), words 0 and nw + 1 are zero guards.  pfx: [nz][ny][nw],
// compact index of the first fluid node at or after x = 64 w of that row.
struct FluidMap {
  const uint64_t* __restrict__ bits;
  const uint32_t* __restrict__ pfx;
  int nx, ny, nz, nw;

  __device__ __forceinline__ size_t row(int y, int z) const { return (size_t)z * ny + y; }
  __device__ __forceinline__ const uint64_t* words(int y, int z) const {
    return bits + row(y, z) * (size_t)(nw + 2) + 1;
  }
  // compact index of node x (valid when the node is fluid), and its fluid bit
  __device__ __forceinline__ uint32_t rank(int x, int y, int z, bool& fluid) const {
    const int w = x >> 6, p = x & 63;
    const uint64_t m = words(y, z)[w];
    fluid = (m >> p) & 1ull;
    return pfx[row(y, z) * nw + w] + (uint32_t)__popcll(m & ((1ull << p) - 1ull));
  }
};

// Arguments of one domain's step.
template <class T>
struct StepArgs {
  const T* __restrict__ src;       // populations of step t
  T* __restrict__ dst;             // populations of step t+1
  FluidMap fm;
  const T* __restrict__ bp_src;    // edge-node moments of step t: [2 sides][D+1][nz*ny]
  T* __restrict__ bp_dst;          // edge-node moments written by this step
  double* __restrict__ partial;    // per-block flux partials (flux variant)
  uint64_t ps;                     // elements between two direction arrays
  int tiles_y;                     // ceil(ny / kRows)
  int blocks;                      // nw * tiles_y * nz
  int xcd_remap;                   // 1: consecutive tiles on the same XCD
  T omega, rho0, drho_in, drho_out;  // 1/tau; rho0; rho_in - rho0; rho_out - rho0
};

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of v over the block in a fixed order; thread 0 stores it.  Every thread
// of the block must call it.
template <int NT>
__device__ __forceinline__ void block_sum_store(double v, double* out) {
  __shared__ double s[NT / 64];
  v = wave_sum(v);
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  if ((tid & 63) == 0) s[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += s[i];
    *out = t;
  }
}

// Deterministic second pass: one block sums n partials, out = scale * sum.
__global__ __launch_bounds__(1024) void k_reduce(const double* __restrict__ partial, int n,
                                                 double scale, double* __restrict__ out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) v += partial[i];
  __shared__ double s[16];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += s[i];
    out[0] = scale * t;
  }
}

// -------------------------------------------------------------- equilibrium

template <class L, int q, class T>
__device__ __forceinline__ T dot_c(T ux, T uy, T uz) {
  T cu = T(0);
  if constexpr (L::cx[q] == 1) cu += ux;
  if constexpr (L::cx[q] == -1) cu -= ux;
  if constexpr (L::cy[q] == 1) cu += uy;
  if constexpr (L::cy[q] == -1) cu -= uy;
  if constexpr (L::cz[q] == 1) cu += uz;
  if constexpr (L::cz[q] == -1) cu -= uz;
  return cu;
}

// g_eq_i as a deviation from w_i rho0 (usq15 = 3/2 u.u).
template <class L, int q, bool LINEAR, class T>
__device__ __forceinline__ T geq(T drho, T rho, T ux, T uy, T uz, T usq15) {
  const T cu = dot_c<L, q>(ux, uy, uz);
  if constexpr (LINEAR) return T(L::w[q]) * (drho + rho * (T(3) * cu));
  return T(L::w[q]) * (drho + rho * (T(3) * cu + T(4.5) * cu * cu - usq15));
}

// Density deviation and velocity of one node's stored (post-collision)
// populations.  The step kernel applies it to the values it stores at the edge
// planes, and the restore path to the values it loads, so both produce the
// same bits.
template <class L, class T, class Get>
__device__ __forceinline__ void stored_moments(Get get, T rho0, T& drho, T& ux, T& uy, T& uz) {
  T d = T(0), jx = T(0), jy = T(0), jz = T(0);
  unroll<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const T v = get(qc);
    d += v;
    if constexpr (L::cx[q] == 1) jx += v;
    if constexpr (L::cx[q] == -1) jx -= v;
    if constexpr (L::cy[q] == 1) jy += v;
    if constexpr (L::cy[q] == -1) jy -= v;
    if constexpr (L::cz[q] == 1) jz += v;
    if constexpr (L::cz[q] == -1) jz -= v;
  });
  const T inv = T(1) / (rho0 + d);
  drho = d;
  ux = jx * inv;
  uy = jy * inv;
  uz = jz * inv;
}

// --------------------------------------------------------------- time step

// Non-equilibrium extrapolation term of a ghost population (rule 3).
template <class L, bool LINEAR, class T>
__device__ __noinline__ T ghost_term(const T* __restrict__ bp, int side, uint32_t plane,
                                     uint32_t at, T drho_set, T wq, int cxk, int cyk, int czk) {
  const T* p = bp + (size_t)side * (L::D + 1) * plane + at;
  const T drb = p[0];
  const T ux = p[plane], uy = p[2 * plane];
  const T uz = L::D == 3 ? p[3 * plane] : T(0);
  const T cu = T(cxk) * ux + T(cyk) * uy + T(czk) * uz;
  T P = T(1) + T(3) * cu;
  if constexpr (!LINEAR) P += T(4.5) * cu * cu - T(1.5) * (ux * ux + uy * uy + uz * uz);
  return wq * (drho_set - drb) * P;
}

// The bitmap of one source row around the wave's word, reduced to what a lane
// needs: its rank in the row (r0 = fluid nodes of the row before x) and the
// fluid bits of x-1, x, x+1 in that row.
struct RowView {
  uint32_t r0;
  uint32_t fm, f0, fp;   // fluid(x-1), fluid(x), fluid(x+1)
};

__device__ __forceinline__ RowView row_view(const FluidMap& fm, int y, int z, int w, int p) {
  const uint64_t* wd = fm.words(y, z) + w;   // uniform address: scalar loads
  const uint64_t lo = wd[-1], mid = wd[0], hi = wd[1];
  const uint32_t base = fm.pfx[fm.row(y, z) * fm.nw + w];
  const uint64_t below = (1ull << p) - 1ull;
  const uint64_t sh_lo = (mid << 1) | (lo >> 63);   // bit p = fluid(x-1)
  const uint64_t sh_hi = (mid >> 1) | (hi << 63);   // bit p = fluid(x+1)
  RowView r;
  r.r0 = base + (uint32_t)__popcll(mid & below);
  r.f0 = (uint32_t)(mid >> p) & 1u;
  r.fm = (uint32_t)(sh_lo >> p) & 1u;
  r.fp = (uint32_t)(sh_hi >> p) & 1u;
  return r;
}

// Updates one node of a wave covering x = 64 w + p of row (y, z) (y, z, w
// uniform across the wave).  Returns the node's x-momentum (0 if not fluid).
template <class L, class T, bool LINEAR>
__device__ __forceinline__ T node_update(const StepArgs<T>& a, int y, int z, int w, int p) {
  const FluidMap& fm = a.fm;
  const int x = (w << 6) + p;
  // mirror planes act on whole rows: the row choice is uniform per wave
  const bool y0 = y == 0, y1 = y == fm.ny - 1;
  const bool z0 = z == 0, z1 = z == fm.nz - 1;
  RowView rv[3][3];   // [dz + 1][dy + 1]: source row (y + dy, z + dz), mirrored
  unroll<0, 3>([&](auto izc) {
    constexpr int dz = decltype(izc)::value - 1;
    if constexpr (L::D == 3 || dz == 0) {
      unroll<0, 3>([&](auto iyc) {
        constexpr int dy = decltype(iyc)::value - 1;
        const int yy = (dy < 0 && y0) || (dy > 0 && y1) ? y : y + dy;
        const int zz = (dz < 0 && z0) || (dz > 0 && z1) ? z : z + dz;
        rv[dz + 1][dy + 1] = row_view(fm, yy, zz, w, p);
      });
    }
  });
  const RowView& me = rv[1][1];
  if (!me.f0) return T(0);   // solid node, or x >= nx
  const uint32_t self = me.r0;
  const bool x0 = x == 0, x1 = x == fm.nx - 1;

  T g[L::Q];
  unroll<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int cx = L::cx[q], cy = L::cy[q], cz = L::cz[q];
    if constexpr (q == 0) {
      g[0] = a.src[self];
    } else {
      bool fy = false, fz = false, gh = false;
      if constexpr (cy > 0) fy = y0;
      if constexpr (cy < 0) fy = y1;
      if constexpr (cz > 0) fz = z0;
      if constexpr (cz < 0) fz = z1;
      if constexpr (cx > 0) gh = x0;
      if constexpr (cx < 0) gh = x1;
      constexpr int kY = L::my[q], kZ = L::mz[q], kYZ = L::mz[L::my[q]];
      const int k = fy ? (fz ? kYZ : kY) : (fz ? kZ : q);
      const RowView& r = rv[1 - cz][1 - cy];
      uint32_t sf, si;   // source fluid?, source compact index
      if constexpr (cx == 0) {
        sf = r.f0;
        si = r.r0;
      } else if constexpr (cx > 0) {
        sf = gh ? r.f0 : r.fm;
        si = gh ? r.r0 : r.r0 - r.fm;
      } else {
        sf = gh ? r.f0 : r.fp;
        si = gh ? r.r0 : r.r0 + r.f0;
      }
      const T* ptr = sf ? a.src + (uint64_t)k * a.ps + si
                        : a.src + (uint64_t)L::opp[q] * a.ps + self;   // bounce-back
      T v = *ptr;
      if constexpr (cx != 0) {
        if (gh && sf) {
          const int ys = fy ? y : y - cy, zs = fz ? z : z - cz;
          v += ghost_term<L, LINEAR, T>(a.bp_src, cx > 0 ? 0 : 1, (uint32_t)fm.nz * fm.ny,
                                        (uint32_t)zs * fm.ny + ys, cx > 0 ? a.drho_in : a.drho_out,
                                        T(L::w[q]), cx, fy ? -cy : cy, fz ? -cz : cz);
        }
      }
      g[q] = v;
    }
  });

  T drho = T(0), jx = T(0), jy = T(0), jz = T(0);
  unroll<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    drho += g[q];
    if constexpr (L::cx[q] == 1) jx += g[q];
    if constexpr (L::cx[q] == -1) jx -= g[q];
    if constexpr (L::cy[q] == 1) jy += g[q];
    if constexpr (L::cy[q] == -1) jy -= g[q];
    if constexpr (L::cz[q] == 1) jz += g[q];
    if constexpr (L::cz[q] == -1) jz -= g[q];
  });
  const T rho = a.rho0 + drho;
  const T inv = T(1) / rho;
  const T ux = jx * inv, uy = jy * inv, uz = jz * inv;
  const T usq15 = T(1.5) * (ux * ux + uy * uy + uz * uz);
  unroll<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const T ge = geq<L, q, LINEAR>(drho, rho, ux, uy, uz, usq15);
    g[q] = g[q] - a.omega * (g[q] - ge);
    a.dst[(uint64_t)q * a.ps + self] = g[q];
  });

  if (x0 || x1) {
    // edge-node moments of the stored state, read by the next step's ghosts
    T bd, bx, by, bz;
    stored_moments<L, T>([&](auto qc) { return g[decltype(qc)::value]; }, a.rho0, bd, bx, by, bz);
    const uint32_t plane = (uint32_t)fm.nz * fm.ny;
    T* bp = a.bp_dst + (size_t)(x0 ? 0 : 1) * (L::D + 1) * plane + (uint32_t)z * fm.ny + y;
    bp[0] = bd;
    bp[plane] = bx;
    bp[2 * plane] = by;
    if constexpr (L::D == 3) bp[3 * plane] = bz;
  }
  return jx;
}

// Tile of logical block b: word w (64 x), rows y0..y0+3, plane z.  With
// xcd_remap the hardware block id, which the dispatcher deals round-robin over
// the 8 XCDs, is mapped so that each XCD gets one contiguous range of tiles:
// neighbouring tiles then share that XCD's L2 for the lines at their edges.
__device__ __forceinline__ int logical_block(int hw, int blocks, int remap) {
  if (!remap) return hw;
  const int per = (blocks + 7) >> 3;
  return (hw & 7) * per + (hw >> 3);
}

// One time step of one domain.  FLUX: also store the block's summed
// x-momentum (FP64) in partial[b].
template <class L, class T, bool FLUX, bool LINEAR>
__global__ __launch_bounds__(kThreads) void k_step(StepArgs<T> a) {
  const int b = logical_block(blockIdx.x, a.blocks, a.xcd_remap);
  if (b >= a.blocks) return;   // whole block: padding of the remapped grid
  const int w = b % a.fm.nw;
  const int r = b / a.fm.nw;
  const int z = r / a.tiles_y;
  const int y = uniform((r % a.tiles_y) * kRows + (int)threadIdx.y);
  T jx = T(0);
  if (y < a.fm.ny) jx = node_update<L, T, LINEAR>(a, y, uniform(z), uniform(w), threadIdx.x);
  if constexpr (FLUX) block_sum_store<kThreads>((double)jx, a.partial + b);
}

// ------------------------------------------------------------ set-up kernels

// Bitmap words and per-word fluid counts from the solid mask (uint8
// [nz][ny][nx], 1 = solid).  One wave per word: the lanes ballot their nodes.
// Also writes the two guard words of each row.
__global__ __launch_bounds__(256) void k_pack_bits(const uint8_t* __restrict__ mask,
                                                   uint64_t* __restrict__ bits,
                                                   uint32_t* __restrict__ count, int nx, int ny,
                                                   int nz, int nw) {
  const uint64_t wave = ((uint64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const uint64_t nwords = (uint64_t)nz * ny * nw;
  if (wave >= nwords) return;   // uniform per wave
  const int w = (int)(wave % nw);
  const uint64_t row = wave / nw;
  const int x = w * 64 + lane;
  const bool fluid = x < nx && mask[row * nx + x] == 0;
  const uint64_t word = __ballot(fluid);
  if (lane == 0) {
    uint64_t* rw = bits + row * (uint64_t)(nw + 2);
    rw[w + 1] = word;
    if (w == 0) rw[0] = 0;
    if (w == nw - 1) rw[nw + 1] = 0;
    count[wave] = (uint32_t)__popcll(word);
  }
}

// Exclusive scan of n uint32 counts in three passes (block scan, scan of the
// block totals by one block, add back).  Integer and deterministic.
constexpr int kScanBlock = 1024;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t s[kScanBlock];
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const uint32_t add = t >= off ? s[t - off] : 0u;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  const uint32_t incl = s[t];
  if (total) *total = s[kScanBlock - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_local(const uint32_t* __restrict__ in,
                                                           uint32_t* __restrict__ out,
                                                           uint32_t* __restrict__ block_tot,
                                                           uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x;
  const uint32_t v = i < n ? in[i] : 0u;
  uint32_t tot;
  const uint32_t ex = block_exclusive_scan(v, &tot);
  if (i < n) out[i] = ex;
  if (threadIdx.x == 0) block_tot[blockIdx.x] = tot;
}

// One block: exclusive scan of nb block totals in place; grand total -> *sum.
__global__ __launch_bounds__(kScanBlock) void k_scan_totals(uint32_t* __restrict__ tot, int nb,
                                                            uint64_t* __restrict__ sum) {
  uint64_t carry = 0;
  for (int base = 0; base < nb; base += kScanBlock) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < nb ? tot[i] : 0u;
    uint32_t chunk;
    const uint32_t ex = block_exclusive_scan(v, &chunk);
    if (i < nb) tot[i] = (uint32_t)(carry + ex);
    carry += chunk;
  }
  if (threadIdx.x == 0) *sum = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(uint32_t* __restrict__ out,
                                                         const uint32_t* __restrict__ block_tot,
                                                         uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) out[i] += block_tot[blockIdx.x];
}

// Rest state: g_i = w_i (rho(x) - rho0), rho uniform (mode 0) or linear in x
// between the ghost planes (mode 1), into f and, if not null, f_other.
template <class L, class T>
__global__ __launch_bounds__(256) void k_init_rest(T* __restrict__ f, T* __restrict__ f_other,
                                                   FluidMap fm, uint64_t ps, int mode,
                                                   double rho_in, double rho_out, double rho0) {
  const uint64_t m = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= (uint64_t)fm.nx * fm.ny * fm.nz) return;
  const int x = (int)(m % fm.nx);
  const uint64_t r = m / fm.nx;
  bool fluid;
  const uint32_t k = fm.rank(x, (int)(r % fm.ny), (int)(r / fm.ny), fluid);
  if (!fluid) return;
  const double rho = mode == 1 ? rho_in + (rho_out - rho_in) * (double)(x + 1) / (double)(fm.nx + 1)
                               : 0.5 * (rho_in + rho_out);
  const double d = rho - rho0;
  unroll<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    f[(uint64_t)q * ps + k] = (T)(L::w[q] * d);
    if (f_other) f_other[(uint64_t)q * ps + k] = (T)(L::w[q] * d);
  });
}

// Equilibrium of given fields: rho [nz][ny][nx], u [D][nz][ny][nx] (float32).
template <class L, class T>
__global__ __launch_bounds__(256) void k_init_fields(T* __restrict__ f, FluidMap fm,
                                                     const float* __restrict__ rho_f,
                                                     const float* __restrict__ u_f, uint64_t ps,
                                                     double rho0) {
  const uint64_t N = (uint64_t)fm.nx * fm.ny * fm.nz;
  const uint64_t m = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= N) return;
  const int x = (int)(m % fm.nx);
  const uint64_t r = m / fm.nx;
  bool fluid;
  const uint32_t k = fm.rank(x, (int)(r % fm.ny), (int)(r / fm.ny), fluid);
  if (!fluid) return;
  const double rho = rho_f[m], ux = u_f[m], uy = u_f[N + m];
  const double uz = L::D == 3 ? (double)u_f[2 * N + m] : 0.0;
  const double usq15 = 1.5 * (ux * ux + uy * uy + uz * uz);
  const double drho = rho - rho0;
  unroll<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    f[(uint64_t)q * ps + k] = (T)geq<L, q, false, double>(drho, rho, ux, uy, uz, usq15);
  });
}

// Edge-node moments of the current state (after init or a restore).
template <class L, class T>
__global__ __launch_bounds__(256) void k_bplane(const T* __restrict__ f, FluidMap fm,
                                                T* __restrict__ bp, uint64_t ps, T rho0) {
  const uint32_t plane = (uint32_t)fm.nz * fm.ny;
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  if (t >= 2 * plane) return;
  const int side = t / plane;
  const uint32_t yz = t % plane;
  bool fluid;
  const uint32_t k = fm.rank(side == 0 ? 0 : fm.nx - 1, (int)(yz % fm.ny), (int)(yz / fm.ny), fluid);
  T d = 0, ux = 0, uy = 0, uz = 0;
  if (fluid)
    stored_moments<L, T>([&](auto qc) { return f[(uint64_t)decltype(qc)::value * ps + k]; }, rho0,
                         d, ux, uy, uz);
  T* p = bp + (size_t)side * (L::D + 1) * plane + yz;
  p[0] = d;
  p[plane] = ux;
  p[2 * plane] = uy;
  if constexpr (L::D == 3) p[3 * plane] = uz;
}

// Macroscopic fields (dense): rho and u [D][nz][ny][nx]; solids rho0 and 0.
template <class L, class T, class O>
__global__ __launch_bounds__(256) void k_macro(const T* __restrict__ f, FluidMap fm,
                                               O* __restrict__ rho, O* __restrict__ u, uint64_t ps,
                                               T rho0) {
  const uint64_t N = (uint64_t)fm.nx * fm.ny * fm.nz;
  const uint64_t m = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= N) return;
  const int x = (int)(m % fm.nx);
  const uint64_t r = m / fm.nx;
  bool fluid;
  const uint32_t k = fm.rank(x, (int)(r % fm.ny), (int)(r / fm.ny), fluid);
  T d = 0, ux = 0, uy = 0, uz = 0;
  if (fluid)
    stored_moments<L, T>([&](auto qc) { return f[(uint64_t)decltype(qc)::value * ps + k]; }, rho0,
                         d, ux, uy, uz);
  rho[m] = (O)((double)rho0 + (double)d);
  u[m] = (O)ux;
  u[N + m] = (O)uy;
  if constexpr (L::D == 3) u[2 * N + m] = (O)uz;
}

// x-momentum of the stored populations, summed per block of 256 compact nodes.
template <class L, class T>
__global__ __launch_bounds__(256) void k_flux(const T* __restrict__ f, uint64_t n_fluid,
                                              uint64_t ps, double* __restrict__ partial) {
  const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  T jx = T(0);
  if (k < n_fluid) {
    unroll<L::xp_begin, L::xp_end>([&](auto qc) { jx += f[(uint64_t)decltype(qc)::value * ps + k]; });
    unroll<L::xm_begin, L::xm_end>([&](auto qc) { jx -= f[(uint64_t)decltype(qc)::value * ps + k]; });
  }
  block_sum_store<256>((double)jx, partial + blockIdx.x);
}

}  // namespace lbm
