// Device kernels of the lattice Boltzmann permeability solver (gfx950).
//
// One fused, pull-scheme kernel does a whole time step: for every fluid node it
// gathers the Q populations that arrive from its neighbours (applying the
// boundary rules), forms density and momentum, relaxes towards the
// equilibrium (BGK with the normalised relaxation time tau), and writes the Q
// post-collision populations to the other buffer.  The step is bound by HBM
// bandwidth (about 1.3 flop per byte for D3Q19 in FP32), so there is no matrix
// core work here: the design goal is one coalesced read and one coalesced write
// of every population per step and nothing else.
//
// Storage: deviations from the rest state, g_i = f_i - w_i rho0, population-
// major: g[i][z][y][x] with the x pitch `xp` padded to 128 bytes.  Lanes of a
// wavefront cover 64 consecutive x of one (y, z) row, so every population load
// and store of a wave is one contiguous 256-byte (FP32) or 512-byte (FP64)
// segment, shifted by at most one element for directions with c_x != 0.
//
// Per-node link word (built once from the solid mask): bit i set when the
// source node of direction i (after the mirror planes, with ghosts copying the
// edge column) is solid, so the value comes from halfway bounce-back; bit 31
// set for solid nodes and x-padding, which are skipped.  One 4-byte load
// replaces Q-1 neighbour mask lookups.
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
//      the edge node's moments of the previous step (stored by that step in a
//      double-buffered boundary-plane array);
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

constexpr uint32_t kSolidBit = 1u << 31;
constexpr int kTileX = 64;   // one wavefront along x
constexpr int kTileY = 4;    // rows per block: 256 threads
constexpr int kThreads = kTileX * kTileY;

template <int I, int N, class F>
__device__ __forceinline__ void unroll(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    unroll<I + 1, N>(f);
  }
}

// Arguments of one domain's step.  Offsets of nodes inside one population
// array are 32-bit (the host checks nz*ny*xp*sizeof(T) < 2^32); the offset of
// a population array is 64-bit.
template <class T>
struct StepArgs {
  const T* __restrict__ src;       // populations of step t
  T* __restrict__ dst;             // populations of step t+1
  const uint32_t* __restrict__ links;
  const T* __restrict__ bp_src;    // edge-node moments of step t: [2 sides][D+1][nz*ny]
  T* __restrict__ bp_dst;          // edge-node moments written by this step
  double* __restrict__ partial;    // per-block flux partials (flux variant)
  uint64_t ps;                     // elements between two population arrays
  int nx, ny, nz, xp;
  int tiles_x, tiles_y;
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
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ partial, int n,
                                                double scale, double* __restrict__ out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += partial[i];
  __shared__ double s[4];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = scale * (((s[0] + s[1]) + s[2]) + s[3]);
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

// Updates one node; returns its x-momentum (0 for solids).
template <class L, class T, bool LINEAR>
__device__ __forceinline__ T node_update(const StepArgs<T>& a, int x, int y, int z) {
  const uint32_t n = ((uint32_t)z * (uint32_t)a.ny + (uint32_t)y) * (uint32_t)a.xp + (uint32_t)x;
  const uint32_t lk = a.links[n];
  if (lk & kSolidBit) return T(0);
  const bool y0 = y == 0, y1 = y == a.ny - 1;
  const bool z0 = z == 0, z1 = z == a.nz - 1;
  const bool x0 = x == 0, x1 = x == a.nx - 1;

  T g[L::Q];
  unroll<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int cx = L::cx[q], cy = L::cy[q], cz = L::cz[q];
    if constexpr (q == 0) {
      g[0] = a.src[n];
    } else {
      bool fy = false, fz = false, gh = false;
      if constexpr (cy > 0) fy = y0;
      if constexpr (cy < 0) fy = y1;
      if constexpr (cz > 0) fz = z0;
      if constexpr (cz < 0) fz = z1;
      if constexpr (cx > 0) gh = x0;
      if constexpr (cx < 0) gh = x1;
      const int ys = fy ? y : y - cy;
      const int zs = fz ? z : z - cz;
      const int xs = gh ? x : x - cx;
      constexpr int kY = L::my[q], kZ = L::mz[q], kYZ = L::mz[L::my[q]];
      const int k = fy ? (fz ? kYZ : kY) : (fz ? kZ : q);
      const bool bb = (lk >> q) & 1u;
      const uint32_t sn = ((uint32_t)zs * (uint32_t)a.ny + (uint32_t)ys) * (uint32_t)a.xp + (uint32_t)xs;
      const T* p = bb ? a.src + (uint64_t)L::opp[q] * a.ps + n : a.src + (uint64_t)k * a.ps + sn;
      T v = *p;
      if constexpr (cx != 0) {
        if (gh && !bb) {
          v += ghost_term<L, LINEAR, T>(a.bp_src, cx > 0 ? 0 : 1, (uint32_t)a.nz * a.ny,
                                        (uint32_t)zs * a.ny + ys, cx > 0 ? a.drho_in : a.drho_out,
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
    a.dst[(uint64_t)q * a.ps + n] = g[q];
  });

  if (x0 || x1) {
    // edge-node moments of the stored state, read by the next step's ghosts
    T bd, bx, by, bz;
    stored_moments<L, T>([&](auto qc) { return g[decltype(qc)::value]; }, a.rho0, bd, bx, by, bz);
    const uint32_t plane = (uint32_t)a.nz * a.ny;
    T* p = a.bp_dst + (size_t)(x0 ? 0 : 1) * (L::D + 1) * plane + (uint32_t)z * a.ny + y;
    p[0] = bd;
    p[plane] = bx;
    p[2 * plane] = by;
    if constexpr (L::D == 3) p[3 * plane] = bz;
  }
  return jx;
}

// One time step of one domain.  Block = 64 (x) by 4 (y) threads; block b
// covers the tile (b % tiles_x, (b / tiles_x) % tiles_y, b / (tiles_x tiles_y)).
// FLUX: also store the block's summed x-momentum (FP64) in partial[b].
template <class L, class T, bool FLUX, bool LINEAR>
__global__ __launch_bounds__(kThreads) void k_step(StepArgs<T> a) {
  const int b = blockIdx.x;
  const int tx = b % a.tiles_x;
  const int r = b / a.tiles_x;
  const int ty = r % a.tiles_y;
  const int z = r / a.tiles_y;
  const int x = tx * kTileX + threadIdx.x;
  const int y = ty * kTileY + threadIdx.y;
  T jx = T(0);
  if (x < a.nx && y < a.ny) jx = node_update<L, T, LINEAR>(a, x, y, z);
  if constexpr (FLUX) block_sum_store<kThreads>((double)jx, a.partial + b);
}

// ------------------------------------------------------------ set-up kernels

// Link words from the solid mask (uint8 [nz][ny][nx], 1 = solid).
template <class L>
__global__ __launch_bounds__(256) void k_links(const uint8_t* __restrict__ mask,
                                               uint32_t* __restrict__ links, int nx, int ny,
                                               int nz, int xp) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t total = (uint64_t)nz * ny * xp;
  if (i >= total) return;
  const int x = (int)(i % xp);
  const uint64_t r = i / xp;
  const int y = (int)(r % ny), z = (int)(r / ny);
  auto solid = [&](int xx, int yy, int zz) {
    return mask[((uint64_t)zz * ny + yy) * nx + xx] != 0;
  };
  if (x >= nx || solid(x, y, z)) {
    links[i] = kSolidBit;
    return;
  }
  uint32_t bits = 0;
  unroll<1, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    int xs = x - L::cx[q], ys = y - L::cy[q], zs = z - L::cz[q];
    ys = ys < 0 ? 0 : (ys >= ny ? ny - 1 : ys);   // mirror: the node's own row
    zs = zs < 0 ? 0 : (zs >= nz ? nz - 1 : zs);
    xs = xs < 0 ? 0 : (xs >= nx ? nx - 1 : xs);   // ghost copies the edge column
    if (solid(xs, ys, zs)) bits |= 1u << q;
  });
  links[i] = bits;
}

// Rest state: g_i = w_i (rho(x) - rho0), rho uniform (mode 0) or linear in x
// between the ghost planes (mode 1).  Solids and padding get 0.  f_other, if
// not null, gets the same values (so both buffers hold defined values).
template <class L, class T>
__global__ __launch_bounds__(256) void k_init_rest(T* __restrict__ f, T* __restrict__ f_other,
                                                   const uint32_t* __restrict__ links,
                                                   uint64_t ps, int nx, int ny, int nz, int xp,
                                                   int mode, double rho_in, double rho_out,
                                                   double rho0) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (uint64_t)nz * ny * xp) return;
  const int x = (int)(i % xp);
  const bool fluid = !(links[i] & kSolidBit);
  const double rho = mode == 1 ? rho_in + (rho_out - rho_in) * (double)(x + 1) / (double)(nx + 1)
                               : 0.5 * (rho_in + rho_out);
  const double d = fluid ? rho - rho0 : 0.0;
  unroll<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    f[(uint64_t)q * ps + i] = (T)(L::w[q] * d);
    if (f_other) f_other[(uint64_t)q * ps + i] = (T)(L::w[q] * d);
  });
}

// Equilibrium of given fields: rho [nz][ny][nx], u [D][nz][ny][nx] (float32).
template <class L, class T>
__global__ __launch_bounds__(256) void k_init_fields(T* __restrict__ f, const uint32_t* __restrict__ links,
                                                     const float* __restrict__ rho_f,
                                                     const float* __restrict__ u_f, uint64_t ps,
                                                     int nx, int ny, int nz, int xp, double rho0) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (uint64_t)nz * ny * xp) return;
  const int x = (int)(i % xp);
  const uint64_t r = i / xp;
  const uint64_t N = (uint64_t)nx * ny * nz;
  const bool fluid = !(links[i] & kSolidBit);
  double rho = rho0, ux = 0, uy = 0, uz = 0;
  if (fluid) {
    const uint64_t m = r * nx + x;
    rho = rho_f[m];
    ux = u_f[m];
    uy = u_f[N + m];
    if constexpr (L::D == 3) uz = u_f[2 * N + m];
  }
  const double usq15 = 1.5 * (ux * ux + uy * uy + uz * uz);
  const double drho = rho - rho0;
  unroll<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const double v = geq<L, q, false, double>(drho, rho, ux, uy, uz, usq15);
    f[(uint64_t)q * ps + i] = fluid ? (T)v : T(0);
  });
}

// Moments of one node from its stored populations.
template <class L, class T>
__device__ __forceinline__ void node_moments(const T* __restrict__ f, uint64_t ps, uint64_t i,
                                             T rho0, T& drho, T& ux, T& uy, T& uz) {
  stored_moments<L, T>([&](auto qc) { return f[(uint64_t)decltype(qc)::value * ps + i]; }, rho0,
                       drho, ux, uy, uz);
}

// Edge-node moments of the current state (after init or a restore).
template <class L, class T>
__global__ __launch_bounds__(256) void k_bplane(const T* __restrict__ f, const uint32_t* __restrict__ links,
                                                T* __restrict__ bp, uint64_t ps, int nx, int ny,
                                                int nz, int xp, T rho0) {
  const uint32_t plane = (uint32_t)nz * ny;
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  if (t >= 2 * plane) return;
  const int side = t / plane;
  const uint32_t yz = t % plane;
  const uint64_t i = (uint64_t)yz * xp + (side == 0 ? 0 : nx - 1);
  T d = 0, ux = 0, uy = 0, uz = 0;
  if (!(links[i] & kSolidBit)) node_moments<L, T>(f, ps, i, rho0, d, ux, uy, uz);
  T* p = bp + (size_t)side * (L::D + 1) * plane + yz;
  p[0] = d;
  p[plane] = ux;
  p[2 * plane] = uy;
  if constexpr (L::D == 3) p[3 * plane] = uz;
}

// Macroscopic fields (unpadded): rho and u [D][nz][ny][nx]; solids rho0, 0.
template <class L, class T, class O>
__global__ __launch_bounds__(256) void k_macro(const T* __restrict__ f, const uint32_t* __restrict__ links,
                                               O* __restrict__ rho, O* __restrict__ u, uint64_t ps,
                                               int nx, int ny, int nz, int xp, T rho0) {
  const uint64_t m = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t N = (uint64_t)nx * ny * nz;
  if (m >= N) return;
  const int x = (int)(m % nx);
  const uint64_t r = m / nx;
  const uint64_t i = r * xp + x;
  T d = 0, ux = 0, uy = 0, uz = 0;
  if (!(links[i] & kSolidBit)) node_moments<L, T>(f, ps, i, rho0, d, ux, uy, uz);
  rho[m] = (O)((double)rho0 + (double)d);
  u[m] = (O)ux;
  u[N + m] = (O)uy;
  if constexpr (L::D == 3) u[2 * N + m] = (O)uz;
}

// x-momentum of the stored populations, summed per block (same tiling as the
// step kernel), for the flux of an arbitrary state.
template <class L, class T>
__global__ __launch_bounds__(kThreads) void k_flux(const T* __restrict__ f,
                                                   const uint32_t* __restrict__ links,
                                                   double* __restrict__ partial, uint64_t ps,
                                                   int nx, int ny, int xp, int tiles_x,
                                                   int tiles_y) {
  const int b = blockIdx.x;
  const int tx = b % tiles_x;
  const int r = b / tiles_x;
  const int ty = r % tiles_y;
  const int z = r / tiles_y;
  const int x = tx * kTileX + threadIdx.x;
  const int y = ty * kTileY + threadIdx.y;
  T jx = T(0);
  if (x < nx && y < ny) {
    const uint64_t i = ((uint64_t)z * ny + y) * xp + x;
    if (!(links[i] & kSolidBit)) {
      unroll<L::xp_begin, L::xp_end>([&](auto qc) { jx += f[(uint64_t)decltype(qc)::value * ps + i]; });
      unroll<L::xm_begin, L::xm_end>([&](auto qc) { jx -= f[(uint64_t)decltype(qc)::value * ps + i]; });
    }
  }
  block_sum_store<kThreads>((double)jx, partial + b);
}

}  // namespace lbm
