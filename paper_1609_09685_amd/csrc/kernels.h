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
//     g[i][k],  i = direction, k = slot of the fluid node,
// as deviations from the rest state, g_i = f_i - w_i rho0.  Each row is cut
// into segments of S = seg bitmap words (S x 64 nodes); a segment's slots start
// on a 128-byte boundary and the slots between its last fluid node and the
// next boundary are padding (always zero).  A block of the step kernel covers
// one segment of each of 4 / S rows, gathers its outputs in LDS and writes
// every segment as whole aligned lines: a wavefront storing its own scattered
// fluid lanes would leave partial lines that the memory system writes at a
// fraction of the bandwidth.
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
// Periodic case (the paper's 3D experiment): every face wraps, so the rows
// and the x-edge lanes pull across the opposite face, with bounce-back at
// solid sources and no mirrors or ghosts; a body force F = rho0 g along x
// enters by the forcing of Guo, Zheng & Shi (2002).
// Collision in deviation form: drho = sum g, j = sum c g, rho = rho0 + drho,
// u = j / rho, g_eq_i = w_i [drho + rho (3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u)],
// g* = g - (g - g_eq)/tau.  The linear ("Stokes") equilibrium drops the two
// quadratic terms (the paper's remedy for inertia in its 3D case).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lattice.h"
#include "pull_index.h"

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
// slot of the first fluid node at or after x = 64 w of that row (fluid nodes of
// one segment have consecutive slots).
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

// Division by a divisor fixed at launch, for 0 <= n < 2^31: q = (mulhi(n, m) +
// n) >> l with l = ceil(log2 d) and m = 2^32 (2^l - d) / d + 1 (round-up
// multiplier; Granlund & Montgomery 1994).  Replaces the scalar division
// sequences of the tile decode.
struct FastDiv {
  uint32_t d, m, l;
  __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
    return (__umulhi(n, m) + n) >> l;
  }
};

// Arguments of one domain's step.
template <class T>
struct StepArgs {
  const T* __restrict__ src;       // populations of step t: direction i at src + i * ps
  T* __restrict__ dst;             // populations of step t+1
  const T* src_g1;                 // src + group_split * ps (second direction group)
  T* dst_g1;
  uint32_t ps_bytes;               // ps * sizeof(T) (32-bit offset kernels)
  const WordDesc* __restrict__ desc;   // D2Q9: per-word records of the fluid bitmap [nz][ny][nw]
  const uint64_t* __restrict__ bits;   // fluid bitmap, guard word at both row ends [nz][ny][nw + 2]
  const uint32_t* __restrict__ pfx;    // slot of each word's first fluid node [nz][ny][nw]
  const T* __restrict__ bp_src;    // edge-node moments of step t: [2 sides][D+1][nz*ny]
  T* __restrict__ bp_dst;          // edge-node moments written by this step
  double* __restrict__ partial;    // per-word flux partials (flux variant)
  uint64_t ps;                     // elements between two direction arrays
  int nx, ny, nz, nw;              // lattice; nw = bitmap words per row
  int seg;                         // S: words (64 x) per segment and tile: 1, 2 or 4
  int seg_log;                     // log2(S)
  int tiles_x, tiles_y;            // ceil(nw / S), ceil(ny / (4 / S))
  uint32_t align;                  // slots per 128 bytes
  int blocks;                      // tiles_x * tiles_y * nz
  int xcd_remap;                   // tile order mode (see logical_block)
  int chunk;                       // tiles per chunk in mode >= 2
  int band;                        // > 0: banded order, band = tile rows per band
  int nbands;                      // ceil(tiles_y / band)
  FastDiv dv_tiles_x, dv_tiles_y, dv_chunk;
  FastDiv dv_band_blocks, dv_band_plane;   // nz * band * tiles_x, band * tiles_x
  T omega, rho0, drho_in, drho_out;  // 1/tau; rho0; rho_in - rho0; rho_out - rho0
  T fx;                            // body-force density along x (rho0 g), periodic case
  T omega_m;                       // TRT: 1/tau- (odd part); omega otherwise
  T trt_a, trt_b;                  // TRT: (omega +- omega_m) / 2
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

// Deterministic reduction of n partials in two passes with a fixed chunking
// (independent of how the partials were produced): pass 1 sums chunk c =
// [c * kChunk, (c + 1) * kChunk) in a fixed order into chunk[c]; pass 2 sums the
// chunks in a fixed order, out = scale * total.
constexpr int kChunk = 8192;

__device__ __forceinline__ double block1024_sum(double v) {
  __shared__ double s[16];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < 16; ++i) t += s[i];
  return t;   // valid in thread 0
}

// Sum of chunk c of n partials (fixed order) -> *out (thread 0).
__device__ __forceinline__ void reduce_chunk(const double* __restrict__ partial, int n, int c,
                                             double* __restrict__ out) {
  const int base = c * kChunk;
  double v = 0.0;
  for (int j = threadIdx.x; j < kChunk; j += 1024)
    if (base + j < n) v += partial[base + j];
  const double t = block1024_sum(v);
  if (threadIdx.x == 0) *out = t;
}

// Sum of nchunks chunk sums (fixed order) times scale -> *out (thread 0).
__device__ __forceinline__ void reduce_final(const double* __restrict__ chunk, int nchunks,
                                             double scale, double* __restrict__ out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nchunks; i += 1024) v += chunk[i];
  const double t = block1024_sum(v);
  if (threadIdx.x == 0) *out = scale * t;
}

static __global__ __launch_bounds__(1024) void k_reduce_chunks(const double* __restrict__ partial, int n,
                                                        double* __restrict__ chunk) {
  reduce_chunk(partial, n, blockIdx.x, chunk + blockIdx.x);
}

static __global__ __launch_bounds__(1024) void k_reduce_final(const double* __restrict__ chunk, int nchunks,
                                                       double scale, double* __restrict__ out) {
  reduce_final(chunk, nchunks, scale, out);
}

// Flux reduction of many domains at once.  Domain d's partials, chunk sums and
// result: part[d], chunk[d], out[d]; its chunks are blocks
// [chunk_start[d], chunk_start[d + 1]) of the first launch and block d of the
// second.  Same arithmetic, chunk by chunk, as the single-domain kernels.
struct BatchReduce {
  const double* const* part;
  double* const* chunk;
  const int* nparts;
  const int* chunk_start;     // [n + 1]
  const int* chunk_owner;     // domain of each chunk block
  const double* scale;        // 1 / nx of each domain
  double* out;
};

static __global__ __launch_bounds__(1024) void k_reduce_chunks_batch(BatchReduce r) {
  const int d = r.chunk_owner[blockIdx.x];
  const int c = blockIdx.x - r.chunk_start[d];
  reduce_chunk(r.part[d], r.nparts[d], c, r.chunk[d] + c);
}

static __global__ __launch_bounds__(1024) void k_reduce_final_batch(BatchReduce r) {
  const int d = blockIdx.x;
  reduce_final(r.chunk[d], r.chunk_start[d + 1] - r.chunk_start[d], r.scale[d], r.out + d);
}

// -------------------------------------------------------------- equilibrium

// 1 / rho for the velocity.  FP32: the hardware reciprocal (1 ulp); FP64: a
// correctly rounded division.
template <class T>
__device__ __forceinline__ T recip(T v) {
  if constexpr (std::is_same<T, float>::value) return __builtin_amdgcn_rcpf(v);
  return T(1) / v;
}


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
  const T inv = recip(rho0 + d);
  drho = d;
  ux = jx * inv;
  uy = jy * inv;
  uz = jz * inv;
}

// --------------------------------------------------------------- time step

// Non-equilibrium extrapolation term of a ghost population (rule 3).
template <class L, bool LINEAR, class T>
__device__ __forceinline__ T ghost_term(const T* __restrict__ bp, int side, uint32_t plane,
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

// The record of word w of row `row` (wave-uniform: scalar loads).  D2Q9 (3
// source rows per wave) reads it from the records stored at set-up; D3Q19 (9
// source rows) forms it from the bitmap words w - 1, w, w + 1 (guard words at
// the row ends) and the first slots of the words.  Measured both ways: the
// stored records make the batched D2Q9 step 17 % faster (1.66 against
// 2.02 ms for 256 samples) and the 512^3 D3Q19 step 1.5 % slower (2.82
// against 2.78 ms).
template <class L, class T>
__device__ __forceinline__ WordDesc load_desc(const StepArgs<T>& a, uint32_t row, int w) {
  if constexpr (L::D == 2) return a.desc[row * (uint32_t)a.nw + (uint32_t)w];
  const uint64_t* wr = a.bits + row * (uint32_t)(a.nw + 2) + 1u;
  const uint32_t* pr = a.pfx + row * (uint32_t)a.nw;
  const bool hp = w > 0, hn = w + 1 < a.nw;
  return make_word_desc(wr[w - 1], wr[w], wr[w + 1], pr[hp ? w - 1 : w], pr[w], pr[hn ? w + 1 : w],
                        hp, hn);
}

// Updates the node x = 64 w + lane of row (y, z); y, z, w are uniform across
// the wave.  YZE: the row touches a symmetric plane (mirrors possible) or, with
// periodic faces, a y / z face (wraps); XE: the word holds x = 0 or x = nx - 1.
// Interior waves (neither) skip all boundary logic.  OFF32: each direction
// group spans less than 4 GiB, so a load is a wave-uniform base plus a 32-bit
// lane offset.  The post-collision populations go to out[i][lds_base + slot]
// (LDS; lds_base = the block-local position of the segment minus its first
// slot).  Returns the node's x-momentum (with a body force, j_x + F/2; 0 if the
// node is not fluid).
//
// Gather.  Every source row is described by its word record (wave-uniform).
// For direction i the lanes whose source is fluid form a 64-bit mask (the
// row's bits, shifted by c_x), which selects per lane between the source slot
// and the node's own slot of the opposite direction (bounce-back).  Both
// candidates lie in one direction group; the load base is the group base plus
// the smaller of the two direction offsets, so each candidate is one 32-bit
// lane offset.
template <class L, class T, bool LINEAR, bool OFF32, bool PER, bool TRT, bool YZE, bool XE>
__device__ __forceinline__ T node_update(const StepArgs<T>& a, int y, int z, int w, int lane,
                                         T (*out)[kThreads], uint32_t lds_base) {
  const WaveLane ln;
  const int x = (w << 6) + lane;
  constexpr bool per = PER;
  // symmetric planes (pressure case only)
  const bool y0 = YZE && !per && y == 0, y1 = YZE && !per && y == a.ny - 1;
  const bool z0 = YZE && !per && L::D == 3 && z == 0;
  const bool z1 = YZE && !per && L::D == 3 && z == a.nz - 1;
  const uint32_t row_self = (uint32_t)z * (uint32_t)a.ny + (uint32_t)y;
  WordEdges we;
  we.x0 = XE && w == 0;
  we.x1 = XE && w == ((a.nx - 1) >> 6);
  we.e = (a.nx - 1) & 63;

  // source rows (y + dy, z + dz): mirrored onto the own row at a symmetric
  // plane, wrapped to the opposite face in the periodic case
  SourceRow rw[3][3];
  unroll<0, 3>([&](auto izc) {
    constexpr int dz = decltype(izc)::value - 1;
    if constexpr (L::D == 3 || dz == 0) {
      unroll<0, 3>([&](auto iyc) {
        constexpr int dy = decltype(iyc)::value - 1;
        int ey = dy, ez = dz;
        if constexpr (YZE) {
          if constexpr (PER) {
            if (dy < 0 && y == 0) ey = a.ny - 1;
            if (dy > 0 && y == a.ny - 1) ey = 1 - a.ny;
            if (dz < 0 && z == 0) ez = a.nz - 1;
            if (dz > 0 && z == a.nz - 1) ez = 1 - a.nz;
          } else {
            if ((dy < 0 && y0) || (dy > 0 && y1)) ey = 0;
            if ((dz < 0 && z0) || (dz > 0 && z1)) ez = 0;
          }
        }
        const uint32_t row = row_self + (uint32_t)(ez * a.ny + ey);
        const WordDesc d = load_desc<L>(a, row, w);
        SourceRow& r = rw[dz + 1][dy + 1];
        r.mid = desc_bits(d);
        r.base = d.base;
        r.info = d.info;
        if constexpr (XE && PER) row_x_faces(load_desc<L>(a, row, 0), load_desc<L>(a, row, a.nw - 1), a.nx, r);
      });
    }
  });
  const SourceRow& me = rw[1][1];
  if (!ln.bit(me.mid)) return T(0);   // solid node, or x >= nx
  const uint32_t self = ln.rank(me.mid, me.base);
  const uint32_t selfb = self * (uint32_t)sizeof(T);

  T g[L::Q];
  bool ghm[L::Q];   // pressure ghost source (x-edge lanes)
  unroll<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int cx = L::cx[q], cy = L::cy[q], cz = L::cz[q];
    ghm[q] = false;
    if constexpr (q == 0) {
      g[0] = a.src[self];
    } else {
      const SourceRow& r = rw[1 - cz][1 - cy];
      // direction read by a fluid source: q, or its mirror image
      int k = q;
      if constexpr (YZE && q != 0) {
        bool fy = false, fz = false;
        if constexpr (cy > 0) fy = y0;
        if constexpr (cy < 0) fy = y1;
        if constexpr (cz > 0) fz = z0;
        if constexpr (cz < 0) fz = z1;
        constexpr int kY = L::my[q], kZ = L::mz[q], kYZ = L::mz[L::my[q]];
        k = fy ? (fz ? kYZ : kY) : (fz ? kZ : q);
      }
      constexpr int o = L::opp[q];
      uint64_t m, gm;
      uint32_t off;
      if constexpr (OFF32) {
        // group base + the smaller of the two direction offsets, so that both
        // candidates are non-negative 32-bit lane offsets
        constexpr int first = q < L::group_split ? 0 : L::group_split;
        const char* base = q < L::group_split ? (const char*)a.src : (const char*)a.src_g1;
        uint32_t lo, dk, dob;   // lo + dk: direction read; lo + dob: opposite direction
        if constexpr (!YZE) {   // k = q
          if constexpr (o > q) {
            lo = (uint32_t)(q - first) * a.ps_bytes;
            dk = 0u;
            dob = (uint32_t)(o - q) * a.ps_bytes;
          } else {
            lo = (uint32_t)(o - first) * a.ps_bytes;
            dk = (uint32_t)(q - o) * a.ps_bytes;
            dob = 0u;
          }
        } else {
          const uint32_t ck = (uint32_t)(k - first) * a.ps_bytes;
          const uint32_t co = (uint32_t)(o - first) * a.ps_bytes;
          lo = ck < co ? ck : co;
          dk = ck - lo;
          dob = co - lo;
        }
        pull_offset<cx, PER, (uint32_t)sizeof(T)>(ln, r, ln.rank(r.mid, 0u), we, dk, m, off, gm);
        const uint32_t ob = selfb + dob;
        off = __builtin_unpredictable(ln.bit(m)) ? off : ob;
        g[q] = *(const T*)(base + lo + off);
      } else {
        pull_offset<cx, PER, 1u>(ln, r, ln.rank(r.mid, 0u), we, 0u, m, off, gm);
        const uint64_t idx = ln.bit(m) ? (uint64_t)k * a.ps + off : (uint64_t)o * a.ps + self;
        g[q] = a.src[idx];
      }
      ghm[q] = ln.bit(gm);
    }
  });

  // Ghost populations: add the non-equilibrium extrapolation term.
  if constexpr (XE && !PER) {
    unroll<1, L::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int cx = L::cx[q], cy = L::cy[q], cz = L::cz[q];
      if constexpr (cx != 0) {
        if (ghm[q]) {
          bool fy = false, fz = false;
          if constexpr (cy > 0) fy = y0;
          if constexpr (cy < 0) fy = y1;
          if constexpr (cz > 0) fz = z0;
          if constexpr (cz < 0) fz = z1;
          const int ys = fy ? y : y - cy, zs = fz ? z : z - cz;
          g[q] += ghost_term<L, LINEAR, T>(a.bp_src, cx > 0 ? 0 : 1, (uint32_t)a.nz * a.ny,
                                           (uint32_t)zs * a.ny + ys,
                                           cx > 0 ? a.drho_in : a.drho_out, T(L::w[q]), cx,
                                           fy ? -cy : cy, fz ? -cz : cz);
        }
      }
    });
  }

  // Moments from the sums and differences of opposite pairs (q, q + 1).
  T drho = g[0], jx = T(0), jy = T(0), jz = T(0);
  unroll<0, (L::Q - 1) / 2>([&](auto pc) {
    constexpr int q = 1 + 2 * decltype(pc)::value, o = q + 1;
    static_assert(L::opp[q] == o && L::w[q] == L::w[o], "opposite pairs (q, q + 1)");
    drho += g[q] + g[o];
    const T d = g[q] - g[o];
    if constexpr (L::cx[q] == 1) jx += d;
    if constexpr (L::cx[q] == -1) jx -= d;
    if constexpr (L::cy[q] == 1) jy += d;
    if constexpr (L::cy[q] == -1) jy -= d;
    if constexpr (L::cz[q] == 1) jz += d;
    if constexpr (L::cz[q] == -1) jz -= d;
  });
  // with a body force (Guo et al. 2002) the velocity carries half the step's
  // force density: rho u = j + F/2
  T jxe = jx;
  if constexpr (PER) jxe += T(0.5) * a.fx;
  // The linear equilibrium w_i (rho + 3 c_i.(rho u)) needs only the momentum:
  // it is formed from rho u directly (geq with rho = 1, u = rho u), so the
  // update stays exactly linear in the deviations and the force.
  T rho, ux, uy, uz;
  if constexpr (LINEAR) {
    rho = T(1);
    ux = jxe;
    uy = jy;
    uz = jz;
  } else {
    rho = a.rho0 + drho;
    const T inv = recip(rho);
    ux = jxe * inv;
    uy = jy * inv;
    uz = jz * inv;
  }
  const T usq15 = T(1.5) * (ux * ux + uy * uy + uz * uz);
  if constexpr (TRT) {
    // Two relaxation times: the non-equilibrium n = g - g_eq of a direction
    // and of its opposite split into an even half, relaxed with omega, and an
    // odd half, relaxed with omega_m; per direction that is
    // g' = g - a n_i - b n_opp(i), a, b = (omega +- omega_m)/2.  The force
    // term splits the same way: its odd half is 3 w_i c_ix F, its even half
    // w_i (9 c_ix (c_i.u) - 3 u_x) F (absent with the linear equilibrium),
    // each with its own (1 - omega/2) factor.
    T nq[L::Q];
    unroll<0, L::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      nq[q] = g[q] - geq<L, q, LINEAR>(drho, rho, ux, uy, uz, usq15);
    });
    T af_even = T(0), af_odd = T(0);
    if constexpr (PER) {
      af_even = (T(1) - T(0.5) * a.omega) * a.fx;
      af_odd = (T(1) - T(0.5) * a.omega_m) * a.fx;
    }
    unroll<0, L::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int cx = L::cx[q];
      T v = g[q] - a.trt_a * nq[q] - a.trt_b * nq[L::opp[q]];
      if constexpr (PER) {
        if constexpr (cx != 0) v += T(3 * cx) * T(L::w[q]) * af_odd;
        if constexpr (!LINEAR) {
          const T cu = dot_c<L, q>(ux, uy, uz);
          v += T(L::w[q]) * af_even * (T(9 * cx) * cu - T(3) * ux);
        }
      }
      out[q][lds_base + self] = v;
      g[q] = v;
    });
  } else if constexpr (!PER) {
    // BGK, g' = (1 - omega) g + omega g_eq.  With a = omega w_i, the relaxed
    // equilibrium is a [drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)]
    // = c0 + c1 (c.u)^2 +- c2 (c.u) for a direction and its opposite, where
    // c0 = a (drho - rho 3/2 u.u), c1 = 9/2 a rho, c2 = 3 a rho depend only on
    // the weight class (the linear equilibrium: c0 = a drho, c1 = 0, c2 = 3 a).
    const T om = a.omega, om1 = T(1) - a.omega;
    T ev = drho;
    if constexpr (!LINEAR) ev = drho - rho * usq15;
    g[0] = om1 * g[0] + (om * T(L::w[0])) * ev;
    out[0][lds_base + self] = g[0];
    T c0[2], c1[2], c2[2];   // [0] axis directions, [1] diagonal ones
    unroll<0, 2>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      const T ac = om * T(L::w[c == 0 ? 1 : L::Q - 1]);
      c0[c] = ac * ev;
      if constexpr (LINEAR) {
        c1[c] = T(0);
        c2[c] = T(3) * ac;
      } else {
        const T ra = ac * rho;
        c1[c] = T(4.5) * ra;
        c2[c] = T(3) * ra;
      }
    });
    unroll<0, (L::Q - 1) / 2>([&](auto pc) {
      constexpr int q = 1 + 2 * decltype(pc)::value, o = q + 1;
      constexpr int c = L::w[q] == L::w[1] ? 0 : 1;
      static_assert(L::w[q] == L::w[c == 0 ? 1 : L::Q - 1], "two weight classes");
      const T cu = dot_c<L, q>(ux, uy, uz);
      T P, M;
      if constexpr (LINEAR) {
        P = c2[c] * cu + c0[c];
        M = c0[c] - c2[c] * cu;
      } else {
        P = (c1[c] * cu + c2[c]) * cu + c0[c];
        M = (c1[c] * cu - c2[c]) * cu + c0[c];
      }
      g[q] = om1 * g[q] + P;
      g[o] = om1 * g[o] + M;
      out[q][lds_base + self] = g[q];
      out[o][lds_base + self] = g[o];
    });
  } else {
    // forcing term (1 - omega/2) F_i, F_i = w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)],
    // or 3 w_i c_i.F with the linear equilibrium; F = (fx, 0, 0)
    const T af = (T(1) - T(0.5) * a.omega) * a.fx;
    unroll<0, L::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int cx = L::cx[q];
      const T ge = geq<L, q, LINEAR>(drho, rho, ux, uy, uz, usq15);
      T fi;
      if constexpr (LINEAR) {
        fi = T(3 * cx) * T(L::w[q]) * af;
      } else {
        const T cu = dot_c<L, q>(ux, uy, uz);
        fi = T(L::w[q]) * af * (T(3) * (T(cx) - ux) + T(9 * cx) * cu);
      }
      g[q] = g[q] - a.omega * (g[q] - ge) + fi;
      out[q][lds_base + self] = g[q];
    });
  }

  if constexpr (XE && !PER) {
    const bool x0 = we.x0 && x == 0, x1 = we.x1 && x == a.nx - 1;
    if (x0 || x1) {
      // edge-node moments of the stored state, read by the next step's ghosts
      T bd, bx, by, bz;
      stored_moments<L, T>([&](auto qc) { return g[decltype(qc)::value]; }, a.rho0, bd, bx, by, bz);
      const uint32_t plane = (uint32_t)a.nz * a.ny;
      T* bp = a.bp_dst + (size_t)(x0 ? 0 : 1) * (L::D + 1) * plane + row_self;
      bp[0] = bd;
      bp[plane] = bx;
      bp[2 * plane] = by;
      if constexpr (L::D == 3) bp[3 * plane] = bz;
    }
  }
  return jxe;
}

// Picks the specialisation of node_update for a wave's (y, z, w).
template <class L, class T, bool LINEAR, bool OFF32, bool PER, bool TRT>
__device__ __forceinline__ T wave_update(const StepArgs<T>& a, int y, int z, int w, int lane,
                                         T (*out)[kThreads], uint32_t lds_base) {
  const bool yze = y == 0 || y == a.ny - 1 || (L::D == 3 && (z == 0 || z == a.nz - 1));
  const bool xe = w == 0 || w == ((a.nx - 1) >> 6);
  if (yze) {
    if (xe) return node_update<L, T, LINEAR, OFF32, PER, TRT, true, true>(a, y, z, w, lane, out, lds_base);
    return node_update<L, T, LINEAR, OFF32, PER, TRT, true, false>(a, y, z, w, lane, out, lds_base);
  }
  if (xe) return node_update<L, T, LINEAR, OFF32, PER, TRT, false, true>(a, y, z, w, lane, out, lds_base);
  return node_update<L, T, LINEAR, OFF32, PER, TRT, false, false>(a, y, z, w, lane, out, lds_base);
}

// Order in which tiles meet the hardware.  The dispatcher deals block ids
// round-robin over the 8 XCDs (block h runs on XCD h % 8), each with its own
// L2.  Neighbouring tiles share the cache lines at the ends of their compact
// ranges, so they should run on one XCD; and all XCDs should work on one
// compact region at a time, so that DRAM pages stay open and the memory-side
// cache catches what the L2s both fetch.  Modes:
//   0  hardware order (neighbouring tiles on different XCDs);
//   1  each XCD gets one contiguous eighth of the tiles;
//   c >= 2  chunks of `chunk` consecutive tiles are dealt round-robin to the
//      XCDs, so the XCDs work side by side on eight neighbouring chunks.
// Modes 1 and 2+ need a grid padded to a multiple of 8 (mode 1) or
// 8 * chunk (mode 2+); blocks whose logical tile is past the end exit.
template <class T>
__device__ __forceinline__ int logical_block(int hw, const StepArgs<T>& a) {
  if (a.xcd_remap == 0) return hw;
  if (a.xcd_remap == 1) {
    const int per = (a.blocks + 7) >> 3;
    return (hw & 7) * per + (hw >> 3);
  }
  const uint32_t k = (uint32_t)hw >> 3;
  const uint32_t kc = a.dv_chunk.div(k);
  return (int)(kc * 8u * a.dv_chunk.d + (uint32_t)(hw & 7) * a.dv_chunk.d + (k - kc * a.dv_chunk.d));
}

// One time step of one domain.  A block's four waves cover one segment (S
// consecutive 64-wide words) of each of 4 / S rows of one z plane, one word per
// wave.  Tile order: logical_block, or with band > 0 the banded order: XCD
// h % 8 takes bands h % 8, h % 8 + 8, ... of `band` tile rows and walks each
// band plane by plane, so the rows a node pulls from (y +- 1, z +- 1) are
// processed close together in time on one XCD and the cache lines two waves
// share are fetched once.  The block gathers its post-collision populations in
// LDS and then writes each segment as whole aligned lines (padding slots get
// zero).  FLUX: each wave also stores the FP64 sum of its 64 nodes'
// x-momentum at the index of its bitmap word, (z ny + y) nw + w, so the flux
// does not depend on the tiling.
template <class L, class T, bool FLUX, bool LINEAR, bool OFF32, bool PER, bool TRT>
__device__ __forceinline__ void step_tile(const StepArgs<T>& a, const uint32_t hw) {
  __shared__ T out[L::Q][kThreads];
  __shared__ uint32_t seg_first[kRows], seg_count[kRows];
  int tx, ty, z;
  if (a.band > 0) {
    const uint32_t k = hw >> 3;
    const uint32_t round = a.dv_band_blocks.div(k);
    const uint32_t kk = k - round * a.dv_band_blocks.d;
    const int bi = (int)(round * 8u + (hw & 7u));
    if (bi >= a.nbands) return;   // whole block: padding band
    const uint32_t zp = a.dv_band_plane.div(kk);
    const uint32_t rem = kk - zp * a.dv_band_plane.d;
    const uint32_t tyl = a.dv_tiles_x.div(rem);
    tx = (int)(rem - tyl * (uint32_t)a.tiles_x);
    ty = bi * a.band + (int)tyl;
    z = (int)zp;
    if (ty >= a.tiles_y) return;   // whole block: past the last tile row
  } else {
    const int b = logical_block((int)hw, a);
    if (b >= a.blocks) return;     // whole block: padding of the remapped grid
    const uint32_t r = a.dv_tiles_x.div((uint32_t)b);
    tx = b - (int)(r * (uint32_t)a.tiles_x);
    const uint32_t zz = a.dv_tiles_y.div(r);
    ty = (int)(r - zz * (uint32_t)a.tiles_y);
    z = (int)zz;
  }
  const int S = a.seg;
  const int wave = threadIdx.y, lane = threadIdx.x;
  const int j = uniform(wave >> a.seg_log);         // row of the tile
  const int y = uniform(ty * (kRows / S) + j);
  const int w0 = tx * S;                            // first word of the segment
  const int w = uniform(w0 + (wave & (S - 1)));
  z = uniform(z);
  const bool row_ok = y < a.ny;
  const uint32_t row = (uint32_t)z * (uint32_t)a.ny + (uint32_t)y;
  // segment of this wave's row: first slot and number of fluid nodes (slots
  // run on without gaps inside a segment)
  uint32_t first = 0u, count = 0u;
  if (row_ok) {
    segment_extent(load_desc<L>(a, row, w0), load_desc<L>(a, row, min(w0 + S, a.nw) - 1), first, count);
  }
  if ((wave & (S - 1)) == 0 && lane == 0) {
    seg_first[j] = first;
    seg_count[j] = count;
  }
  T jx = T(0);
  if (row_ok && w < a.nw) {
    const uint32_t lds_base = (uint32_t)(j * S * kWave) - first;
    jx = wave_update<L, T, LINEAR, OFF32, PER, TRT>(a, y, z, w, lane, out, lds_base);
  }
  if constexpr (FLUX) {
    if (row_ok && w < a.nw) {
      const double s = wave_sum((double)jx);
      if (lane == 0) a.partial[(size_t)row * a.nw + w] = s;
    }
  }
  __syncthreads();
  // whole-line stores: thread t writes position t of its row's segment (zero
  // past the segment's fluid nodes, up to the next 128-byte boundary); the
  // next step reads them from HBM anyway, so they bypass the caches
  // (nontemporal)
  const int t = wave * kWave + lane;
  const int sh = a.seg_log + 6;                     // log2(S * 64)
  const int jj = t >> sh;
  const uint32_t r = (uint32_t)t & ((1u << sh) - 1u);
  const uint32_t n = seg_count[jj];
  const uint32_t lim = (n + a.align - 1u) & ~(a.align - 1u);
  if (r < lim) {
    const uint32_t slot = seg_first[jj] + r;
    const bool live = r < n;
    unroll<0, L::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      T v = out[q][t];
      v = live ? v : T(0);
      if constexpr (OFF32) {
        constexpr int f = q < L::group_split ? 0 : L::group_split;
        char* base = (q < L::group_split ? (char*)a.dst : (char*)a.dst_g1) +
                     (uint32_t)(q - f) * a.ps_bytes;
        __builtin_nontemporal_store(v, (T*)(base + slot * (uint32_t)sizeof(T)));
      } else {
        __builtin_nontemporal_store(v, a.dst + ((uint64_t)q * a.ps + slot));
      }
    });
  }
}

// Waves per SIMD the step kernels ask the register allocator for: the
// single-domain FP32 pressure-driven BGK kernels fit 8 (the LDS limit) by
// moving scalar values into vector lanes; the others (FP64, periodic, TRT,
// and the batch kernels, which read their arguments from memory) would spill
// to scratch and keep the allocator's own choice.
template <class T, bool PER, bool TRT>
constexpr int step_min_waves() { return sizeof(T) == 4 && !PER && !TRT ? 8 : 1; }

template <class L, class T, bool FLUX, bool LINEAR, bool OFF32, bool PER, bool TRT>
__global__ __launch_bounds__(kThreads) __attribute__((
    amdgpu_waves_per_eu(step_min_waves<T, PER, TRT>()))) void k_step(const StepArgs<T> a) {
  step_tile<L, T, FLUX, LINEAR, OFF32, PER, TRT>(a, blockIdx.x);
}

// One time step of many domains in one launch.  Block b runs block owner[b].y
// of the launch of domain owner[b].x, or nothing when owner[b].x < 0 (table
// padding, and the tail left by domains that have retired).  Each domain's
// blocks start at a multiple of 8, so block b runs on the XCD that block
// owner[b].y of the domain's own launch would: the tile orders carry over.
// args[2 d + flip] holds the arguments of domain d for this step (the two
// entries of a domain differ by the ping-pong parity).
// p, re-derived through the global address space: a pointer loaded from
// memory is generic to the compiler (flat loads and stores, vector loads of
// uniform values); the cast lets it use global and scalar memory
// instructions, as it does for pointers passed as kernel arguments.
template <class P>
__device__ __forceinline__ P* in_global(P* p) {
  return (P*)(__attribute__((address_space(1))) P*)(uintptr_t)p;
}

template <class L, class T, bool FLUX, bool LINEAR, bool OFF32, bool PER, bool TRT>
__global__ __launch_bounds__(kThreads) void k_step_batch(const StepArgs<T>* __restrict__ args,
                                                         const int2* __restrict__ owner, int flip) {
  const int2 o = owner[blockIdx.x];
  if (o.x < 0) return;   // whole block
  StepArgs<T> a = args[2 * o.x + flip];
  // every buffer of a context is device memory
  a.src = in_global(a.src);
  a.dst = in_global(a.dst);
  a.src_g1 = in_global(a.src_g1);
  a.dst_g1 = in_global(a.dst_g1);
  a.desc = in_global(a.desc);
  a.bits = in_global(a.bits);
  a.pfx = in_global(a.pfx);
  a.bp_src = in_global(a.bp_src);
  a.bp_dst = in_global(a.bp_dst);
  a.partial = in_global(a.partial);
  step_tile<L, T, FLUX, LINEAR, OFF32, PER, TRT>(a, (uint32_t)o.y);
}

// ------------------------------------------------------------ set-up kernels

// Bitmap words and per-word fluid counts from the solid mask (uint8
// [nz][ny][nx], 1 = solid).  One wave per word: the lanes ballot their nodes.
// Also writes the two guard words of each row.
static __global__ __launch_bounds__(256) void k_pack_bits(const uint8_t* __restrict__ mask,
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

static __global__ __launch_bounds__(kScanBlock) void k_scan_local(const uint32_t* __restrict__ in,
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
static __global__ __launch_bounds__(kScanBlock) void k_scan_totals(uint32_t* __restrict__ tot, int nb,
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

static __global__ __launch_bounds__(kScanBlock) void k_scan_add(uint32_t* __restrict__ out,
                                                         const uint32_t* __restrict__ block_tot,
                                                         uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) out[i] += block_tot[blockIdx.x];
}

// Padded size of every segment (S words of a row): its fluid count rounded up
// to `align` slots.
static __global__ __launch_bounds__(256) void k_seg_sizes(const uint32_t* __restrict__ count,
                                                   uint32_t* __restrict__ seg_size, uint64_t nsegs,
                                                   int nw, int S, int segs_per_row, uint32_t align) {
  const uint64_t sg = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (sg >= nsegs) return;
  const uint64_t row = sg / segs_per_row;
  const int w0 = (int)(sg % segs_per_row) * S;
  const int we = min(w0 + S, nw);
  uint32_t n = 0;
  for (int i = w0; i < we; ++i) n += count[row * nw + i];
  seg_size[sg] = (n + align - 1u) & ~(align - 1u);
}

// Slot of the first fluid node of every word: the segment's first slot plus the
// fluid nodes of the segment's earlier words.
static __global__ __launch_bounds__(256) void k_word_pfx(const uint32_t* __restrict__ count,
                                                  const uint32_t* __restrict__ seg_first,
                                                  uint32_t* __restrict__ pfx, uint64_t nwords, int nw,
                                                  int S, int segs_per_row) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nwords) return;
  const uint64_t row = i / nw;
  const int w = (int)(i % nw);
  const int s = w / S;
  uint32_t p = seg_first[row * segs_per_row + s];
  for (int k = s * S; k < w; ++k) p += count[row * nw + k];
  pfx[i] = p;
}

// Per-word records (WordDesc) from the bitmap (guard words of zeros at both
// row ends) and the slots of the words; the D2Q9 step kernels read them.
static __global__ __launch_bounds__(256) void k_word_desc(FluidMap fm, WordDesc* __restrict__ desc,
                                                   uint64_t nwords) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nwords) return;
  const uint64_t row = i / fm.nw;
  const int w = (int)(i % fm.nw);
  const uint64_t* wr = fm.bits + row * (uint64_t)(fm.nw + 2) + 1;
  const uint32_t* pr = fm.pfx + row * (uint64_t)fm.nw;
  const bool has_prev = w > 0, has_next = w + 1 < fm.nw;
  desc[i] = make_word_desc(wr[w - 1], wr[w], wr[w + 1], has_prev ? pr[w - 1] : 0u, pr[w],
                           has_next ? pr[w + 1] : 0u, has_prev, has_next);
}

// Slot of every node (x fastest), -1 for solids.
static __global__ __launch_bounds__(256) void k_slot_map(FluidMap fm, int32_t* __restrict__ map) {
  const uint64_t m = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= (uint64_t)fm.nx * fm.ny * fm.nz) return;
  const int x = (int)(m % fm.nx);
  const uint64_t r = m / fm.nx;
  bool fluid;
  const uint32_t k = fm.rank(x, (int)(r % fm.ny), (int)(r / fm.ny), fluid);
  map[m] = fluid ? (int32_t)k : -1;
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

// Equilibrium of given fields: rho [nz][ny][nx], u [D][nz][ny][nx] (float32);
// the model's own equilibrium (LINEAR: without the terms quadratic in u).
template <class L, class T, bool LINEAR>
__global__ __launch_bounds__(256) void k_init_fields(T* __restrict__ f, FluidMap fm,
                                                     const float* __restrict__ rho_f,
                                                     const float* __restrict__ u_f, uint64_t ps,
                                                     double rho0, double fhalf) {
  const uint64_t N = (uint64_t)fm.nx * fm.ny * fm.nz;
  const uint64_t m = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= N) return;
  const int x = (int)(m % fm.nx);
  const uint64_t r = m / fm.nx;
  bool fluid;
  const uint32_t k = fm.rank(x, (int)(r % fm.ny), (int)(r / fm.ny), fluid);
  if (!fluid) return;
  // stored (post-collision) momentum rho u + F/2 for a body force F along x
  const double rho = rho_f[m], ux = u_f[m] + fhalf / rho, uy = u_f[N + m];
  const double uz = L::D == 3 ? (double)u_f[2 * N + m] : 0.0;
  const double usq15 = 1.5 * (ux * ux + uy * uy + uz * uz);
  const double drho = rho - rho0;
  unroll<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    f[(uint64_t)q * ps + k] = (T)geq<L, q, LINEAR, double>(drho, rho, ux, uy, uz, usq15);
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
// fhalf = F/2 of a body force along x (0 without one): the stored populations
// are post-collision, so the velocity of the forcing scheme is (j - F/2)/rho.
template <class L, class T, class O>
__global__ __launch_bounds__(256) void k_macro(const T* __restrict__ f, FluidMap fm,
                                               O* __restrict__ rho, O* __restrict__ u, uint64_t ps,
                                               T rho0, T fhalf) {
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
  if (fluid && fhalf != T(0)) ux -= fhalf * recip(rho0 + d);
  rho[m] = (O)((double)rho0 + (double)d);
  u[m] = (O)ux;
  u[N + m] = (O)uy;
  if constexpr (L::D == 3) u[2 * N + m] = (O)uz;
}

// x-momentum of the stored populations, summed per block of 256 compact nodes.
// a[k] = (a[k] + b[k]) / 2 over n values: the mean of two consecutive states
// (padding slots are zero in both and stay zero).
template <class T>
__global__ __launch_bounds__(256) void k_mean_states(T* __restrict__ a, const T* __restrict__ b,
                                                     uint64_t n) {
  const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) a[k] = T(0.5) * (a[k] + b[k]);
}

template <class L, class T>
__global__ __launch_bounds__(256) void k_flux(const T* __restrict__ f, uint64_t n_fluid,
                                              uint64_t ps, double* __restrict__ partial) {
  const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  T jx = T(0);
  if (k < n_fluid) {
    unroll<1, L::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if constexpr (L::cx[q] == 1) jx += f[(uint64_t)q * ps + k];
      if constexpr (L::cx[q] == -1) jx -= f[(uint64_t)q * ps + k];
    });
  }
  block_sum_store<256>((double)jx, partial + blockIdx.x);
}

}  // namespace lbm
