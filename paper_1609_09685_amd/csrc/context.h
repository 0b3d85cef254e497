// Host-side internals shared by the library's translation units: the
// context of one domain, its work-buffer layout and the step arguments built
// from it.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"
#include "lbm.h"

namespace lbm {
namespace host {

// Records the message (printf format) for lbm_last_error() and returns s.
lbm_status fail(lbm_status s, const char* fmt, ...);
// Clears the message and returns LBM_OK.
lbm_status ok();

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::lbm::host::fail(LBM_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                               __FILE__, __LINE__);                                     \
  } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  int Q, D;
  size_t esize;          // bytes per population value
  int nw;                // bitmap words per row
  int S;                 // words per segment (and per step tile row): 1, 2 or 4
  int segs_per_row;      // ceil(nw / S)
  uint32_t align;        // slots per 128 bytes
  uint64_t rows;         // ny * nz
  uint64_t nsegs;        // rows * segs_per_row
  uint64_t n_fluid;
  uint64_t ps;           // slots per direction array: room for every segment's padding
  size_t f_bytes;
  int scan_blocks, seg_scan_blocks;
  size_t off_bits, off_pfx, off_desc, off_count, off_scan, off_seg, off_seg_scan, off_bplane, off_partial,
      off_scalar, work_bytes;
  size_t bplane_one;     // elements of one parity of the boundary-plane array
  int partials;          // capacity of the partial array
  int chunks;            // capacity of the chunk-sum array
};

}  // namespace host
}  // namespace lbm

struct lbm_ctx {
  lbm_geom g;
  lbm::host::Layout L;
  void* f[2];
  const uint8_t* mask;
  uint8_t* work;
  hipStream_t stream;
  double tau, rho_in, rho_out;
  int parity;          // f[parity] holds the current state
  int64_t steps;
  int linear_eq;
  int xcd_remap;
  uint64_t n_slots;    // slots in use per direction array (fluid nodes + padding)
  int band;            // 0 or tile rows per band (banded tile order)
  double trt_magic;    // > 0: TRT collision with this magic parameter; 0: BGK
  int wide_offsets;    // 1: 64-bit population offsets even where 32-bit ones fit

  uint64_t* bits() const { return (uint64_t*)(work + L.off_bits); }
  uint32_t* pfx() const { return (uint32_t*)(work + L.off_pfx); }
  lbm::WordDesc* desc() const { return (lbm::WordDesc*)(work + L.off_desc); }   // D2Q9 only
  uint32_t* count() const { return (uint32_t*)(work + L.off_count); }
  uint32_t* scan() const { return (uint32_t*)(work + L.off_scan); }
  uint32_t* seg() const { return (uint32_t*)(work + L.off_seg); }
  uint32_t* seg_scan() const { return (uint32_t*)(work + L.off_seg_scan); }
  void* bplane(int p) const { return work + L.off_bplane + (size_t)p * L.bplane_one * L.esize; }
  double* partial() const { return (double*)(work + L.off_partial); }
  double* scalar() const { return (double*)(work + L.off_scalar); }
  lbm::FluidMap fmap() const {
    lbm::FluidMap m;
    m.bits = bits();
    m.pfx = pfx();
    m.nx = g.nx;
    m.ny = g.ny;
    m.nz = g.nz;
    m.nw = L.nw;
    return m;
  }
};

namespace lbm {
namespace host {

// Every direction group (at most 10 arrays of ps values) spans less than
// 4 GiB: the step kernel can use 32-bit group-relative offsets.
inline bool off32_ok(const lbm_ctx* c) {
  return !c->wide_offsets && 10ull * c->L.ps * c->L.esize < (1ull << 32);
}

// Divisor d >= 1 for FastDiv: l = ceil(log2 d), m = 2^32 (2^l - d) / d + 1.
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d < 1 ? 1 : d;
  f.l = 0;
  while ((1ull << f.l) < f.d) ++f.l;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << f.l) - f.d)) / f.d + 1);
  return f;
}

// Body-force density F = rho0 g along x in the storage precision T, as the
// kernels apply it (0 in the pressure-driven case).
template <class T>
inline T force_density(const lbm_ctx* c) {
  return c->g.boundary == LBM_BC_PERIODIC ? (T)(c->g.rho0 * c->g.body_force) : T(0);
}

template <class T>
StepArgs<T> step_args(const lbm_ctx* c) {
  StepArgs<T> a;
  a.src = (const T*)c->f[c->parity];
  a.dst = (T*)c->f[c->parity ^ 1];
  const int split = c->g.lattice == LBM_D2Q9 ? D2Q9::group_split : D3Q19::group_split;
  a.src_g1 = a.src + (uint64_t)split * c->L.ps;
  a.dst_g1 = a.dst + (uint64_t)split * c->L.ps;
  a.ps_bytes = off32_ok(c) ? (uint32_t)(c->L.ps * sizeof(T)) : 0u;
  a.desc = c->desc();
  a.bits = c->bits();
  a.pfx = c->pfx();
  a.bp_src = (const T*)c->bplane(c->parity);
  a.bp_dst = (T*)c->bplane(c->parity ^ 1);
  a.partial = c->partial();
  a.ps = c->L.ps;
  a.nx = c->g.nx;
  a.ny = c->g.ny;
  a.nz = c->g.nz;
  a.nw = c->L.nw;
  a.seg = c->L.S;
  a.seg_log = c->L.S == 4 ? 2 : (c->L.S == 2 ? 1 : 0);
  a.align = c->L.align;
  a.tiles_x = c->L.segs_per_row;
  const int rows = kRows / c->L.S;
  a.tiles_y = (c->g.ny + rows - 1) / rows;
  a.blocks = a.tiles_x * a.tiles_y * c->g.nz;
  a.xcd_remap = c->xcd_remap;
  // mode >= 2: chunks of (mode - 1) rows of tiles
  a.chunk = c->xcd_remap >= 2 ? (c->xcd_remap - 1) * a.tiles_x : 1;
  a.dv_tiles_x = make_fastdiv((uint32_t)a.tiles_x);
  a.dv_tiles_y = make_fastdiv((uint32_t)a.tiles_y);
  a.dv_chunk = make_fastdiv((uint32_t)a.chunk);
  a.band = c->band;
  a.nbands = a.band > 0 ? (a.tiles_y + a.band - 1) / a.band : 0;
  a.dv_band_blocks = make_fastdiv((uint32_t)(a.band > 0 ? c->g.nz * a.band * a.tiles_x : 1));
  a.dv_band_plane = make_fastdiv((uint32_t)(a.band > 0 ? a.band * a.tiles_x : 1));
  a.fx = force_density<T>(c);
  a.omega = (T)(1.0 / c->tau);
  {
    // TRT: tau- from the magic parameter (tau+ - 1/2)(tau- - 1/2); BGK: tau- = tau
    const double wp = 1.0 / c->tau;
    const double wm = c->trt_magic > 0.0 ? 1.0 / (0.5 + c->trt_magic / (c->tau - 0.5)) : wp;
    a.omega_m = (T)wm;
    a.trt_a = (T)(0.5 * (wp + wm));
    a.trt_b = (T)(0.5 * (wp - wm));
  }
  a.rho0 = (T)c->g.rho0;
  a.drho_in = (T)(c->rho_in - c->g.rho0);
  a.drho_out = (T)(c->rho_out - c->g.rho0);
  return a;
}


inline unsigned grid_1d(uint64_t n) { return (unsigned)((n + 255) / 256); }
// Partials of the flux pass over the slots of c (one per block of 256 slots).
inline unsigned flux_partials(const lbm_ctx* c) { return grid_1d(c->n_slots ? c->n_slots : 1); }
inline uint64_t n_nodes(const lbm_ctx* c) { return (uint64_t)c->g.nx * c->g.ny * c->g.nz; }


// Blocks of one step launch of domain c (whole rounds of 8 in the XCD-aware
// orders, so that block i runs on XCD i mod 8 as the order assumes).
template <class T>
int step_grid(const lbm_ctx* c, const StepArgs<T>& a) {
  if (a.band > 0) return (int)(align_up((size_t)a.nbands, 8) * a.dv_band_blocks.d);
  if (c->xcd_remap == 0) return a.blocks;
  return (int)align_up((size_t)a.blocks, (size_t)(c->xcd_remap == 1 ? 8 : 8 * a.chunk));
}

// The flux pass sums the x-momentum of the stored populations, which holds
// the whole step's force; the momentum of a node is rho u = j - F/2, so the
// pass result is lowered by n_fluid F / (2 nx), with F the force density the
// kernels use (rounded to the storage precision).
inline double flux_pass_offset(const lbm_ctx* c) {
  const double F = c->g.precision == LBM_FP64 ? (double)force_density<double>(c)
                                              : (double)force_density<float>(c);
  return (double)c->L.n_fluid * F / (2.0 * c->g.nx);
}

// Launches the flux pass over the current populations of c; *nparts partials.
lbm_status flux_pass(lbm_ctx* c, int* nparts);
// Reduces c's n flux partials into c's scalar and reads it back (synchronises).
lbm_status reduce_flux(lbm_ctx* c, int n, double* q);
// Flux of the current populations (flux pass + reduction; synchronises).
lbm_status current_flux(lbm_ctx* c, double* q);
// k = nu Q L / (A c_s^2 (rho_in - rho_out)) of domain c.
double perm_from_flux(const lbm_ctx* c, double q);

}  // namespace host
}  // namespace lbm
