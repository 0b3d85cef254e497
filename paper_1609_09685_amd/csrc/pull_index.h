// Index arithmetic of the step kernel's pull: where the population of each
// direction that arrives at a fluid node comes from, in the compact
// fluid-only slot layout.  Written once for the device (one wavefront = 64
// consecutive x of one row, the row data wave-uniform) and for the host (one
// lane at a time), so that a CPU check can run exactly this code over every
// node of a mask and compare it with a direct application of the boundary
// rules.  No HIP headers: the host build is plain C++.
//
// Layout recap.  Per (y, z) row, 64-bit words hold the fluid bits of x = 64 w
// .. 64 w + 63.  Fluid nodes get slots in x-fastest order; a row is cut into
// segments of S words whose first slot sits on a 128-byte boundary, the slots
// between the last fluid node of a segment and the next segment's first slot
// being zero padding.  The step kernel forms one record per word (WordDesc)
// from the bitmap words and the slots of the words' first fluid nodes: the
// slot of the word's first fluid node, the word's fluid bits, and what a
// wavefront needs about the words on either side (whether node 64 w - 1 /
// 64 w + 64 is fluid, and the padding between the words).
//
// Pull rules for direction i at a fluid node x (the readings of the paper's
// boundary conditions): the source is x - c_i; (1) a source row outside the
// lattice in y or z is mirrored onto the node's own row (symmetric plane) and
// the mirrored direction is read, or, with periodic faces, wraps to the
// opposite face; (2) a solid source means halfway bounce-back: the node's own
// slot of the opposite direction is read; (3) a source at x = -1 or x = nx is a
// pressure ghost: the edge node b of the source row is read (and a
// non-equilibrium term added by the caller), or, with periodic faces, the
// node across the x faces; a ghost copies b's solidity; (4) otherwise plain
// streaming from the source slot.
#pragma once

#include <stdint.h>

#if defined(__HIP__) || defined(__HIPCC__)
#define LBM_HD __host__ __device__ __forceinline__
#else
#define LBM_HD inline
#endif

namespace lbm {

// One word of one row, as the step kernel sees it.
struct WordDesc {
  uint32_t base;   // slot of the first fluid node at or after x = 64 w (next slot if none)
  uint32_t lo;     // fluid bits of x = 64 w .. 64 w + 31
  uint32_t hi;     // fluid bits of x = 64 w + 32 .. 64 w + 63
  uint32_t info;   // kPrevFluid | kNextFluid | gap before << 8 | gap after << 16
};

constexpr uint32_t kPrevFluid = 1u;   // node 64 w - 1 exists and is fluid
constexpr uint32_t kNextFluid = 2u;   // node 64 w + 64 exists and is fluid

LBM_HD uint32_t popc64(uint64_t m) {
#if defined(__HIP_DEVICE_COMPILE__)
  return (uint32_t)__popcll(m);
#else
  return (uint32_t)__builtin_popcountll(m);
#endif
}

LBM_HD uint64_t desc_bits(const WordDesc& d) { return (uint64_t)d.hi << 32 | d.lo; }
// padding slots between the end of word w - 1 and the first slot of word w
LBM_HD uint32_t gap_before(uint32_t info) { return (info >> 8) & 0xffu; }
// padding slots between the end of word w and the first slot of word w + 1
LBM_HD uint32_t gap_after(uint32_t info) { return (info >> 16) & 0xffu; }

// Record of word w from the bitmap words of w - 1, w, w + 1 (zero where they do
// not exist) and the first slots of the three words (pfx_prev / pfx_next are
// ignored where the words do not exist).  Padding only ever lies between two
// words of a row, never inside one, and is less than 128 bytes of slots.
LBM_HD WordDesc make_word_desc(uint64_t lo, uint64_t mid, uint64_t hi, uint32_t pfx_prev,
                               uint32_t pfx, uint32_t pfx_next, bool has_prev, bool has_next) {
  WordDesc d;
  d.base = pfx;
  d.lo = (uint32_t)mid;
  d.hi = (uint32_t)(mid >> 32);
  uint32_t info = 0;
  if (has_prev && (lo >> 63)) info |= kPrevFluid;
  if (has_next && (hi & 1ull)) info |= kNextFluid;
  if (has_prev) info |= (pfx - (pfx_prev + popc64(lo))) << 8;
  if (has_next) info |= (pfx_next - (pfx + popc64(mid))) << 16;
  d.info = info;
  return d;
}

// First slot and fluid count of the segment whose first and last words have
// the records d0 and d1 (slots run on without gaps inside a segment).
LBM_HD void segment_extent(const WordDesc& d0, const WordDesc& d1, uint32_t& first,
                           uint32_t& count) {
  first = d0.base;
  count = d1.base + popc64(desc_bits(d1)) - d0.base;
}

// Per-lane primitives over wave-uniform 64-bit masks.  On the device a
// wavefront evaluates them for its 64 lanes at once (v_mbcnt, a select on the
// mask as a lane condition, v_writelane); on the host one lane is evaluated.
#if defined(__HIP__)
struct WaveLane {
  // base + number of set bits of m below the lane
  __device__ __forceinline__ uint32_t rank(uint64_t m, uint32_t base) const {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, base));
#else
    return base + (uint32_t)(m & 0u);
#endif
  }
  // bit `lane` of m
  __device__ __forceinline__ bool bit(uint64_t m) const {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_inverse_ballot_w64(m);
#else
    return m != 0;
#endif
  }
  // v with lane L replaced by the wave-uniform s (one v_writelane)
  template <int L>
  __device__ __forceinline__ uint32_t set_lane(uint32_t v, uint32_t s) const {
#if defined(__HIP_DEVICE_COMPILE__)
    // s is wave-uniform by construction; readfirstlane only tells the compiler
    // so where its analysis cannot (it folds away when s sits in a scalar register)
    const uint32_t su = (uint32_t)__builtin_amdgcn_readfirstlane((int)s);
    uint32_t r;
    asm("v_writelane_b32 %0, %1, %2" : "=v"(r) : "s"(su), "n"(L), "0"(v));
    return r;
#else
    return s + (v & 0u);
#endif
  }
  // v with lane l (wave-uniform) replaced by the wave-uniform s
  __device__ __forceinline__ uint32_t set_lane_at(uint32_t v, uint32_t s, int l) const {
    return bit(1ull << l) ? s : v;
  }
};
#endif

struct HostLane {
  int lane;
  uint32_t rank(uint64_t m, uint32_t base) const {
    return base + (uint32_t)__builtin_popcountll(lane ? m & ((1ull << lane) - 1ull) : 0ull);
  }
  bool bit(uint64_t m) const { return (m >> lane) & 1ull; }
  template <int L>
  uint32_t set_lane(uint32_t v, uint32_t s) const { return lane == L ? s : v; }
  uint32_t set_lane_at(uint32_t v, uint32_t s, int l) const { return lane == l ? s : v; }
};

// Wave-uniform description of one source row around the wave's word: its
// fluid bits, first slot and record flags, and (periodic x faces only) node
// nx - 1 and node 0 of the row.
struct SourceRow {
  uint64_t mid;
  uint32_t base, info;
  uint32_t last_fluid, last_slot, first_fluid, first_slot;
};

// Edge flags of the wave's word (wave-uniform).
struct WordEdges {
  bool x0;        // the word holds x = 0 (lane 0)
  bool x1;        // the word holds x = nx - 1 (lane e)
  int e;          // (nx - 1) & 63
};

// Source of the population with x-velocity CX that a lane pulls from row r
// (after the y / z mirror or wrap).  Out: m, the lanes whose source is a fluid
// node (wave-uniform); off = E * (source slot) + dk, valid in the lanes of m
// (E = bytes per value, dk a wave-uniform byte offset); gm, the lanes whose
// source is a pressure ghost (the caller adds the non-equilibrium term).
// cnt = the number of fluid nodes of row r's word below the lane,
// rank(r.mid, 0) (the slot of the lane's own node is r.base + cnt); the
// wave-uniform parts of an offset are formed apart from it.  PER: periodic x
// faces, else pressure ghosts.  Within a segment slots run on across words, so the
// neighbours of lanes 0 and 63 follow from the lane ranks unless padding lies
// between the words (gap_before / gap_after): those two lanes are set from the
// record.
template <int CX, bool PER, uint32_t E, class Lane>
LBM_HD void pull_offset(const Lane& ln, const SourceRow& r, uint32_t cnt, const WordEdges& we,
                        uint32_t dk, uint64_t& m, uint32_t& off, uint64_t& gm) {
  gm = 0;
  const uint32_t ub = r.base * E + dk;   // wave-uniform: offset of the word's first slot
  if (CX == 0) {
    m = r.mid;
    off = cnt * E + ub;
  } else if (CX > 0) {   // source x - 1; lane 0 reads node 64 w - 1 of the previous word
    m = (r.mid << 1) | (uint64_t)(r.info & kPrevFluid);
    uint32_t s0 = r.base - gap_before(r.info) - 1u;
    if (we.x0) {          // lane 0 is x = 0: the source is across the inlet face
      if (PER) {
        m = (m & ~1ull) | (uint64_t)r.last_fluid;
        s0 = r.last_slot;
      } else {            // ghost at x = -1: edge node b = (0, ys, zs) of this row
        m = (m & ~1ull) | (r.mid & 1ull);
        s0 = r.base;
        gm = r.mid & 1ull;
      }
    }
    off = ln.template set_lane<0>(cnt * E + (ub - E), s0 * E + dk);
  } else {               // source x + 1; lane 63 reads node 64 w + 64 of the next word
    m = (r.mid >> 1) | ((uint64_t)((r.info & kNextFluid) != 0u) << 63);
    const uint32_t s63 = r.base + popc64(r.mid) + gap_after(r.info);
    off = ln.template set_lane<63>((cnt + (uint32_t)ln.bit(r.mid)) * E + ub, s63 * E + dk);
    if (we.x1) {          // lane e is x = nx - 1: the source is across the outlet face
      const uint64_t eb = 1ull << we.e;
      if (PER) {
        m = (m & ~eb) | ((uint64_t)r.first_fluid << we.e);
        off = ln.set_lane_at(off, r.first_slot * E + dk, we.e);
      } else {            // ghost at x = nx: edge node b = (nx - 1, ys, zs) of this row
        m = (m & ~eb) | (r.mid & eb);
        off = ln.bit(eb) ? cnt * E + ub : off;
        gm = r.mid & eb;
      }
    }
  }
}

// Node nx - 1 and node 0 of a row from the records of its last and first
// words (periodic x faces).
LBM_HD void row_x_faces(const WordDesc& first, const WordDesc& last, int nx, SourceRow& r) {
  const int bl = (nx - 1) & 63;
  const uint64_t wl = desc_bits(last);
  r.last_fluid = (uint32_t)((wl >> bl) & 1ull);
  r.last_slot = last.base + popc64(bl ? wl & ((1ull << bl) - 1ull) : 0ull);
  r.first_fluid = first.lo & 1u;
  r.first_slot = first.base;
}

}  // namespace lbm
