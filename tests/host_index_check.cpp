// CPU check of the step kernel's index arithmetic (test infrastructure).
//
// Runs, for every node of a mask, the very functions the GPU step kernel uses
// to find its pull sources and its segment stores (pull_index.h: the per-word
// records, pull_offset, segment_extent), one lane at a time, and compares them
// with a direct application of the boundary rules to an independently built
// slot map:
//   source x - c_i; a row outside [0, ny) / [0, nz) is mirrored onto the own
//   row with the mirrored direction (pressure case) or wraps (periodic case);
//   a solid source bounces back (own slot, opposite direction); a source at
//   x = -1 / nx is the pressure ghost of the edge node of the source row
//   (bounce-back if that node is solid), or wraps (periodic case).
// Also checks that every slot read or written lies inside the population
// arrays, that the block stores write every slot exactly once in whole
// 128-byte lines (padding as zero), that padding slots are never read, and
// that a block's LDS staging index stays inside its 256 positions.
//
// Build: g++ -std=c++17 -I<package>/csrc, as a program (LBM_CHECK_MAIN, reads
// the cases from stdin; built with ASan/UBSan by the tests) or a library.
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <type_traits>
#include <vector>

#include "lattice.h"
#include "pull_index.h"

namespace {

template <int I, int N, class F>
void unroll_h(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    unroll_h<I + 1, N>(f);
  }
}

struct Checker {
  int Q, nx, ny, nz, E;
  bool per;
  const uint8_t* mask;   // [nz][ny][nx], 1 = solid
  uint64_t ps;           // slots per direction array (capacity)
  int nw, S, align;
  std::vector<uint64_t> bits;        // [row][nw]
  std::vector<uint32_t> pfx;         // [row][nw]
  std::vector<int64_t> slot;         // [node] or -1
  std::vector<lbm::WordDesc> desc;   // [row][nw]
  std::vector<uint8_t> is_padding;   // [slot]
  char* msg;
  int msglen;
  long errors = 0;
  long checked = 0;

  void report(const char* fmt, ...) __attribute__((format(printf, 2, 3))) {
    if (errors++ == 0 && msg) {
      va_list ap;
      va_start(ap, fmt);
      vsnprintf(msg, msglen, fmt, ap);
      va_end(ap);
    }
  }

  bool fluid(int x, int y, int z) const { return mask[((size_t)z * ny + y) * nx + x] == 0; }

  // The slot layout, built directly: fluid nodes in x-fastest order, every
  // segment of S words of a row starting on a 128-byte boundary.
  bool build_layout() {
    nw = (nx + 63) / 64;
    S = nw >= 4 ? 4 : (nw >= 2 ? 2 : 1);
    align = 128 / E;
    const size_t rows = (size_t)ny * nz;
    bits.assign(rows * nw, 0);
    pfx.assign(rows * nw, 0);
    slot.assign((size_t)nx * ny * nz, -1);
    uint64_t next = 0;
    for (size_t row = 0; row < rows; ++row) {
      const int y = (int)(row % ny), z = (int)(row / ny);
      for (int w = 0; w < nw; ++w) {
        if (w % S == 0) next = (next + align - 1) / align * align;
        pfx[row * nw + w] = (uint32_t)next;
        for (int p = 0; p < 64; ++p) {
          const int x = 64 * w + p;
          if (x < nx && fluid(x, y, z)) {
            bits[row * nw + w] |= 1ull << p;
            slot[row * nx + x] = (int64_t)next++;
          }
        }
      }
    }
    const uint64_t used = (next + align - 1) / align * align;
    if (used > ps) {
      report("capacity: slots used %ld > capacity %ld", (long)used, (long)ps);
      return false;
    }
    is_padding.assign(ps, 1);
    for (int64_t s : slot)
      if (s >= 0) is_padding[s] = 0;
    desc.resize(rows * nw);
    for (size_t row = 0; row < rows; ++row)
      for (int w = 0; w < nw; ++w) {
        const size_t i = row * nw + w;
        const bool hp = w > 0, hn = w + 1 < nw;
        desc[i] = lbm::make_word_desc(hp ? bits[i - 1] : 0ull, bits[i], hn ? bits[i + 1] : 0ull,
                                      hp ? pfx[i - 1] : 0u, pfx[i], hn ? pfx[i + 1] : 0u, hp, hn);
      }
    return true;
  }

  // What node_update loads for one lane and direction, through pull_offset.
  template <class L, int q>
  void check_direction(int x, int y, int z, int w, int lane, uint32_t self, uint32_t dk_test) {
    constexpr int cx = L::cx[q], cy = L::cy[q], cz = L::cz[q];
    // source row exactly as the kernel forms it
    int ey = -cy, ez = -cz;
    bool fy = false, fz = false;
    if (per) {
      if (ey < 0 && y == 0) ey = ny - 1;
      if (ey > 0 && y == ny - 1) ey = 1 - ny;
      if (ez < 0 && z == 0) ez = nz - 1;
      if (ez > 0 && z == nz - 1) ez = 1 - nz;
    } else {
      if ((ey < 0 && y == 0) || (ey > 0 && y == ny - 1)) { ey = 0; fy = true; }
      if (L::D == 3 && ((ez < 0 && z == 0) || (ez > 0 && z == nz - 1))) { ez = 0; fz = true; }
    }
    const size_t srow = (size_t)(z + ez) * ny + (y + ey);
    const lbm::WordDesc& d = desc[srow * nw + w];
    lbm::SourceRow r;
    r.mid = lbm::desc_bits(d);
    r.base = d.base;
    r.info = d.info;
    r.last_fluid = r.last_slot = r.first_fluid = r.first_slot = 0;
    if (per) lbm::row_x_faces(desc[srow * nw], desc[srow * nw + nw - 1], nx, r);
    lbm::WordEdges we;
    we.x0 = w == 0;
    we.x1 = w == (nx - 1) / 64;
    we.e = (nx - 1) & 63;
    const lbm::HostLane ln{lane};
    uint64_t m = 0, gm = 0;
    uint32_t off = 0;
    const uint32_t cnt = ln.rank(r.mid, 0u);
    if (per) lbm::pull_offset<cx, true, 1u>(ln, r, cnt, we, dk_test, m, off, gm);
    else lbm::pull_offset<cx, false, 1u>(ln, r, cnt, we, dk_test, m, off, gm);
    int k = q;
    {
      const int kY = L::my[q], kZ = L::mz[q], kYZ = L::mz[L::my[q]];
      k = fy ? (fz ? kYZ : kY) : (fz ? kZ : q);
    }
    const bool got_fluid = ln.bit(m), got_ghost = ln.bit(gm);
    const int64_t got_slot = got_fluid ? (int64_t)(uint32_t)(off - dk_test) : (int64_t)self;
    const int got_dir = got_fluid ? k : L::opp[q];

    // the rules, applied directly
    int xs = x - cx, ys = y - cy, zs = z - cz, kk = q;
    bool ghost = false;
    if (per) {
      xs = (xs + nx) % nx;
      ys = (ys + ny) % ny;
      zs = (zs + nz) % nz;
    } else {
      bool my = false, mz = false;
      if (ys < 0 || ys >= ny) { ys = y; my = true; }
      if (L::D == 3 && (zs < 0 || zs >= nz)) { zs = z; mz = true; }
      kk = my ? (mz ? L::mz[L::my[q]] : L::my[q]) : (mz ? L::mz[q] : q);
      if (xs < 0 || xs >= nx) {
        xs = xs < 0 ? 0 : nx - 1;
        ghost = true;
      }
    }
    int64_t want_slot;
    int want_dir;
    bool want_ghost = false;
    if (fluid(xs, ys, zs)) {
      want_slot = slot[((size_t)zs * ny + ys) * nx + xs];
      want_dir = kk;
      want_ghost = ghost;
    } else {
      want_slot = self;
      want_dir = L::opp[q];
    }
    ++checked;
    if (got_slot != want_slot || got_dir != want_dir || got_ghost != want_ghost)
      report("node (%d,%d,%d) direction %d: slot %ld, expected %ld", x, y, z, q, (long)got_slot,
             (long)want_slot);
    if (got_slot < 0 || (uint64_t)got_slot >= ps)
      report("node (%d,%d,%d) direction %d: slot %ld outside the arrays (%ld)", x, y, z, q,
             (long)got_slot, (long)ps);
    else if (is_padding[got_slot])
      report("node (%d,%d,%d) direction %d: reads padding slot %ld", x, y, z, q, (long)got_slot);
  }

  template <class L>
  void check_node(int x, int y, int z, int w, int lane, uint32_t self, uint32_t dk) {
    unroll_h<1, L::Q>([&](auto qc) {
      check_direction<L, decltype(qc)::value>(x, y, z, w, lane, self, dk);
    });
  }

  // Gathers of every fluid node, and the rank of the node's own slot.
  template <class L>
  void check_pulls(uint32_t dk) {
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y) {
        const size_t row = (size_t)z * ny + y;
        for (int w = 0; w < nw; ++w) {
          const lbm::WordDesc& d = desc[row * nw + w];
          for (int lane = 0; lane < 64; ++lane) {
            const int x = 64 * w + lane;
            const lbm::HostLane ln{lane};
            const bool f = ln.bit(lbm::desc_bits(d));
            if (x >= nx) {
              if (f) report("row %d %d word %d lane %d: fluid bit past nx", y, z, w, lane);
              continue;
            }
            if (f != fluid(x, y, z))
              report("node (%d,%d,%d) word %d: fluid bit %d", x, y, z, w, (int)f);
            if (!f) continue;
            const uint32_t self = d.base + ln.rank(lbm::desc_bits(d), 0u);
            if ((int64_t)self != slot[row * nx + x])
              report("node (%d,%d,%d) word %d: own slot %ld, expected %ld", x, y, z, w, (long)self,
                     (long)slot[row * nx + x]);
            check_node<L>(x, y, z, w, lane, self, dk);
          }
        }
      }
  }

  // The store phase: a block covers one segment of each of 4 / S rows; the
  // segment's first slot and fluid count come from segment_extent, thread t
  // writes position r = t mod (64 S) of its row's segment (LDS position t) up
  // to the next 128-byte boundary.  Every slot must be written exactly once,
  // fluid slots by the position that holds their node, padding as zero.
  void check_stores() {
    const int segs = (nw + S - 1) / S;
    std::vector<uint8_t> written(ps, 0);
    for (size_t row = 0; row < (size_t)ny * nz; ++row)
      for (int sg = 0; sg < segs; ++sg) {
        const int w0 = sg * S, w1 = (w0 + S < nw ? w0 + S : nw) - 1;
        uint32_t first, count;
        lbm::segment_extent(desc[row * nw + w0], desc[row * nw + w1], first, count);
        uint32_t want = 0;
        for (int w = w0; w <= w1; ++w) want += (uint32_t)__builtin_popcountll(bits[row * nw + w]);
        const uint32_t lim = (count + align - 1) & ~(uint32_t)(align - 1);
        if (count != want)
          report("row %d segment %d: count %d, expected %d", (int)row, sg, (int)count, (int)want);
        if (first % align)
          report("row %d segment %d: first slot %d not on a 128-byte boundary", (int)row, sg,
                 (int)first);
        if (lim > (uint32_t)(64 * S))
          report("row %d segment %d: %d stores exceed the block's %d positions", (int)row, sg,
                 (int)lim, 64 * S);
        for (uint32_t r = 0; r < lim; ++r) {
          const uint64_t s = (uint64_t)first + r;
          if (s >= ps) {
            report("row %d segment %d: store slot %ld outside the arrays (%ld)", (int)row, sg,
                   (long)s, (long)ps);
            break;
          }
          if (written[s]++) report("row %d segment %d: slot %ld written twice", (int)row, sg, (long)s);
          if ((r < count) == (bool)is_padding[s])
            report("row %d segment %d: position %d live=%d but padding=%d", (int)row, sg, (int)r,
                   (int)(r < count), (int)is_padding[s]);
        }
        // the staging position of the segment's fluid node is its slot minus
        // first: it must stay below the segment's fluid count
        for (int w = w0; w <= w1; ++w) {
          const lbm::WordDesc& d = desc[row * nw + w];
          const uint64_t m = lbm::desc_bits(d);
          for (int lane = 0; lane < 64; ++lane)
            if ((m >> lane) & 1ull) {
              const uint32_t self = d.base + lbm::HostLane{lane}.rank(m, 0u);
              if (self - first >= count)
                report("row %d word %d lane %d: LDS position %d past the segment (%d)", (int)row, w,
                       lane, (int)(self - first), (int)count);
            }
        }
      }
    for (uint64_t sl = 0; sl < ps; ++sl)
      if (!written[sl] && !is_padding[sl]) report("fluid slot %lu never written", (unsigned long)sl);
  }
};

}  // namespace

extern "C" {

// Returns the number of mismatches (0: all checks passed); msg gets the first.
// checked_out (may be NULL): number of (node, direction) pairs compared.
long lbm_check_pull_index(int Q, const uint8_t* mask, int nx, int ny, int nz, int esize,
                          int periodic, uint64_t ps, char* msg, int msglen, long* checked_out) {
  if (msg && msglen > 0) msg[0] = 0;
  Checker c;
  c.Q = Q;
  c.nx = nx;
  c.ny = ny;
  c.nz = nz;
  c.E = esize;
  c.per = periodic != 0;
  c.mask = mask;
  c.ps = ps;
  c.msg = msg;
  c.msglen = msglen;
  if (!c.build_layout()) return c.errors;
  // the uniform byte offset of the kernel (direction distance) must cancel out
  for (uint32_t dk : {0u, 0x12345u}) {
    if (Q == 9) c.check_pulls<lbm::D2Q9>(dk);
    else c.check_pulls<lbm::D3Q19>(dk);
  }
  c.check_stores();
  if (checked_out) *checked_out = c.checked;
  return c.errors;
}

}  // extern "C"

#ifdef LBM_CHECK_MAIN
#include <stdlib.h>

// stdin: cases "Q nx ny nz esize periodic ps\n" each followed by nx*ny*nz mask
// bytes.  stdout: one line per case, "case <i> errors <n> checked <m> <first>".
int main() {
  int Q, nx, ny, nz, esize, periodic;
  unsigned long long ps;
  long total = 0;
  for (int i = 0; scanf("%d %d %d %d %d %d %llu", &Q, &nx, &ny, &nz, &esize, &periodic, &ps) == 7; ++i) {
    getchar();   // the newline
    const size_t n = (size_t)nx * ny * nz;
    std::vector<uint8_t> mask(n);
    if (fread(mask.data(), 1, n, stdin) != n) return 2;
    char msg[256];
    long checked = 0;
    const long e = lbm_check_pull_index(Q, mask.data(), nx, ny, nz, esize, periodic, ps, msg,
                                        (int)sizeof msg, &checked);
    printf("case %d errors %ld checked %ld %s\n", i, e, checked, msg);
    total += e;
  }
  return total ? 1 : 0;
}
#endif
