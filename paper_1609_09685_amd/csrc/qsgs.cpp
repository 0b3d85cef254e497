// Quartet structure generation set (QSGS) porous masks, 2D and 3D.
//
// The paper's 2D media are "randomly generated quartet structures" (Results,
// the paragraph after Fig. 1); the growth rule is that of Wang, Pan & Chen
// (2007): solid cores are seeded with probability p_core, then every solid
// cell grows into each neighbouring cell with a probability that depends on
// the neighbour class (face / diagonal in 2D; face / edge / vertex in 3D),
// until the solid fraction reaches 1 - porosity.
//
// This file is an input generator: it builds the solid mask that both the GPU
// solver and the CPU checker consume.  It holds none of the lattice Boltzmann
// arithmetic.
//
// Determinism: every random draw is a pure function of (seed, attempt, sweep,
// cell, direction) through the SplitMix64 output function (Steele, Lea & Flood,
// "Fast splittable pseudorandom number generators", OOPSLA 2014), so a mask
// depends only on its arguments, not on thread count or scheduling.
//
// Readings of what the paper leaves open:
//   * growth sweeps are synchronous (a cell grown in sweep s only grows from
//     sweep s+1 on);
//   * the overshoot of the final sweep is removed by reverting the cells grown
//     in that sweep with the largest trim keys, so the porosity is exact
//     (solid count = round((1 - porosity) * N));
//   * a mask must percolate: a fluid path from the inlet column/plane x = 0 to
//     the outlet x = nx-1, 8-connected in 2D and 18-connected in 3D (the links
//     along which D2Q9 / D3Q19 populations move); otherwise the next attempt
//     is drawn.

#include <stdint.h>
#include <string.h>
#include <math.h>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Uniform double in [0, 1) from a 64-bit counter.
inline double u01(uint64_t key) { return (double)(mix64(key) >> 11) * 0x1.0p-53; }

struct Dir { int dx, dy, dz, cls; };  // cls: 0 face, 1 diagonal/edge, 2 vertex

std::vector<Dir> neighbour_dirs(int dim) {
  std::vector<Dir> d;
  for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int n = (dx != 0) + (dy != 0) + (dz != 0);
        if (n == 0) continue;
        d.push_back({dx, dy, dz, n - 1});
      }
  return d;
}

// Counter layout: [stream key of (seed, attempt)] + sweep, cell, direction.
inline uint64_t stream_key(uint64_t seed, int attempt) {
  return mix64(mix64(seed) ^ (0xA5A5000000000000ull + (uint64_t)attempt));
}
inline uint64_t draw_key(uint64_t sk, int sweep, uint64_t cell, int dir) {
  return mix64(sk + (uint64_t)sweep * 0x632BE59BD9B4E019ull) + cell * 32u + (uint64_t)dir;
}

bool percolates(const uint8_t* solid, int dim, int nx, int ny, int nz) {
  const int64_t N = (int64_t)nx * ny * nz;
  std::vector<uint8_t> seen(N, 0);
  std::vector<int64_t> stack;
  // In 2D and 3D the connectivity is that of the lattice's moving directions:
  // faces + diagonals (2D, 8) or faces + edges (3D, 18); corners excluded in 3D.
  std::vector<Dir> dirs;
  for (const Dir& d : neighbour_dirs(dim)) if (d.cls <= 1) dirs.push_back(d);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y) {
      int64_t i = ((int64_t)z * ny + y) * nx;
      if (!solid[i]) { seen[i] = 1; stack.push_back(i); }
    }
  while (!stack.empty()) {
    int64_t i = stack.back(); stack.pop_back();
    int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    if (x == nx - 1) return true;
    for (const Dir& d : dirs) {
      int xx = x + d.dx, yy = y + d.dy, zz = z + d.dz;
      if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) continue;
      int64_t j = ((int64_t)zz * ny + yy) * nx + xx;
      if (!solid[j] && !seen[j]) { seen[j] = 1; stack.push_back(j); }
    }
  }
  return false;
}

// Fluid nodes reachable along lattice links from a fluid node on the x = 0 or
// x = nx - 1 plane (the inlet and outlet): open[i] = 1, else 0 (solid nodes
// and closed pockets, which no steady through-flow can reach).
void open_fluid(const uint8_t* solid, int dim, int nx, int ny, int nz, uint8_t* open) {
  const int64_t N = (int64_t)nx * ny * nz;
  std::fill(open, open + N, (uint8_t)0);
  std::vector<int64_t> stack;
  std::vector<Dir> dirs;
  for (const Dir& d : neighbour_dirs(dim)) if (d.cls <= 1) dirs.push_back(d);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x : {0, nx - 1}) {
        const int64_t i = ((int64_t)z * ny + y) * nx + x;
        if (!solid[i] && !open[i]) { open[i] = 1; stack.push_back(i); }
      }
  while (!stack.empty()) {
    const int64_t i = stack.back();
    stack.pop_back();
    const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    for (const Dir& d : dirs) {
      const int xx = x + d.dx, yy = y + d.dy, zz = z + d.dz;
      if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) continue;
      const int64_t j = ((int64_t)zz * ny + yy) * nx + xx;
      if (!solid[j] && !open[j]) { open[j] = 1; stack.push_back(j); }
    }
  }
}

// One attempt.  Returns 0 on success, -2 if growth stalls before the target.
int grow(int dim, int nx, int ny, int nz, double porosity, const double p[4],
         uint64_t sk, uint8_t* out) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t target = llround((1.0 - porosity) * (double)N);
  std::vector<uint8_t> cur(N), nxt(N);
  std::vector<int32_t> grown_in(N, -1);
  const std::vector<Dir> dirs = neighbour_dirs(dim);
  const int nd = (int)dirs.size();
  double pd[32];
  for (int k = 0; k < nd; ++k) pd[k] = p[1 + dirs[k].cls];

  int64_t count = 0;
#pragma omp parallel for reduction(+ : count) schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    cur[i] = u01(draw_key(sk, 0, (uint64_t)i, 31)) < p[0];
    if (cur[i]) grown_in[i] = 0;
    count += cur[i];
  }
  int sweep = 0;
  while (count < target) {
    ++sweep;
    if (sweep > 100000) return -2;
    int64_t added = 0;
#pragma omp parallel for reduction(+ : added) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      if (cur[i]) { nxt[i] = 1; continue; }
      const int x = (int)(i % nx), y = (int)((i / nx) % ny);
      const int z = (int)(i / ((int64_t)nx * ny));
      uint8_t s = 0;
      for (int k = 0; k < nd && !s; ++k) {
        // growth from the solid neighbour n = i - e_k into i along e_k
        int xx = x - dirs[k].dx, yy = y - dirs[k].dy, zz = z - dirs[k].dz;
        if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) continue;
        int64_t j = ((int64_t)zz * ny + yy) * nx + xx;
        if (cur[j] && u01(draw_key(sk, sweep, (uint64_t)i, k)) < pd[k]) s = 1;
      }
      nxt[i] = s;
      if (s) { grown_in[i] = sweep; ++added; }
    }
    if (added == 0 && sweep > 64) {
      // Growth probabilities too small to ever reach the target.
      bool any_p = false;
      for (int k = 0; k < nd; ++k) any_p |= pd[k] > 0;
      if (!any_p) return -2;
    }
    cur.swap(nxt);
    count += added;
  }
  // Remove the overshoot among the cells grown in the final sweep.
  int64_t excess = count - target;
  if (excess > 0) {
    std::vector<std::pair<uint64_t, int64_t>> cand;
    for (int64_t i = 0; i < N; ++i)
      if (cur[i] && grown_in[i] == sweep) cand.push_back({mix64(draw_key(sk, 1 << 20, (uint64_t)i, 0)), i});
    std::nth_element(cand.begin(), cand.begin() + (cand.size() - excess), cand.end());
    for (size_t r = cand.size() - excess; r < cand.size(); ++r) cur[cand[r].second] = 0;
  }
  memcpy(out, cur.data(), (size_t)N);
  return 0;
}

}  // namespace

extern "C" {

// Generates a solid mask (1 = solid, 0 = fluid), laid out [nz][ny][nx] with x
// fastest.  dim is 2 (then nz must be 1) or 3.  probs = {p_core, p_face,
// p_diag_or_edge, p_vertex}; p_vertex is ignored in 2D.  With
// require_percolation != 0 attempts are drawn until one percolates in x, at
// most max_attempts.  Returns 0 on success, -1 on invalid arguments, -2 if the
// growth cannot reach the porosity, -3 if no attempt percolated.
int qsgs_generate(int dim, int nx, int ny, int nz, double porosity, const double* probs,
                  uint64_t seed, int require_percolation, int max_attempts,
                  uint8_t* out_mask, int* attempts_used) {
  if (!out_mask || !probs || (dim != 2 && dim != 3) || nx < 1 || ny < 1 || nz < 1) return -1;
  if (dim == 2 && nz != 1) return -1;
  if (!(porosity >= 0.0 && porosity <= 1.0) || max_attempts < 1) return -1;
  for (int a = 0; a < max_attempts; ++a) {
    int rc = grow(dim, nx, ny, nz, porosity, probs, stream_key(seed, a), out_mask);
    if (rc) return rc;
    if (!require_percolation || percolates(out_mask, dim, nx, ny, nz)) {
      if (attempts_used) *attempts_used = a + 1;
      return 0;
    }
  }
  return -3;
}

// 1 if the fluid phase connects x = 0 to x = nx-1 (8-connected in 2D,
// 18-connected in 3D), else 0.
int qsgs_percolates(int dim, int nx, int ny, int nz, const uint8_t* mask) {
  return percolates(mask, dim, nx, ny, nz) ? 1 : 0;
}

// open[i] = 1 for fluid nodes connected to the inlet or outlet plane (see
// open_fluid), 0 otherwise.  Returns 0, or -1 on bad arguments.
int qsgs_open_fluid(int dim, int nx, int ny, int nz, const uint8_t* mask, uint8_t* open) {
  if ((dim != 2 && dim != 3) || nx < 1 || ny < 1 || nz < 1 || !mask || !open) return -1;
  open_fluid(mask, dim, nx, ny, nz, open);
  return 0;
}

int qsgs_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
