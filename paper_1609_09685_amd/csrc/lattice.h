// Lattice velocity sets of the solver: D2Q9 and D3Q19 (Qian, d'Humieres &
// Lallemand 1992), the two lattices the paper uses for its 2D and 3D cases.
//
// Direction order (this library's own, and also the order of the population
// arrays in memory): the rest direction first, then the moving directions in
// opposite pairs, (1, 2), (3, 4), ...: opp(i) = i + 1 for odd i, i - 1 for even
// i > 0.  The arrays form groups of at most 10 that are closed under opp, my
// and mz (D3Q19: the in-plane directions 0..8, and 9..18), so everything one
// node loads for one direction (streaming, mirrored, or bounce-back) lies in
// one group, which lets the kernel address a group with 32-bit offsets.  The
// first nine D3Q19 directions are the D2Q9 set.
//
//   opp(i): c_opp = -c_i        (halfway bounce-back)
//   my(i):  c_y flipped          (symmetric plane normal to y)
//   mz(i):  c_z flipped          (symmetric plane normal to z)
//
// Weights: D2Q9 4/9, 1/9 (axis), 1/36 (diagonal); D3Q19 1/3, 1/18 (axis),
// 1/36 (edge).  c_s^2 = 1/3.  The static_asserts at the end check every table
// against the velocity vectors at compile time.
#pragma once

namespace lbm {

struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int D = 2;
  static constexpr int cx[Q] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
  static constexpr int cy[Q] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
  static constexpr int cz[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr double w[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
  static constexpr int my[Q] = {0, 1, 2, 4, 3, 7, 8, 5, 6};
  static constexpr int mz[Q] = {0, 1, 2, 3, 4, 5, 6, 7, 8};
  static constexpr int group_split = 9;   // one group
};

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int D = 3;
  static constexpr int cx[Q] = {0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[Q] = {0, 0, 0, 1, -1, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr double w[Q] = {
      1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36,
      1.0 / 36, 1.0 / 36, 1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  static constexpr int my[Q] = {0, 1, 2, 4, 3, 7, 8, 5, 6, 9, 10, 11, 12, 13, 14, 18, 17, 16, 15};
  static constexpr int mz[Q] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 10, 9, 13, 14, 11, 12, 17, 18, 15, 16};
  static constexpr int group_split = 9;   // groups [0, 9) and [9, 19)
};

namespace detail {

template <class L>
constexpr int find(int x, int y, int z) {
  for (int i = 0; i < L::Q; ++i)
    if (L::cx[i] == x && L::cy[i] == y && L::cz[i] == z) return i;
  return -1;
}

template <class L>
constexpr bool tables_consistent() {
  double wsum = 0;
  if (L::cx[0] != 0 || L::cy[0] != 0 || L::cz[0] != 0) return false;
  for (int i = 0; i < L::Q; ++i) {
    if (L::opp[i] != find<L>(-L::cx[i], -L::cy[i], -L::cz[i])) return false;
    if (L::my[i] != find<L>(L::cx[i], -L::cy[i], L::cz[i])) return false;
    if (L::mz[i] != find<L>(L::cx[i], L::cy[i], -L::cz[i])) return false;
    if (find<L>(L::cx[i], L::cy[i], L::cz[i]) != i) return false;  // distinct vectors
    if (i > 0 && L::opp[i] != (i % 2 ? i + 1 : i - 1)) return false;  // adjacent pairs
    const bool g = i < L::group_split;   // groups closed under opp, my, mz
    if (g != (L::opp[i] < L::group_split) || g != (L::my[i] < L::group_split) ||
        g != (L::mz[i] < L::group_split))
      return false;
    if (L::Q - L::group_split > 10 || L::group_split > 10) return false;
    wsum += L::w[i];
  }
  return wsum > 1.0 - 1e-15 && wsum < 1.0 + 1e-15;
}

template <class L>
constexpr bool second_moment_isotropic() {
  // sum_i w_i c_ia c_ib = delta_ab / 3 over the lattice's D dimensions
  for (int a = 0; a < L::D; ++a)
    for (int b = 0; b < L::D; ++b) {
      double s = 0;
      for (int i = 0; i < L::Q; ++i) {
        const int ca = a == 0 ? L::cx[i] : (a == 1 ? L::cy[i] : L::cz[i]);
        const int cb = b == 0 ? L::cx[i] : (b == 1 ? L::cy[i] : L::cz[i]);
        s += L::w[i] * ca * cb;
      }
      const double e = a == b ? 1.0 / 3.0 : 0.0;
      if (s - e > 1e-15 || e - s > 1e-15) return false;
    }
  return true;
}

}  // namespace detail

static_assert(detail::tables_consistent<D2Q9>(), "D2Q9 tables");
static_assert(detail::tables_consistent<D3Q19>(), "D3Q19 tables");
static_assert(detail::second_moment_isotropic<D2Q9>(), "D2Q9 weights");
static_assert(detail::second_moment_isotropic<D3Q19>(), "D3Q19 weights");

}  // namespace lbm
