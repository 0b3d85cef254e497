// Lattice velocity sets of the solver: D2Q9 and D3Q19 (Qian, d'Humieres &
// Lallemand 1992), the two lattices the paper uses for its 2D and 3D cases.
//
// Direction order (this library's own): the rest direction, then the
// directions moving towards +x, then those moving towards -x, then those with
// no x component.  Grouping by the x component keeps the inlet/outlet ghost
// logic to compile-time ranges.
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
  static constexpr int cx[Q] = {0, 1, 1, 1, -1, -1, -1, 0, 0};
  static constexpr int cy[Q] = {0, 0, 1, -1, 0, 1, -1, 1, -1};
  static constexpr int cz[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr double w[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 9, 1.0 / 9};
  static constexpr int opp[Q] = {0, 4, 6, 5, 1, 3, 2, 8, 7};
  static constexpr int my[Q] = {0, 1, 3, 2, 4, 6, 5, 8, 7};
  static constexpr int mz[Q] = {0, 1, 2, 3, 4, 5, 6, 7, 8};
  // directions with c_x = +1 are [xp_begin, xp_end), c_x = -1 [xm_begin, xm_end)
  static constexpr int xp_begin = 1, xp_end = 4, xm_begin = 4, xm_end = 7;
};

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int D = 3;
  static constexpr int cx[Q] = {0, 1, 1, 1, 1, 1, -1, -1, -1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int cy[Q] = {0, 0, 1, -1, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[Q] = {0, 0, 0, 0, 1, -1, 0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1};
  static constexpr double w[Q] = {
      1.0 / 3,  1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 18,
      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 18, 1.0 / 18, 1.0 / 18,
      1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr int opp[Q] = {0, 6, 8, 7, 10, 9, 1, 3, 2, 5, 4, 12, 11, 14, 13, 16, 15, 18, 17};
  static constexpr int my[Q] = {0, 1, 3, 2, 4, 5, 6, 8, 7, 9, 10, 12, 11, 13, 14, 18, 17, 16, 15};
  static constexpr int mz[Q] = {0, 1, 2, 3, 5, 4, 6, 7, 8, 10, 9, 11, 12, 14, 13, 17, 18, 15, 16};
  static constexpr int xp_begin = 1, xp_end = 6, xm_begin = 6, xm_end = 11;
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
  for (int i = 0; i < L::Q; ++i) {
    if (L::opp[i] != find<L>(-L::cx[i], -L::cy[i], -L::cz[i])) return false;
    if (L::my[i] != find<L>(L::cx[i], -L::cy[i], L::cz[i])) return false;
    if (L::mz[i] != find<L>(L::cx[i], L::cy[i], -L::cz[i])) return false;
    int n = (L::cx[i] != 0) + (L::cy[i] != 0) + (L::cz[i] != 0);
    if (find<L>(L::cx[i], L::cy[i], L::cz[i]) != i) return false;  // distinct vectors
    if (i >= L::xp_begin && i < L::xp_end && L::cx[i] != 1) return false;
    if (i >= L::xm_begin && i < L::xm_end && L::cx[i] != -1) return false;
    if ((i < L::xp_begin || i >= L::xm_end) && L::cx[i] != 0) return false;
    (void)n;
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
