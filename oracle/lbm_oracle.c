/*
 * Plain FP64 CPU oracle of the lattice Boltzmann permeability computation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the GPU solver is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it; the solver never
 * does, and it shares no code, header or table with the solver.
 *
 * What it computes (Li, Ho, Wu & Zhang, "Lattice Boltzmann modelling of
 * intrinsic permeability"):
 *   - single-relaxation-time (BGK) lattice Boltzmann with the normalised
 *     relaxation time tau and viscosity nu = (tau - 1/2)/3 in lattice units
 *     (Eq. 1 with c = dx = dt = 1); optionally the two-relaxation-time
 *     collision (TRT, Ginzburg), a multi-relaxation scheme of the kind the
 *     paper names for a wider tau range;
 *   - the D2Q9 and D3Q19 lattices (Qian, d'Humieres & Lallemand 1992), which the
 *     paper uses for its 2D and 3D cases;
 *   - pressure-driven flow along x (Results, first paragraph): density imposed
 *     on ghost planes at x = -1 and x = nx by non-equilibrium extrapolation
 *     (Guo, Zheng & Shi 2002), symmetric (free-slip mirror) planes on the
 *     y (and z) faces as in Fig. 1, halfway bounce-back on solid voxels;
 *   - the Darcy permeability from the mass flow rate (Results, first
 *     paragraph), i.e. Eq. 2 with the body force replaced by the pressure
 *     gradient per unit density;
 *   - Kn = sqrt(pi/6) (tau - 1/2) / Nx (discussion of Fig. 2);
 *   - the paper's 3D case: force-driven flow with six periodic faces and the
 *     permeability of Eq. 2, with the body force entering by the forcing of
 *     Guo, Zheng & Shi (2002) (the paper names no scheme).
 * The readings of what the paper leaves unstated (solid boundary rule, the
 * pressure-boundary mechanism, the flux definition, the convergence test) are
 * listed with the design notes of the repository.
 *
 * Conventions: lattice units; populations stored node-major f[node*Q + i],
 * nodes ordered x fastest, then y, then z.  All arithmetic is IEEE binary64,
 * compiled without floating-point contraction, with a fixed loop order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define QMAX 19

typedef struct {
  int Q, nx, ny, nz;
  int c[QMAX][3];
  double w[QMAX];
  int opp[QMAX], my[QMAX], mz[QMAX];
  double tau, rho_in, rho_out;
  int linear_eq;          /* 1: equilibrium without the terms nonlinear in u */
  int periodic;           /* 1: all six faces periodic (force-driven case) */
  double force;           /* body-force density along x, F = rho0 g (periodic case) */
  double rho0;            /* reference density of the force and of Eq. 2 */
  int trt;                /* 1: two-relaxation-time collision */
  double tau_minus;       /* TRT: relaxation time of the odd (antisymmetric) part */
  unsigned char *solid;   /* [nz][ny][nx], 1 = solid */
  double *f;              /* post-collision populations of the current step */
  double *tmp;
  long long steps;
} oracle_t;

/* ------------------------------------------------------------------ lattice */

static int find_dir(const oracle_t *o, int cx, int cy, int cz) {
  for (int i = 0; i < o->Q; ++i)
    if (o->c[i][0] == cx && o->c[i][1] == cy && o->c[i][2] == cz) return i;
  return -1;
}

/* D2Q9: rest, 4 axis directions (w = 1/9), 4 diagonals (w = 1/36).
 * D3Q19: rest (1/3), 6 axis directions (1/18), 12 edge diagonals (1/36).
 * The ordering is this file's own convention. */
static int set_lattice(oracle_t *o, int Q) {
  static const int d2q9[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                                 {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
  o->Q = Q;
  if (Q == 9) {
    for (int i = 0; i < 9; ++i) {
      for (int a = 0; a < 3; ++a) o->c[i][a] = d2q9[i][a];
      int n = abs(d2q9[i][0]) + abs(d2q9[i][1]);
      o->w[i] = n == 0 ? 4.0 / 9.0 : (n == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
  } else if (Q == 19) {
    int i = 0;
    o->c[i][0] = o->c[i][1] = o->c[i][2] = 0;
    o->w[i++] = 1.0 / 3.0;
    for (int a = 0; a < 3; ++a)
      for (int s = 1; s >= -1; s -= 2) {
        o->c[i][0] = o->c[i][1] = o->c[i][2] = 0;
        o->c[i][a] = s;
        o->w[i++] = 1.0 / 18.0;
      }
    for (int a = 0; a < 3; ++a)
      for (int b = a + 1; b < 3; ++b)
        for (int sa = 1; sa >= -1; sa -= 2)
          for (int sb = 1; sb >= -1; sb -= 2) {
            o->c[i][0] = o->c[i][1] = o->c[i][2] = 0;
            o->c[i][a] = sa;
            o->c[i][b] = sb;
            o->w[i++] = 1.0 / 36.0;
          }
  } else {
    return -1;
  }
  for (int i = 0; i < Q; ++i) {
    o->opp[i] = find_dir(o, -o->c[i][0], -o->c[i][1], -o->c[i][2]);
    o->my[i] = find_dir(o, o->c[i][0], -o->c[i][1], o->c[i][2]);
    o->mz[i] = find_dir(o, o->c[i][0], o->c[i][1], -o->c[i][2]);
  }
  return 0;
}

/* Bracket of the second-order equilibrium: f_eq_i = w_i rho P_i(u) with
 * P_i(u) = 1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u, c_s^2 = 1/3.  The linear
 * variant drops the two terms quadratic in u. */
static double poly(const oracle_t *o, int i, const double u[3]) {
  double cu = o->c[i][0] * u[0] + o->c[i][1] * u[1] + o->c[i][2] * u[2];
  if (o->linear_eq) return 1.0 + 3.0 * cu;
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
}

static void moments(const oracle_t *o, const double *fn, double *rho, double u[3]) {
  double r = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < o->Q; ++i) {
    r += fn[i];
    for (int a = 0; a < 3; ++a) j[a] += o->c[i][a] * fn[i];
  }
  *rho = r;
  for (int a = 0; a < 3; ++a) u[a] = j[a] / r;
}

static long long node(const oracle_t *o, int x, int y, int z) {
  return ((long long)z * o->ny + y) * o->nx + x;
}

/* ------------------------------------------------------------------ stepping */

/* Value pulled into direction i at fluid node (x,y,z): the population that
 * left the source node x - c_i during the previous step, after the boundary
 * rules (mirror planes, then solid, then inlet/outlet ghost). */
static double pulled(const oracle_t *o, int x, int y, int z, int i) {
  const double *f = o->f;
  const int Q = o->Q;
  int sx = x - o->c[i][0], sy = y - o->c[i][1], sz = z - o->c[i][2];
  int k = i;
  long long here = node(o, x, y, z);
  if (o->periodic) {
    /* the source wraps around every face; solid sources bounce back */
    sx = (sx + o->nx) % o->nx;
    sy = (sy + o->ny) % o->ny;
    sz = (sz + o->nz) % o->nz;
    long long s = node(o, sx, sy, sz);
    if (o->solid[s]) return f[here * Q + o->opp[i]];
    return f[s * Q + i];
  }
  /* symmetric planes half a spacing outside the first/last row */
  if (sy < 0 || sy >= o->ny) {
    sy = sy < 0 ? 0 : o->ny - 1;
    k = o->my[k];
  }
  if (sz < 0 || sz >= o->nz) {
    sz = sz < 0 ? 0 : o->nz - 1;
    k = o->mz[k];
  }
  if (sx >= 0 && sx < o->nx) {
    long long s = node(o, sx, sy, sz);
    if (o->solid[s]) return f[here * Q + o->opp[i]]; /* halfway bounce-back */
    return f[s * Q + k];
  }
  /* ghost plane x = -1 (inlet) or x = nx (outlet): solidity copies the edge
   * column; value by non-equilibrium extrapolation from the edge node b. */
  int bx = sx < 0 ? 0 : o->nx - 1;
  long long b = node(o, bx, sy, sz);
  if (o->solid[b]) return f[here * Q + o->opp[i]];
  double rho_b, u_b[3];
  moments(o, f + b * Q, &rho_b, u_b);
  double rho_set = sx < 0 ? o->rho_in : o->rho_out;
  return f[b * Q + k] + o->w[i] * (rho_set - rho_b) * poly(o, k, u_b);
}

/* BGK collision.  With a body force F = (force, 0, 0) the forcing of Guo,
 * Zheng & Shi (2002): the equilibrium takes u = (j + F/2)/rho and the
 * population i gains (1 - 1/(2 tau)) F_i with
 *   F_i = w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)],
 * or F_i = 3 w_i c_i.F with the linear equilibrium (both linear in the
 * deviations from rest then). */
static void collide_trt(const oracle_t *o, const double *fin, double *fout);

static void collide(const oracle_t *o, const double *fin, double *fout) {
  if (o->trt) {
    collide_trt(o, fin, fout);
    return;
  }
  double rho, u[3];
  moments(o, fin, &rho, u);
  const double F = o->force;
  if (F != 0.0) u[0] += 0.5 * F / rho;
  for (int i = 0; i < o->Q; ++i) {
    double feq = o->w[i] * rho * poly(o, i, u);
    fout[i] = fin[i] - (fin[i] - feq) / o->tau;
    if (F != 0.0) {
      double cx = o->c[i][0];
      double Fi;
      if (o->linear_eq) {
        Fi = 3.0 * o->w[i] * cx * F;
      } else {
        double cu = o->c[i][0] * u[0] + o->c[i][1] * u[1] + o->c[i][2] * u[2];
        Fi = o->w[i] * (3.0 * (cx - u[0]) * F + 9.0 * cu * cx * F);
      }
      fout[i] += (1.0 - 0.5 / o->tau) * Fi;
    }
  }
}

/* Two-relaxation-time collision (Ginzburg's TRT; the paper names
 * multi-relaxation-time schemes as the way to a wider tau range).  Every
 * population and its opposite direction split into a symmetric (even) and an
 * antisymmetric (odd) half: x+_i = (x_i + x_opp(i))/2, x-_i = (x_i - x_opp(i))/2.
 * The even non-equilibrium half relaxes with tau+ = tau (which sets the
 * viscosity), the odd half with tau-; the magic parameter
 * Lambda = (tau+ - 1/2)(tau- - 1/2) fixes the bounce-back wall position, so
 * with Lambda held the steady solutions do not depend on tau.  The body force
 * term of the BGK collision splits the same way, each half with its own
 * (1 - 1/(2 tau+-)) factor.  Lambda = (tau - 1/2)^2 (tau- = tau) is BGK. */
static void collide_trt(const oracle_t *o, const double *fin, double *fout) {
  double rho, u[3];
  moments(o, fin, &rho, u);
  const double F = o->force;
  if (F != 0.0) u[0] += 0.5 * F / rho;
  double neq[QMAX], src[QMAX];
  for (int i = 0; i < o->Q; ++i) {
    neq[i] = fin[i] - o->w[i] * rho * poly(o, i, u);
    src[i] = 0.0;
    if (F != 0.0) {
      double cx = o->c[i][0];
      if (o->linear_eq) {
        src[i] = 3.0 * o->w[i] * cx * F;
      } else {
        double cu = o->c[i][0] * u[0] + o->c[i][1] * u[1] + o->c[i][2] * u[2];
        src[i] = o->w[i] * (3.0 * (cx - u[0]) * F + 9.0 * cu * cx * F);
      }
    }
  }
  const double tp = o->tau, tm = o->tau_minus;
  for (int i = 0; i < o->Q; ++i) {
    const int j = o->opp[i];
    const double n_even = 0.5 * (neq[i] + neq[j]), n_odd = 0.5 * (neq[i] - neq[j]);
    const double s_even = 0.5 * (src[i] + src[j]), s_odd = 0.5 * (src[i] - src[j]);
    fout[i] = fin[i] - n_even / tp - n_odd / tm + (1.0 - 0.5 / tp) * s_even +
              (1.0 - 0.5 / tm) * s_odd;
  }
}

static void step_once(oracle_t *o) {
  const int Q = o->Q;
  const long long rows = (long long)o->nz * o->ny;
#pragma omp parallel for schedule(static)
  for (long long r = 0; r < rows; ++r) {
    int z = (int)(r / o->ny), y = (int)(r % o->ny);
    double fin[QMAX];
    for (int x = 0; x < o->nx; ++x) {
      long long n = node(o, x, y, z);
      if (o->solid[n]) continue;
      for (int i = 0; i < Q; ++i) fin[i] = pulled(o, x, y, z, i);
      collide(o, fin, o->tmp + n * Q);
    }
  }
  double *t = o->f;
  o->f = o->tmp;
  o->tmp = t;
  o->steps += 1;
}

/* --------------------------------------------------------------- public API */

oracle_t *oracle_create(int Q, int nx, int ny, int nz, const unsigned char *solid,
                        double tau, double rho_in, double rho_out, int linear_eq) {
  if (nx < 1 || ny < 1 || nz < 1 || (Q == 9 && nz != 1)) return NULL;
  oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
  if (!o) return NULL;
  if (set_lattice(o, Q)) { free(o); return NULL; }
  o->nx = nx; o->ny = ny; o->nz = nz;
  o->tau = tau; o->rho_in = rho_in; o->rho_out = rho_out; o->linear_eq = linear_eq;
  long long N = (long long)nx * ny * nz;
  o->solid = (unsigned char *)malloc((size_t)N);
  o->f = (double *)malloc((size_t)N * Q * sizeof(double));
  o->tmp = (double *)malloc((size_t)N * Q * sizeof(double));
  if (!o->solid || !o->f || !o->tmp) {
    free(o->solid); free(o->f); free(o->tmp); free(o);
    return NULL;
  }
  for (long long n = 0; n < N; ++n) o->solid[n] = solid[n] ? 1 : 0;
  /* Solid slots are never read: they hold NaN so that any read would show. */
  for (long long n = 0; n < N * Q; ++n) o->f[n] = o->tmp[n] = NAN;
  return o;
}

/* Periodic, force-driven case (the paper's 3D experiment): all six faces
 * periodic and a body force along x of density force = rho0 g.  periodic = 0
 * returns to the pressure-driven case (force must then be 0). */
int oracle_set_periodic(oracle_t *o, int periodic, double force, double rho0) {
  if (!periodic && force != 0.0) return -1;
  o->periodic = periodic ? 1 : 0;
  o->force = force;
  o->rho0 = rho0;
  return 0;
}

/* Collision model: magic > 0 selects TRT with Lambda = magic, i.e.
 * tau- = 1/2 + magic / (tau - 1/2); magic = 0 returns to BGK.  Returns -1 for
 * a negative or non-finite magic. */
int oracle_set_trt(oracle_t *o, double magic) {
  if (!(magic >= 0.0) || !isfinite(magic)) return -1;
  o->trt = magic > 0.0;
  o->tau_minus = o->trt ? 0.5 + magic / (o->tau - 0.5) : o->tau;
  return 0;
}

void oracle_destroy(oracle_t *o) {
  if (!o) return;
  free(o->solid); free(o->f); free(o->tmp); free(o);
}

/* Zero-velocity start: f_i = w_i rho at every fluid node.  mode 0: uniform
 * rho = (rho_in + rho_out)/2.  mode 1: rho linear in x between the ghost
 * planes, rho(x) = rho_in + (rho_out - rho_in)(x + 1)/(nx + 1). */
void oracle_init_rest(oracle_t *o, int mode) {
  const int Q = o->Q;
  for (int z = 0; z < o->nz; ++z)
    for (int y = 0; y < o->ny; ++y)
      for (int x = 0; x < o->nx; ++x) {
        long long n = node(o, x, y, z);
        if (o->solid[n]) continue;
        double rho = mode == 1 ? o->rho_in + (o->rho_out - o->rho_in) * (x + 1) / (double)(o->nx + 1)
                               : 0.5 * (o->rho_in + o->rho_out);
        for (int i = 0; i < Q; ++i) o->f[n * Q + i] = o->w[i] * rho;
      }
  o->steps = 0;
}

/* Start from given fields: f_i = f_eq_i(rho, u) at fluid nodes.  rho[N],
 * u[N*3] (x,y,z components per node). */
void oracle_init_fields(oracle_t *o, const double *rho, const double *u) {
  const int Q = o->Q;
  long long N = (long long)o->nx * o->ny * o->nz;
  for (long long n = 0; n < N; ++n) {
    if (o->solid[n]) continue;
    for (int i = 0; i < Q; ++i) o->f[n * Q + i] = o->w[i] * rho[n] * poly(o, i, u + 3 * n);
  }
  o->steps = 0;
}

void oracle_set_f(oracle_t *o, const double *f) {
  long long N = (long long)o->nx * o->ny * o->nz;
  for (long long n = 0; n < N; ++n)
    if (!o->solid[n])
      for (int i = 0; i < o->Q; ++i) o->f[n * o->Q + i] = f[n * o->Q + i];
}

void oracle_get_f(const oracle_t *o, double *f) {
  long long N = (long long)o->nx * o->ny * o->nz;
  memcpy(f, o->f, (size_t)(N * o->Q) * sizeof(double));
}

void oracle_step(oracle_t *o, long long n) {
  for (long long s = 0; s < n; ++s) step_once(o);
}

long long oracle_steps(const oracle_t *o) { return o->steps; }

/* Density and velocity of every node (NaN on solids).  With a body force the
 * stored populations are post-collision and hold the whole step's force, so
 * the velocity of the forcing scheme is u = (j - F/2)/rho, the same velocity
 * the flux and Eq. 2 use. */
void oracle_macro(const oracle_t *o, double *rho, double *u) {
  long long N = (long long)o->nx * o->ny * o->nz;
  for (long long n = 0; n < N; ++n) {
    if (o->solid[n]) {
      rho[n] = NAN;
      u[3 * n] = u[3 * n + 1] = u[3 * n + 2] = NAN;
      continue;
    }
    moments(o, o->f + n * o->Q, rho + n, u + 3 * n);
    if (o->force != 0.0) u[3 * n] -= 0.5 * o->force / rho[n];
  }
}

/* Mass flow rate: x-momentum summed over the fluid nodes, divided by nx, i.e.
 * the mean over x of the mass flux through a cross-section.  With a body
 * force the momentum of a node is rho u = j - F/2 in terms of its stored
 * (post-collision) populations, whose momentum already holds the step's F. */
double oracle_flux(const oracle_t *o) {
  double s = 0.0;
  long long N = (long long)o->nx * o->ny * o->nz;
  for (long long n = 0; n < N; ++n) {
    if (o->solid[n]) continue;
    double j = 0.0;
    for (int i = 0; i < o->Q; ++i) j += o->c[i][0] * o->f[n * o->Q + i];
    s += j - 0.5 * o->force;
  }
  return s / o->nx;
}

/* Total mass: sum of all fluid populations. */
double oracle_mass(const oracle_t *o) {
  double s = 0.0;
  long long N = (long long)o->nx * o->ny * o->nz;
  for (long long n = 0; n < N; ++n) {
    if (o->solid[n]) continue;
    for (int i = 0; i < o->Q; ++i) s += o->f[n * o->Q + i];
  }
  return s;
}

/* Darcy permeability in lattice units (dx^2) from the mass flow rate:
 * k = nu Q_m L / (A c_s^2 (rho_in - rho_out)), nu = (tau - 1/2)/3 (Eq. 1),
 * L = nx + 1 (distance between the density-imposing ghost planes), A = ny*nz. */
double oracle_permeability(const oracle_t *o) {
  double nu = (o->tau - 0.5) / 3.0;
  if (o->periodic) {
    /* Eq. 2: kappa = nu <u>_Omega / g, <u>_Omega = sum_fluid u_x / N_grid,
     * with rho u / rho0 for u (Stokes regime) and g = force / rho0:
     * kappa = nu (nx Q_m) / (N_grid force) */
    double N = (double)o->nx * o->ny * o->nz;
    return nu * oracle_flux(o) * o->nx / (N * o->force);
  }
  double L = o->nx + 1.0, A = (double)o->ny * o->nz;
  return nu * oracle_flux(o) * L / (A * (1.0 / 3.0) * (o->rho_in - o->rho_out));
}

/* Iterate until the relative change of the flux over a window of K steps is
 * below tol (first check after K steps, against the starting flux), or until
 * max_steps.  Returns 0 when converged, 1 otherwise. */
int oracle_run_to_steady(oracle_t *o, double tol, int K, long long max_steps,
                         long long *steps, double *resid) {
  double prev = oracle_flux(o), r = INFINITY;
  int rc = 1;
  while (o->steps + K <= max_steps) {
    oracle_step(o, K);
    double q = oracle_flux(o);
    r = fabs(q - prev) / fabs(q);
    prev = q;
    if (r < tol) { rc = 0; break; }
  }
  if (steps) *steps = o->steps;
  if (resid) *resid = r;
  return rc;
}

/* ------------------------------------------------ single-node entry points */

/* Lattice tables: c[Q*3], w[Q], opp[Q], my[Q], mz[Q].  Returns Q or -1. */
int oracle_lattice(int Q, int *c, double *w, int *opp, int *my, int *mz) {
  oracle_t o;
  memset(&o, 0, sizeof o);
  if (set_lattice(&o, Q)) return -1;
  for (int i = 0; i < Q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = o.c[i][a];
    w[i] = o.w[i]; opp[i] = o.opp[i]; my[i] = o.my[i]; mz[i] = o.mz[i];
  }
  return Q;
}

void oracle_feq(int Q, double rho, const double *u, int linear_eq, double *out) {
  oracle_t o;
  memset(&o, 0, sizeof o);
  set_lattice(&o, Q);
  o.linear_eq = linear_eq;
  for (int i = 0; i < Q; ++i) out[i] = o.w[i] * rho * poly(&o, i, u);
}

void oracle_collide(int Q, const double *fin, double tau, int linear_eq, double *out) {
  oracle_t o;
  memset(&o, 0, sizeof o);
  set_lattice(&o, Q);
  o.tau = tau;
  o.linear_eq = linear_eq;
  collide(&o, fin, out);
}

/* One TRT collision of a node's populations (no force); magic as in
 * oracle_set_trt (> 0). */
void oracle_collide_trt(int Q, const double *fin, double tau, double magic, int linear_eq,
                        double *out) {
  oracle_t o;
  memset(&o, 0, sizeof o);
  set_lattice(&o, Q);
  o.tau = tau;
  o.linear_eq = linear_eq;
  o.trt = 1;
  o.tau_minus = 0.5 + magic / (tau - 0.5);
  collide(&o, fin, out);
}

double oracle_knudsen(double tau, int nx) { return sqrt(M_PI / 6.0) * (tau - 0.5) / nx; }

/* Thread control for the node loop (the results do not depend on it: every
 * node is computed independently and every reduction runs sequentially). */
#ifdef _OPENMP
#include <omp.h>
void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int oracle_threads(void) { return omp_get_max_threads(); }
#else
void oracle_set_threads(int n) { (void)n; }
int oracle_threads(void) { return 1; }
#endif
