/* Drives every entry point of the CPU oracle (oracle/lbm_oracle.c) on the
 * domains it reads from stdin, so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks the oracle's memory accesses and integer
 * arithmetic on ragged and degenerate shapes (tests/test_oracle_sanitized.py
 * compares the printed results with the regular build's).
 *
 * Input, per domain: one text line
 *   Q nx ny nz tau rho_in rho_out linear periodic force trt start steps
 * (start: 0 uniform, 1 linear, 2 given fields), then nx*ny*nz mask bytes
 * (1 = solid).  Output, per domain: one line of results.  The fields of
 * start 2 are rho = 1 + 1e-3 sin(n), u_d = 1e-3 cos((d + 1) n) at node n. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct oracle oracle_t;
oracle_t *oracle_create(int Q, int nx, int ny, int nz, const unsigned char *solid, double tau,
                        double rho_in, double rho_out, int linear_eq);
int oracle_set_periodic(oracle_t *o, int periodic, double force, double rho0);
int oracle_set_trt(oracle_t *o, double magic);
void oracle_destroy(oracle_t *o);
void oracle_init_rest(oracle_t *o, int mode);
void oracle_init_fields(oracle_t *o, const double *rho, const double *u);
void oracle_set_f(oracle_t *o, const double *f);
void oracle_get_f(const oracle_t *o, double *f);
void oracle_step(oracle_t *o, long long n);
long long oracle_steps(const oracle_t *o);
void oracle_macro(const oracle_t *o, double *rho, double *u);
double oracle_flux(const oracle_t *o);
double oracle_mass(const oracle_t *o);
double oracle_permeability(const oracle_t *o);
int oracle_run_to_steady(oracle_t *o, double tol, int K, long long max_steps, long long *steps,
                         double *resid);
int oracle_lattice(int Q, int *c, double *w, int *opp, int *my, int *mz);
void oracle_feq(int Q, double rho, const double *u, int linear_eq, double *out);
void oracle_collide(int Q, const double *fin, double tau, int linear_eq, double *out);
void oracle_collide_trt(int Q, const double *fin, double tau, double magic, int linear_eq,
                        double *out);
double oracle_knudsen(double tau, int nx);

static void single_node(int Q) {
  int c[19 * 3], opp[19], my[19], mz[19];
  double w[19], u[3] = {0.01, -0.02, 0.005}, feq[19], out[19], out2[19];
  if (oracle_lattice(Q, c, w, opp, my, mz) != Q) {
    printf("lattice %d failed\n", Q);
    exit(1);
  }
  oracle_feq(Q, 1.01, u, 0, feq);
  for (int i = 0; i < Q; ++i) feq[i] *= 1.0 + 0.01 * (i % 3);
  oracle_collide(Q, feq, 0.7, 0, out);
  oracle_collide_trt(Q, feq, 0.7, 0.1875, 1, out2);
  double s = 0, s2 = 0;
  for (int i = 0; i < Q; ++i) {
    s += out[i] * (i + 1) + w[i] * (opp[i] + my[i] + mz[i] + c[3 * i]);
    s2 += out2[i] * (i + 1);
  }
  printf("node %d %.17g %.17g %.17g\n", Q, s, s2, oracle_knudsen(0.75, 100));
}

int main(void) {
  single_node(9);
  single_node(19);
  int Q, nx, ny, nz, linear, periodic, start;
  double tau, rin, rout, force, trt;
  long long steps;
  while (scanf("%d %d %d %d %lf %lf %lf %d %d %lf %lf %d %lld", &Q, &nx, &ny, &nz, &tau, &rin,
               &rout, &linear, &periodic, &force, &trt, &start, &steps) == 13) {
    getchar();  /* the newline before the mask bytes */
    const long long N = (long long)nx * ny * nz;
    unsigned char *mask = (unsigned char *)malloc((size_t)N);
    if (fread(mask, 1, (size_t)N, stdin) != (size_t)N) return 2;
    oracle_t *o = oracle_create(Q, nx, ny, nz, mask, tau, rin, rout, linear);
    if (!o) return 3;
    if (oracle_set_periodic(o, periodic, force, 1.0) || oracle_set_trt(o, trt)) return 4;
    double *rho = (double *)malloc((size_t)N * sizeof(double));
    double *u = (double *)malloc((size_t)N * 3 * sizeof(double));
    double *f = (double *)malloc((size_t)N * Q * sizeof(double));
    if (start == 2) {
      for (long long n = 0; n < N; ++n) {
        rho[n] = 1.0 + 1e-3 * sin((double)n);
        for (int d = 0; d < 3; ++d) u[3 * n + d] = 1e-3 * cos((double)((d + 1) * n));
      }
      oracle_init_fields(o, rho, u);
    } else {
      oracle_init_rest(o, start);
    }
    oracle_step(o, steps);
    /* a round trip through get_f / set_f must not change the state */
    oracle_get_f(o, f);
    oracle_set_f(o, f);
    oracle_step(o, 1);
    oracle_macro(o, rho, u);
    double srho = 0, su = 0;
    for (long long n = 0; n < N; ++n) {
      if (mask[n]) continue;
      srho += rho[n] * (double)(n % 7 + 1);
      su += u[3 * n] + 2.0 * u[3 * n + 1] + 3.0 * u[3 * n + 2];
    }
    long long st = 0;
    double resid = 0;
    const int rc = oracle_run_to_steady(o, 1e-3, 4, oracle_steps(o) + 40, &st, &resid);
    printf("case %.17g %.17g %.17g %.17g %.17g %d %lld %.17g\n", oracle_flux(o), oracle_mass(o),
           (periodic ? force != 0.0 : rin != rout) ? oracle_permeability(o) : 0.0, srho, su,
           rc, st, resid);
    free(f);
    free(u);
    free(rho);
    free(mask);
    oracle_destroy(o);
  }
  return 0;
}
