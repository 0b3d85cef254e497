// The library's host-side argument checks and size queries, called through
// the C ABI from a program built with AddressSanitizer and
// UndefinedBehaviorSanitizer together with host-only builds of the library
// sources (tests/test_abi_sanitized.py).  Every call here must return before
// any HIP call: the pointers passed are never dereferenced.  Prints one line
// per failed expectation and exits with the number of failures.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <initializer_list>

#include "lbm.h"
#include "wsn.h"

static int failures = 0;

#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      ++failures;                                                      \
      printf("FAIL line %d: %s (%s)\n", __LINE__, #cond, lbm_last_error()); \
    }                                                                  \
  } while (0)

static lbm_geom geom(int lattice, int nx, int ny, int nz, int precision, int64_t n_fluid) {
  lbm_geom g;
  memset(&g, 0, sizeof g);
  g.lattice = lattice;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.precision = precision;
  g.check_every = 100;
  g.rho0 = 1.0;
  g.n_fluid = n_fluid;
  g.boundary = LBM_BC_PRESSURE;
  g.body_force = 0.0;
  return g;
}

static void query_sizes() {
  size_t fb = 0, wb = 0;
  const lbm_geom ok = geom(LBM_D2Q9, 100, 50, 1, LBM_FP64, 5000);
  lbm_geom bad[16];
  int n = 0;
  bad[n] = ok; bad[n++].lattice = 7;
  bad[n] = ok; bad[n++].nz = 2;
  bad[n] = ok; bad[n++].nx = 1;
  bad[n] = ok; bad[n++].ny = 0;
  bad[n] = ok; bad[n++].precision = 5;
  bad[n] = ok; bad[n++].check_every = 0;
  bad[n] = ok; bad[n++].rho0 = 0.0;
  bad[n] = ok; bad[n++].rho0 = NAN;
  bad[n] = ok; bad[n++].n_fluid = -1;
  bad[n] = ok; bad[n++].n_fluid = 5001;
  bad[n] = geom(LBM_D3Q19, 2048, 2048, 1025, LBM_FP32, (1ll << 32) + 5); ++n;
  bad[n] = ok; bad[n++].boundary = 2;
  bad[n] = ok; bad[n++].boundary = -1;
  bad[n] = ok; bad[n].boundary = LBM_BC_PERIODIC; bad[n++].body_force = INFINITY;
  bad[n] = ok; bad[n++].body_force = 1e-5;
  for (int i = 0; i < n; ++i) {
    EXPECT(lbm_query_sizes(&bad[i], &fb, &wb) == LBM_EINVAL);
    EXPECT(lbm_last_error()[0] != '\0');
  }
  EXPECT(lbm_query_sizes(nullptr, &fb, &wb) == LBM_EINVAL);
  // valid geometries, ragged and degenerate, both lattices and precisions
  const int shapes[][4] = {{9, 100, 50, 1},  {9, 2, 1, 1},     {9, 7, 3, 1},    {9, 65, 2, 1},
                           {9, 257, 9, 1},   {9, 1200, 600, 1}, {19, 2, 1, 1},  {19, 33, 7, 5},
                           {19, 130, 9, 7},  {19, 512, 512, 512}};
  for (const auto& s : shapes)
    for (int prec : {LBM_FP64, LBM_FP32})
      for (int64_t frac : {0, 1, 2}) {
        const int64_t nodes = (int64_t)s[1] * s[2] * s[3];
        lbm_geom g = geom(s[0], s[1], s[2], s[3], prec, nodes * frac / 2);
        fb = wb = 0;
        EXPECT(lbm_query_sizes(&g, &fb, &wb) == LBM_OK);
        EXPECT(fb >= (size_t)s[0] * (size_t)g.n_fluid * (prec == LBM_FP64 ? 8u : 4u));
        EXPECT(wb > 0);
        g.boundary = LBM_BC_PERIODIC;
        g.body_force = 1e-6;
        EXPECT(lbm_query_sizes(&g, &fb, &wb) == LBM_OK);
      }
}

static void init_and_null_contexts() {
  const lbm_geom g = geom(LBM_D2Q9, 100, 50, 1, LBM_FP64, 5000);
  const uintptr_t fake = 1u << 20;
  lbm_buffers b;
  b.f[0] = (void*)fake;
  b.f[1] = (void*)(fake * 2);
  b.mask = (const void*)(fake * 3);
  b.work = (void*)(fake * 4);
  b.stream = nullptr;
  lbm_ctx* h = nullptr;
  const double bad[][3] = {{0.5, 1.0, 1.0}, {0.2, 1.0, 1.0}, {NAN, 1.0, 1.0},
                           {0.8, 0.0, 1.0}, {0.8, 1.0, -1.0}, {INFINITY, 1.0, 1.0}};
  for (const auto& a : bad) {
    EXPECT(lbm_init(&h, &g, &b, a[0], a[1], a[2]) == LBM_EINVAL);
    EXPECT(h == nullptr);
  }
  lbm_buffers none;
  memset(&none, 0, sizeof none);
  EXPECT(lbm_init(&h, &g, &none, 0.8, 1.0, 1.0) == LBM_EINVAL);
  lbm_buffers same = b;
  same.f[1] = same.f[0];
  EXPECT(lbm_init(&h, &g, &same, 0.8, 1.0, 1.0) == LBM_EINVAL);
  lbm_buffers odd = b;
  odd.f[0] = (void*)(fake + 4);
  EXPECT(lbm_init(&h, &g, &odd, 0.8, 1.0, 1.0) == LBM_EINVAL);
  EXPECT(lbm_init(nullptr, &g, &b, 0.8, 1.0, 1.0) == LBM_EINVAL);
  EXPECT(lbm_init(&h, nullptr, &b, 0.8, 1.0, 1.0) == LBM_EINVAL);
  EXPECT(lbm_init(&h, &g, nullptr, 0.8, 1.0, 1.0) == LBM_EINVAL);
  lbm_geom gp = g;
  gp.boundary = LBM_BC_PERIODIC;
  gp.body_force = 1e-5;
  EXPECT(lbm_init(&h, &gp, &b, 0.8, 1.001, 0.999) == LBM_EINVAL);
  EXPECT(h == nullptr);

  double d = 0;
  int64_t s = 0;
  float fl = 0;
  int32_t map = 0;
  EXPECT(lbm_reset(nullptr, LBM_START_UNIFORM) == LBM_EINVAL);
  EXPECT(lbm_set_macro(nullptr, &fl, &fl) == LBM_EINVAL);
  EXPECT(lbm_smooth(nullptr, 1) == LBM_EINVAL);
  EXPECT(lbm_step(nullptr, 1) == LBM_EINVAL);
  EXPECT(lbm_flux(nullptr, &d) == LBM_EINVAL);
  EXPECT(lbm_flux_noalloc(nullptr, &d) == LBM_EINVAL);
  EXPECT(lbm_permeability(nullptr, &d) == LBM_EINVAL);
  EXPECT(lbm_run_to_steady(nullptr, 1e-9, 100, &s, &d) == LBM_EINVAL);
  EXPECT(lbm_get_macro(nullptr, &fl, &fl, 0) == LBM_EINVAL);
  EXPECT(lbm_get_populations(nullptr, &fl) == LBM_EINVAL);
  EXPECT(lbm_set_populations(nullptr, &fl) == LBM_EINVAL);
  EXPECT(lbm_get_slot_map(nullptr, &map) == LBM_EINVAL);
  EXPECT(lbm_set_option(nullptr, 1, 0) == LBM_EINVAL);
  EXPECT(lbm_set_trt(nullptr, 0.1875) == LBM_EINVAL);
  EXPECT(lbm_steps(nullptr, &s) == LBM_EINVAL);
  EXPECT(lbm_destroy(nullptr) == LBM_OK);
}

static void tables() {
  int32_t c[19 * 3];
  double w[19];
  for (int lat : {LBM_D2Q9, LBM_D3Q19}) {
    EXPECT(lbm_lattice(lat, c, w) == LBM_OK);
    const int Q = lat == LBM_D2Q9 ? 9 : 19;
    double sw = 0;
    for (int i = 0; i < Q; ++i) sw += w[i];
    EXPECT(fabs(sw - 1.0) < 1e-15);
  }
  EXPECT(lbm_lattice(7, c, w) == LBM_EINVAL);
  EXPECT(fabs(lbm_knudsen(0.8, 100) - sqrt(M_PI / 6.0) * 0.3 / 100) < 1e-18);
  EXPECT(lbm_version() != nullptr && lbm_version()[0] != '\0');
}

static void batches() {
  size_t wb = 0;
  EXPECT(lbm_batch_query_sizes(0, nullptr, &wb) == LBM_EINVAL);
  EXPECT(lbm_batch_query_sizes(2, nullptr, &wb) == LBM_EINVAL);
  lbm_ctx* nulls[2] = {nullptr, nullptr};
  EXPECT(lbm_batch_query_sizes(2, nulls, &wb) == LBM_EINVAL);
  lbm_batch* h = nullptr;
  EXPECT(lbm_batch_create(&h, 2, nulls, (void*)(1u << 20), nullptr) == LBM_EINVAL);
  EXPECT(h == nullptr);
  EXPECT(lbm_batch_create(nullptr, 1, nulls, (void*)(1u << 20), nullptr) == LBM_EINVAL);
  EXPECT(lbm_batch_step(nullptr, 1) == LBM_EINVAL);
  EXPECT(lbm_batch_run_to_steady(nullptr, 1e-9, 10, nullptr, nullptr, nullptr, nullptr, 0) ==
         LBM_EINVAL);
  EXPECT(lbm_batch_flux(nullptr, nullptr) == LBM_EINVAL);
  EXPECT(lbm_batch_permeability(nullptr, nullptr, nullptr) == LBM_EINVAL);
  EXPECT(lbm_batch_set_option(nullptr, LBM_BATCH_OPT_GRAPH, 1) == LBM_EINVAL);
  EXPECT(lbm_batch_destroy(nullptr) == LBM_OK);
}

static void network() {
  int64_t np = 0;
  size_t ab = 0, wb = 0;
  wsn_config cfg = {4, 32, 2, 3, 128, 256};
  EXPECT(wsn_query_sizes(&cfg, 8, &np, &ab, &wb) == LBM_OK);
  EXPECT(np == 1946659);
  EXPECT(ab > 0 && wb > ab);
  const wsn_config bad[] = {{0, 32, 2, 3, 128, 256}, {4, 32, 2, 3, 100, 256},
                            {4, 32, 2, 3, 128, 200}, {4, 0, 2, 3, 128, 256},
                            {4, 32, 2, 0, 128, 256}};
  for (const auto& c : bad) EXPECT(wsn_query_sizes(&c, 8, nullptr, nullptr, nullptr) == LBM_EINVAL);
  EXPECT(wsn_query_sizes(&cfg, 0, nullptr, nullptr, nullptr) == LBM_EINVAL);
  float* fake = (float*)(uintptr_t)(1u << 20);
  EXPECT(wsn_conv_forward(fake, fake, nullptr, fake, 1, 8, 24, 4, 4, 3, 1, nullptr) == LBM_EINVAL);
  EXPECT(wsn_conv_forward(fake, fake, nullptr, fake, 1, 8, 32, 4, 4, 5, 1, nullptr) == LBM_EINVAL);
  EXPECT(wsn_conv_forward(nullptr, fake, nullptr, fake, 1, 8, 32, 4, 4, 3, 1, nullptr) == LBM_EINVAL);
  size_t n = 0;
  EXPECT(wsn_conv_wgrad_work(2, 16, 32, 8, 8, 3, &n) == LBM_OK && n > 0);
  for (int ks : {1, 3})
    for (int cin : {2, 16, 32, 96, 256})
      for (int cout : {3, 16, 32, 64, 128}) {
        size_t m = 0;
        EXPECT(wsn_conv_wgrad_work(32, 128, 256, cin, cout, ks, &m) == LBM_OK && m > 0);
      }
  EXPECT(wsn_conv_backward_weight(fake, fake, fake, nullptr, 2, 16, 32, 8, 8, 3, fake, n - 1,
                                  nullptr) == LBM_ENOMEM);
  EXPECT(wsn_pool_forward(fake, fake, 1, 7, 8, 4, nullptr) == LBM_EINVAL);
  EXPECT(wsn_upcat_forward(fake, fake, fake, 1, 8, 8, 0, 4, nullptr) == LBM_EINVAL);
  EXPECT(wsn_adam(fake, fake, fake, fake, 10, 1e-3, 0.9, 0.999, 1e-8, 0, nullptr) == LBM_EINVAL);
  EXPECT(wsn_adam(fake, fake, fake, fake, 10, 1e-3, 1.0, 0.999, 1e-8, 1, nullptr) == LBM_EINVAL);
  EXPECT(wsn_mse_work(0, &n) == LBM_EINVAL);
}

int main() {
  query_sizes();
  init_and_null_contexts();
  tables();
  batches();
  network();
  printf("failures %d\n", failures);
  return failures;
}
