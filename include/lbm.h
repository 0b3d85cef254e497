/*
 * lbm.h - C ABI of the MI355X lattice Boltzmann permeability solver.
 *
 * The solver computes the Darcy permeability of a voxelised porous medium as
 * in Li, Ho, Wu & Zhang, "Lattice Boltzmann modelling of intrinsic
 * permeability": single-relaxation-time (BGK) lattice Boltzmann with the
 * normalised relaxation time tau (viscosity nu = (tau - 1/2)/3 in lattice
 * units, Eq. 1; optionally two relaxation times, lbm_set_trt), with the full
 * or the linear ("Stokes") equilibrium, the D2Q9 and D3Q19 lattices,
 * pressure-driven flow along x
 * with density imposed at the inlet and outlet and symmetric side planes
 * (Fig. 1 and the first paragraph of the Results), iterated to steady Stokes
 * flow; the permeability follows from Darcy's law and the mass flow rate
 * (same paragraph; Eq. 2 with the body force replaced by the pressure
 * gradient), and Kn = sqrt(pi/6)(tau - 1/2)/Nx (discussion of Fig. 2).
 *
 * Boundary rules (the paper names them without giving a scheme):
 *   solid voxels   halfway bounce-back;
 *   y / z faces    specular mirror half a spacing outside the last node row;
 *   x faces        ghost planes at x = -1 and x = nx carrying rho_in / rho_out
 *                  by non-equilibrium extrapolation from the edge node
 *                  (Guo, Zheng & Shi 2002); a ghost copies the solidity of the
 *                  edge node it extrapolates from.
 * With LBM_BC_PERIODIC the faces wrap instead, the flow is driven by the body
 * force (forcing of Guo, Zheng & Shi 2002), rho_in = rho_out is the starting
 * density, and the permeability is Eq. 2: k = nu Q nx / (rho0 g nx ny nz).
 * Lengths are in lattice units; the permeability is in dx^2 with the pressure
 * gradient taken between the ghost planes: k = nu Q L / (A c_s^2 (rho_in -
 * rho_out)), L = nx + 1, A = ny * nz, c_s^2 = 1/3, and Q the mass flow rate,
 * i.e. the x-momentum summed over the fluid nodes divided by nx.
 *
 * Conventions for every entry point:
 *   - All device buffers are allocated and owned by the caller; the library
 *     never allocates or frees device memory through these entry points.  The
 *     buffers must stay alive, unmoved, until lbm_destroy.
 *   - Work is enqueued on the caller's HIP stream (lbm_buffers.stream; NULL =
 *     the legacy default stream).  Entry points that return values computed on
 *     the device synchronise that stream only.
 *   - Every function returns an lbm_status; on failure a message is available
 *     from lbm_last_error() (per thread, valid until the next call on that
 *     thread).  Arguments are validated before any HIP call; an invalid
 *     argument leaves the context unchanged.  A fault inside a kernel shows up
 *     as LBM_EHIP at the next call that checks the stream.
 *   - One context may be driven by one host thread at a time; distinct
 *     contexts are independent.
 *
 * Storage: populations are kept for fluid nodes only, as deviations from the
 * rest state, g_i = f_i - w_i rho0 (so that the tiny Stokes-regime pressure
 * differences survive FP32 rounding), direction-major: g[i][k] where k is the
 * node's slot.  Slots follow the fluid nodes in x-fastest order (x, then y,
 * then z); each row is cut into segments of up to 256 nodes along x, and every
 * segment starts on a 128-byte boundary, the slots between two segments being
 * zero padding.  lbm_get_slot_map gives the slot of every node.  The solid mask
 * is uint8, [nz][ny][nx] with x fastest, 1 = solid, 0 = fluid.
 */
#ifndef LBM_H_
#define LBM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,      /* invalid argument (see lbm_last_error)              */
  LBM_EHIP = -2,        /* a HIP runtime call or kernel launch failed           */
  LBM_ENOMEM = -3,      /* a caller buffer is smaller than lbm_query_sizes says */
  LBM_ENONFINITE = -4,  /* the flux became NaN or infinite                      */
  LBM_ENOTCONV = -5,    /* max_steps reached before the residual tolerance      */
  LBM_ENOFLOW = -6,     /* zero mass flow rate: the medium does not percolate   */
  LBM_ESTATE = -7       /* call not valid in the context's current state        */
} lbm_status;

enum { LBM_D2Q9 = 9, LBM_D3Q19 = 19 };
enum { LBM_FP64 = 0, LBM_FP32 = 1 };          /* storage and in-kernel arithmetic */
enum { LBM_START_UNIFORM = 0, LBM_START_LINEAR = 1 };
/* Boundary cases: pressure-driven flow along x (density on ghost planes at
 * x = -1 and x = nx, symmetric y / z faces; the paper's 2D case), or the
 * paper's 3D case: all six faces periodic and a body force along x, with the
 * permeability of Eq. 2, kappa = nu <u>_Omega / g, <u>_Omega the x-velocity
 * summed over the fluid nodes per grid node (rho u / rho0 for u). */
enum { LBM_BC_PRESSURE = 0, LBM_BC_PERIODIC = 1 };
enum {
  LBM_OPT_XCD_REMAP = 1,  /* tile order over the 8 XCDs when LBM_OPT_BAND is 0: 0 hardware
                             order; 1 one contiguous eighth per XCD (default); m >= 2 chunks
                             of m - 1 tile rows dealt round-robin */
  LBM_OPT_LINEAR_EQ = 2,  /* 1: equilibrium without the terms quadratic in u (Stokes); 0 (default) */
  LBM_OPT_BAND = 6,       /* > 0: banded tile order: bands of this many tile rows, one band
                             per XCD at a time, each walked plane by plane (overrides
                             LBM_OPT_XCD_REMAP); default 16; 0: off */
  LBM_OPT_WIDE_OFFSETS = 7 /* 1: address the populations with 64-bit offsets even when a
                             direction group fits the 32-bit form (the form domains above
                             4 GiB per group use; results are bitwise the same); 0 (default) */
};

typedef struct lbm_ctx lbm_ctx;               /* opaque; host metadata only */

typedef struct {
  int32_t lattice;      /* LBM_D2Q9 or LBM_D3Q19                                  */
  int32_t nx, ny, nz;   /* lattice nodes; nz must be 1 for D2Q9; each >= 1, nx >= 2 */
  int32_t precision;    /* LBM_FP64 or LBM_FP32                                    */
  int32_t check_every;  /* K: steps between two convergence checks (>= 1)          */
  double rho0;          /* reference density of the deviation storage (> 0)        */
  int64_t n_fluid;      /* number of fluid (0) voxels in the mask; lbm_init checks it */
  int32_t boundary;     /* LBM_BC_PRESSURE (0, default) or LBM_BC_PERIODIC             */
  double body_force;    /* LBM_BC_PERIODIC: acceleration g along x (force density
                           rho0 g, forcing of Guo, Zheng & Shi 2002); must be 0 with
                           LBM_BC_PRESSURE                                          */
} lbm_geom;

typedef struct {
  void *f[2];           /* two population buffers, f_bytes each (ping-pong)        */
  const void *mask;     /* device uint8 [nz][ny][nx], 1 = solid; read at init only */
  void *work;           /* device scratch of work_bytes: fluid bitmap and prefix
                           counts, boundary-plane moments, reduction partials      */
  void *stream;         /* hipStream_t the context enqueues on                     */
} lbm_buffers;

/* Bytes the caller must allocate for a geometry.  Fails with LBM_EINVAL on an
 * invalid geometry. */
lbm_status lbm_query_sizes(const lbm_geom *geom, size_t *f_bytes, size_t *work_bytes);

/* Creates a context and starts from rest with uniform density
 * (rho_in + rho_out)/2 (zero-velocity start).  Requires tau > 1/2 (positive
 * viscosity, Eq. 1), rho_in > 0, rho_out > 0, non-NULL 256-byte aligned
 * buffers, and a mask with exactly geom->n_fluid fluid voxels (LBM_EINVAL
 * otherwise).  Builds the fluid bitmap on the device and synchronises the
 * stream once to check the fluid count. */
lbm_status lbm_init(lbm_ctx **out, const lbm_geom *geom, const lbm_buffers *bufs,
                    double tau, double rho_in, double rho_out);

/* Restarts from rest: LBM_START_UNIFORM (rho = (rho_in + rho_out)/2) or
 * LBM_START_LINEAR (rho linear in x between the ghost planes,
 * rho(x) = rho_in + (rho_out - rho_in)(x + 1)/(nx + 1)).  Resets the step count. */
lbm_status lbm_reset(lbm_ctx *ctx, int32_t start);

/* Restarts from given macroscopic fields: every fluid node gets the
 * equilibrium populations of (rho, u).  rho: device float32 [nz][ny][nx];
 * u: device float32 [D][nz][ny][nx] (D = 2 for D2Q9, 3 for D3Q19).  Values at
 * solid nodes are ignored.  Resets the step count.  With a body force F
 * (periodic case) u is the velocity of the forcing scheme, as lbm_get_macro
 * reports it: the stored populations are the equilibrium of rho and
 * u + F/(2 rho). */
lbm_status lbm_set_macro(lbm_ctx *ctx, const float *rho, const float *u);

/* Damps the lattice modes that change sign every step (eigenvalue -1 of the
 * step map, e.g. momentum trapped in dead-end pores by bounce-back): n times,
 * one time step and then the mean of the states before and after it.  Such
 * modes carry no net mass over two steps but never decay, so a state started
 * from fields that excite them converges to a flux offset by them; the
 * smoothing multiplies them by (1 + lambda)/2 per pass and leaves slow modes
 * (lambda near 1) almost unchanged.  Counts n steps. */
lbm_status lbm_smooth(lbm_ctx *ctx, int32_t n);

/* Enqueues n >= 0 time steps (stream + collide). */
lbm_status lbm_step(lbm_ctx *ctx, int64_t n);

/* Mass flow rate Q of the current state (FP64 reduction, deterministic). */
lbm_status lbm_flux(lbm_ctx *ctx, double *q_out);

/* lbm_flux for callers that cannot allocate device memory or that must not
 * touch the context's work buffer (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same kernels and the
 * same result, bitwise, but the flux pass's partials, their chunk sums and the
 * result live in a scratch array of the library (one per GPU, 2 MiB plus a
 * few chunk sums, allocated with the library's code object and held until the
 * process ends).  Allocates nothing.  Limit: at most 2^26 population slots
 * (lbm_query_sizes' f_bytes / (Q * element size)), LBM_EINVAL beyond.  Every
 * call on one GPU uses that GPU's one scratch array: calls that overlap on one
 * GPU (other threads, other streams) race and may return each other's flux. */
lbm_status lbm_flux_noalloc(lbm_ctx *ctx, double *q_out);

/* Darcy permeability of the current state in lattice units (dx^2).
 * LBM_ENOFLOW (k_out = 0) if the flux is exactly zero. */
lbm_status lbm_permeability(lbm_ctx *ctx, double *k_out);

/* Steps until the relative change of the flux over one check window,
 * |Q_t - Q_{t-K}| / |Q_t|, is below tol, checking every K = check_every steps
 * (the first check compares with the flux of the starting state), or until
 * the total step count would exceed max_steps.  steps_out: total steps of the
 * context; resid_out: the last residual.  LBM_ENOTCONV if tol was not reached,
 * LBM_ENONFINITE if the flux is NaN or infinite. */
lbm_status lbm_run_to_steady(lbm_ctx *ctx, double tol, int64_t max_steps,
                             int64_t *steps_out, double *resid_out);

/* Macroscopic fields of the current state into caller device buffers:
 * rho [nz][ny][nx], u [D][nz][ny][nx]; dtype 0 = float32, 1 = float64.
 * Solid nodes get rho = rho0 and u = 0.  With a body force F (periodic case)
 * u = (j - F/2)/rho, j the momentum of the stored post-collision populations:
 * the velocity of the forcing scheme's collision in the last step, which
 * Eq. 2 averages. */
lbm_status lbm_get_macro(lbm_ctx *ctx, void *rho, void *u, int32_t dtype);

/* Checkpoint / restore: copies the current population buffer (f_bytes, the
 * slot layout above, in the direction order of lbm_lattice) to / from device
 * memory.  Padding and unused slots must hold zero (as lbm_get_populations
 * returns them).  lbm_set_populations keeps the step count. */
lbm_status lbm_get_populations(lbm_ctx *ctx, void *dst);
lbm_status lbm_set_populations(lbm_ctx *ctx, const void *src);

/* Slot of every node in the population arrays into a caller device buffer:
 * int32 [nz][ny][nx], -1 for solid nodes. */
lbm_status lbm_get_slot_map(lbm_ctx *ctx, int32_t *map);

/* Tuning and model options (LBM_OPT_*); take effect at the next step. */
lbm_status lbm_set_option(lbm_ctx *ctx, int32_t option, int64_t value);

/* Collision model.  magic > 0: two-relaxation-time collision (TRT,
 * Ginzburg), a multi-relaxation scheme of the kind the paper names for a
 * wider tau range (discussion of Fig. 2): for every direction and its
 * opposite the even half of the non-equilibrium part relaxes with tau (the
 * viscosity, Eq. 1) and the odd half with tau- = 1/2 + magic/(tau - 1/2), so
 * that (tau - 1/2)(tau- - 1/2) = magic; the body-force term splits the same
 * way.  With the magic parameter held the bounce-back wall position no longer
 * moves with tau: a channel of H fluid rows has k = phi (H^2 - 1 + 8 magic)/12
 * at every tau.  magic = 0: BGK (default).  Takes effect at the next step;
 * LBM_EINVAL for a negative or non-finite magic. */
lbm_status lbm_set_trt(lbm_ctx *ctx, double magic);

/* Direction table of the internal order: c[3*Q] (x,y,z per direction) and
 * w[Q].  Q = 9 or 19. */
lbm_status lbm_lattice(int32_t lattice, int32_t *c, double *w);

/* Steps taken since the last start. */
lbm_status lbm_steps(const lbm_ctx *ctx, int64_t *steps_out);

/* Kn = sqrt(pi/6)(tau - 1/2)/nx (discussion of Fig. 2). */
double lbm_knudsen(double tau, int32_t nx);

/* Releases the host-side context.  Does not touch caller buffers.  NULL is
 * accepted. */
lbm_status lbm_destroy(lbm_ctx *ctx);

/* Message of the last failure on the calling thread ("" if none). */
const char *lbm_last_error(void);

/* Version of the library, e.g. "1.0.0". */
const char *lbm_version(void);

/* ------------------------------------------------------------------------
 * Batches: many independent domains (samples of different size, porosity,
 * tau, rho_in / rho_out) advanced together, one kernel launch per time step
 * for all of them.  A batch is a scheduler over existing contexts: each
 * sample is an lbm_ctx created with lbm_init (its buffers, options and state
 * stay its own), and after every batch call each context holds exactly the
 * state, step count and ping-pong parity that the same number of lbm_step
 * calls would have left: per-sample results are bitwise those of running the
 * samples one by one (same tiles, same deterministic reductions).
 *
 * Requirements: 1 <= n samples, all with the same lattice, precision,
 * check_every, boundary case, collision model (BGK or TRT; the magic
 * parameters may differ) and linear-equilibrium option, all on the batch's stream (the
 * stream given to lbm_batch_create).  While a batch exists its contexts may
 * still be used directly (on that stream), but their tile-order options must
 * not change.  Convergence: after every window of K = check_every steps the
 * flux of every running sample is reduced on the device (FP64, one launch for
 * all samples) and read back; a sample whose residual fell below tol, whose
 * flux is not finite, or whose next window would pass max_steps retires: its
 * blocks are dropped from the launch table (a device table that maps every
 * block of the launch to a sample and a block of that sample's own grid), so
 * the remaining samples run without it.  With LBM_BATCH_OPT_GRAPH on, the
 * K-step window and its reductions are captured once as a HIP graph and
 * replayed.
 */
typedef struct lbm_batch lbm_batch;           /* opaque; host metadata only */

enum {
  LBM_BATCH_OPT_GRAPH = 1  /* 1 (default): replay each check window as a HIP graph; 0: launch */
};

/* Device work bytes for a batch of the n contexts ctxs[0..n-1] (launch and
 * reduction tables).  The tile-order options of the contexts at this call
 * fix the size. */
lbm_status lbm_batch_query_sizes(int32_t n, lbm_ctx *const *ctxs, size_t *work_bytes);

/* Creates a batch over ctxs[0..n-1] (the contexts are not copied: they must
 * outlive the batch).  work: device buffer of work_bytes, 256-byte aligned;
 * stream: hipStream_t shared by all contexts.  Uploads the tables and
 * synchronises the stream. */
lbm_status lbm_batch_create(lbm_batch **out, int32_t n, lbm_ctx *const *ctxs, void *work,
                            void *stream);

/* Enqueues nsteps >= 0 time steps of every sample. */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* lbm_run_to_steady for every sample at once, with the same tol, max_steps
 * and check rule as the single-domain call.  Per-sample results go to
 * caller host arrays of n entries (each may be NULL): steps_out (total steps
 * of the context), resid_out (last residual), status_out (LBM_OK,
 * LBM_ENOTCONV or LBM_ENONFINITE).  q_log (host, may be NULL when
 * log_windows is 0): the flux of sample d after window w of this call at
 * q_log[w * n + d] for the first log_windows windows, NaN once the sample
 * has retired.  Returns LBM_OK if every sample converged, else the status of
 * the first sample that did not. */
lbm_status lbm_batch_run_to_steady(lbm_batch *b, double tol, int64_t max_steps,
                                   int64_t *steps_out, double *resid_out,
                                   int32_t *status_out, double *q_log, int64_t log_windows);

/* Mass flow rate of every sample's current state into q_out[n] (host). */
lbm_status lbm_batch_flux(lbm_batch *b, double *q_out);

/* Permeability of every sample into k_out[n] (host), bitwise equal to
 * lbm_permeability of each context; status_out[n] (may be NULL) as there.
 * Returns the first non-OK sample status, else LBM_OK. */
lbm_status lbm_batch_permeability(lbm_batch *b, double *k_out, int32_t *status_out);

/* Batch options (LBM_BATCH_OPT_*). */
lbm_status lbm_batch_set_option(lbm_batch *b, int32_t option, int64_t value);

/* Releases the batch (graphs and host tables).  Contexts and buffers are
 * untouched.  NULL is accepted. */
lbm_status lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H_ */
