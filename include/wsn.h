/*
 * wsn.h - C ABI of the warm-start network (part of liblbm.so).
 *
 * A small convolutional U-Net maps a D2Q9 solid mask and the Knudsen number
 * Kn = sqrt(pi/6)(tau - 1/2)/Nx (the paper's discussion of Fig. 2) to an
 * initial density / velocity field for lbm_set_macro, so that the plain
 * lattice Boltzmann iteration starts close to its steady state.  The network
 * is trained on steady states of the solver itself; the solver always runs to
 * the same residual from whatever start it is given, so the network changes
 * only the number of steps, never the converged answer.
 *
 * Layout and conventions:
 *   - images are float32 NHWC arrays [batch][height][width][channels] in device
 *     memory owned by the caller;
 *   - a convolution has ks x ks taps (ks = 3 with zero padding 1, or ks = 1)
 *     in row-major order over (dy, dx), weights w[t][cin][cout] (t = 3 (dy + 1)
 *     + (dx + 1) for ks = 3) and bias b[cout]:
 *         y[b,h,x,co] = b[co] + sum_t sum_ci x[b, h+dy, x+dx, ci] w[t,ci,co];
 *   - widths must be multiples of 16; pooled / upsampled sizes halve / double;
 *   - every call enqueues on the HIP stream `stream` and returns an
 *     lbm_status (message via lbm_last_error); arguments are checked before
 *     any HIP call.  Calls never allocate device memory: scratch comes from
 *     caller buffers sized by the *_work / wsn_query_sizes queries.
 *   - results are deterministic: every reduction has a fixed order.
 *
 * Network (wsn_config): `levels` encoder levels with base * 2^l channels, two
 * 3x3 convolutions + ReLU each, 2x2 max pooling between levels; decoder levels
 * upsample (nearest, 2x), concatenate the upsampled channels and then the
 * encoder output of the same level, two 3x3 convolutions + ReLU; a 1x1 head.
 * Parameters are one float32 vector, layer by layer (w then b) in the order
 * enc0a, enc0b, ..., enc{L-1}b, dec{L-2}a, dec{L-2}b, ..., dec0b, head.
 */
#ifndef WSN_H_
#define WSN_H_

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t levels;    /* encoder levels (>= 1)                                   */
  int32_t base;      /* channels of level 0 (>= 1)                              */
  int32_t in_ch;     /* input channels (2: solid mask, scaled Kn)               */
  int32_t out_ch;    /* output channels (3: rho', u'_x, u'_y)                    */
  int32_t height;    /* divisible by 2^(levels-1)                               */
  int32_t width;     /* width >> (levels-1) a multiple of 16                    */
} wsn_config;

/* Sizes for a batch: parameter count, activation bytes (written by the
 * forward pass, read by the backward pass) and work bytes (backward). */
lbm_status wsn_query_sizes(const wsn_config *cfg, int32_t batch, int64_t *n_params,
                           size_t *act_bytes, size_t *work_bytes);

/* y [batch][height][width][out_ch] = network(x [batch][height][width][in_ch]).
 * act: activations of act_bytes, kept for wsn_backward. */
lbm_status wsn_forward(const wsn_config *cfg, int32_t batch, const float *params, const float *x,
                       float *y, void *act, void *stream);

/* Parameter gradient (grad, n_params floats, overwritten) for the output
 * gradient dy, using the activations of the last wsn_forward on the same x
 * and params.  work: work_bytes. */
lbm_status wsn_backward(const wsn_config *cfg, int32_t batch, const float *params, const float *x,
                        const float *dy, float *grad, const void *act, void *work, void *stream);

/* Masked mean squared error over the pixels with solid == 0 and all channels:
 * loss (device double) = sum (pred - target)^2 / (channels * fluid pixels),
 * grad = d loss / d pred (0 on solid pixels).  work: wsn_mse_work bytes. */
lbm_status wsn_mse_work(int64_t npix, size_t *work_bytes);
lbm_status wsn_masked_mse(const float *pred, const float *target, const uint8_t *solid,
                          int64_t npix, int32_t channels, double *loss, float *grad, void *work,
                          size_t work_bytes, void *stream);

/* One Adam step (Kingma & Ba 2015) on n parameters; t >= 1 is the step number
 * (bias corrections 1 - b1^t, 1 - b2^t). */
lbm_status wsn_adam(float *p, const float *g, float *m, float *v, int64_t n, double lr, double b1,
                    double b2, double eps, int64_t t, void *stream);

/* ---- single layers (the network's building blocks) ---------------------- */

/* y = conv(x) (+ ReLU if relu). bias may be NULL. */
lbm_status wsn_conv_forward(const float *x, const float *w, const float *bias, float *y,
                            int32_t batch, int32_t height, int32_t width, int32_t cin,
                            int32_t cout, int32_t ks, int32_t relu, void *stream);

/* dx = gradient of conv's input for output gradient dy.  wflip: scratch of
 * ks*ks*cin*cout floats. */
lbm_status wsn_conv_backward_data(const float *dy, const float *w, float *dx, float *wflip,
                                  int32_t batch, int32_t height, int32_t width, int32_t cin,
                                  int32_t cout, int32_t ks, void *stream);

/* Scratch bytes of wsn_conv_backward_weight for one layer shape. */
lbm_status wsn_conv_wgrad_work(int32_t batch, int32_t height, int32_t width, int32_t cin,
                               int32_t cout, int32_t ks, size_t *work_bytes);

/* dw [ks*ks][cin][cout] and db [cout] (db may be NULL) from the layer input x
 * and the output gradient dy (overwritten, not accumulated). */
lbm_status wsn_conv_backward_weight(const float *x, const float *dy, float *dw, float *db,
                                    int32_t batch, int32_t height, int32_t width, int32_t cin,
                                    int32_t cout, int32_t ks, void *work, size_t work_bytes,
                                    void *stream);

/* g = (y > 0) ? g : 0 elementwise (gradient through a ReLU with output y). */
lbm_status wsn_relu_backward(const float *y, float *g, int64_t n, void *stream);

/* 2x2 max pooling of x [batch][height][width][c] into y [batch][height/2][width/2][c]. */
lbm_status wsn_pool_forward(const float *x, float *y, int32_t batch, int32_t height,
                            int32_t width, int32_t c, void *stream);

/* gx = pooling gradient of gy (to the first maximal element of each window in
 * row-major order) + add (NULL: nothing added); x, add, gx full resolution. */
lbm_status wsn_pool_backward(const float *x, const float *gy, const float *add, float *gx,
                             int32_t batch, int32_t height, int32_t width, int32_t c,
                             void *stream);

/* cat [batch][height][width][c1 + c2]: channels < c1 from deep
 * [batch][height/2][width/2][c1] upsampled 2x (nearest), then skip
 * [batch][height][width][c2]. */
lbm_status wsn_upcat_forward(const float *deep, const float *skip, float *cat, int32_t batch,
                             int32_t height, int32_t width, int32_t c1, int32_t c2, void *stream);

/* Gradients of wsn_upcat_forward: gdeep (2x2 block sums) and gskip. */
lbm_status wsn_upcat_backward(const float *gcat, float *gdeep, float *gskip, int32_t batch,
                              int32_t height, int32_t width, int32_t c1, int32_t c2,
                              void *stream);

/* ---- moving fields between the solver and the network ------------------- */

/* Network input: x[b][p][0] = solid[b][p] (uint8 0/1), x[b][p][1] = feat[b]
 * (one scalar per sample, the scaled Knudsen number). */
lbm_status wsn_pack_input(const uint8_t *solid, const float *feat, int32_t batch, int32_t height,
                          int32_t width, float *x, void *stream);

/* Resistance profile along x of each mask (solid: device uint8 [batch][height][width],
 * 1 = solid; profile: device float [batch][width], width <= 16384): with phi(x)
 * the fluid fraction of column x (at least 1/height) and the Kozeny-Carman
 * resistance R(x) = (1 - phi + 1/height)^2 / phi^3, profile[b][x] =
 * (x + 1)/(width + 1) - sum_{x' <= x} R(x') / sum_x' R(x'): how a density drop
 * that concentrates in the resistive columns departs from the linear drop
 * between the pressure ghost planes (the paper's inlet and outlet
 * conditions), in units of the drop.  An optional network input that carries
 * information along the whole length, which a convolution cannot see. */
lbm_status wsn_column_profile(const uint8_t *solid, int32_t batch, int32_t height, int32_t width,
                              float *profile, void *stream);

/* Network input with the profile as a third channel: x[b][p][0..1] as
 * wsn_pack_input, x[b][p][2] = scale * profile[b][column of p]. */
lbm_status wsn_pack_input_profile(const uint8_t *solid, const float *feat, const float *profile,
                                  float scale, int32_t batch, int32_t height, int32_t width,
                                  float *x, void *stream);

/* Solver fields of a batch (rho [batch][height][width] and u [batch][2][height][width],
 * the layout of lbm_get_macro per sample) into NHWC [batch][height][width][3]:
 * y_k = (f_k - shift[3 b + k] - slope[3 b + k] (x + 1)) * scale[3 b + k],
 * f = (rho, u_x, u_y), x the column; slope may be NULL (no term). */
lbm_status wsn_fields_to_nhwc(const float *rho, const float *u, const float *shift,
                              const float *slope, const float *scale, int32_t batch,
                              int32_t height, int32_t width, float *y, void *stream);

/* The inverse direction: f_k = y_k * scale[3 b + k] + shift[3 b + k]
 * + slope[3 b + k] (x + 1), into the layout of lbm_set_macro; u = 0 wherever
 * keep_u[b][p] == 0 (keep_u: device uint8 [batch][height][width], or NULL to
 * keep every velocity); bad[b] (device int32) becomes 1 if sample b has a
 * non-finite value, else 0. */
lbm_status wsn_nhwc_to_fields(const float *y, const float *shift, const float *slope,
                              const float *scale, const uint8_t *keep_u, int32_t batch,
                              int32_t height, int32_t width, float *rho, float *u, int32_t *bad,
                              void *stream);

/* ---- training data ------------------------------------------------------ */

/* Mirror image of a batch of NHWC images in[batch][height][width][channels]
 * (elem_bytes 4: float32; 1: uint8) into out (same shape; must not overlap
 * in): out[b][h][w][c] = scale[c] * in[b][h'][w'][c] (+ out[b][h][w][c] if
 * accumulate) with h' = height - 1 - h if flip_h else h, and w' likewise with
 * flip_w.  scale: host array of `channels` (<= 8) factors, or NULL for 1;
 * scale and accumulate need float images.  For the warm start's training
 * data and predictions: by the symmetries of the paper's setup (Fig. 1) the
 * symmetric top and bottom boundaries make a steady state mirrored in y a
 * steady state of the mirrored mask (u_y changes sign), and Stokes linearity
 * makes one mirrored in x, with the pressure drop reversed, the steady state
 * of the x-mirrored mask (the deviation from the linear density drop and u_y
 * change sign). */
lbm_status wsn_mirror(const void *in, int32_t elem_bytes, int32_t batch, int32_t height,
                      int32_t width, int32_t channels, int32_t flip_h, int32_t flip_w,
                      const float *scale, int32_t accumulate, void *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* WSN_H_ */
