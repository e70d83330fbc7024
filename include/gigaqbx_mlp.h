/*
 * gigaqbx_mlp.h -- small dense network that predicts per-center QBX orders (MI355X, gfx950).
 *
 * Sec. 4.1 of Wala & Kloeckner chooses the QBX order from the truncation error, which depends on
 * the local geometry through the expansion radius and the distance to the rest of the curve; the
 * paper then uses one uniform order. This network maps per-center geometry features to predicted
 * log10 errors of QBX at a fixed set of candidate orders, so that each center can take the
 * lowest order whose predicted error meets a tolerance (the caller then passes the orders to
 * gq_set_qbx_orders). It is an addition on top of the method, not part of the paper.
 *
 * Network: x (n_in) -> relu(x W1 + b1) (n_hidden) -> relu(. W2 + b2) (n_hidden) -> . W3 + b3
 * (n_out). Matrix products take BF16 operands (weights and activations rounded to nearest even)
 * with FP32 accumulation on the matrix cores; biases, activations, the loss and the Adam update
 * are FP32, with FP32 master weights.
 *
 * Parameters are one FP32 vector in the order W1 (n_in x n_hidden, row-major), b1 (n_hidden),
 * W2 (n_hidden x n_hidden), b2, W3 (n_hidden x n_out), b3 (n_out).
 * Conventions as in gigaqbx.h: status codes, caller-owned device inputs/outputs, work enqueued on
 * the network's stream. Sizes: 1 <= n_in <= 64, 16 <= n_hidden <= 256 (multiple of 16),
 * 1 <= n_out <= 64.
 */
#ifndef GIGAQBX_MLP_H
#define GIGAQBX_MLP_H

#include <stdint.h>

#include "gigaqbx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gq_mlp gq_mlp;

/* Create a network on `device` with weights drawn from a seeded uniform +-sqrt(6/(fan_in +
 * fan_out)) distribution (biases zero) and Adam moments at zero. */
gq_status gq_mlp_create(gq_mlp **out, int device, void *hip_stream, int n_in, int n_hidden,
                        int n_out, uint64_t seed);
gq_status gq_mlp_destroy(gq_mlp *net);

/* Number of FP32 parameters. */
int64_t gq_mlp_param_count(const gq_mlp *net);

/* Layer sizes given at creation (any output pointer may be NULL). */
gq_status gq_mlp_shape(const gq_mlp *net, int *n_in, int *n_hidden, int *n_out);

/* Copy the FP32 master parameters from / to host memory (synchronous); set also resets Adam. */
gq_status gq_mlp_set_params(gq_mlp *net, const float *host_params);
gq_status gq_mlp_get_params(gq_mlp *net, float *host_params);

/* y = network(x) for n rows; x (n, n_in) and y (n, n_out) are FP32 device arrays. */
gq_status gq_mlp_forward(gq_mlp *net, int64_t n, const float *x, float *y);

/* Loss L = mean over the n rows and n_out outputs of w (y - t)^2 with per-entry weights w (NULL:
 * all ones) and its gradient with respect to the parameters, written to host memory `grads`
 * (param_count FP32) and *loss. x, t, w are FP32 device arrays. Synchronous. */
gq_status gq_mlp_gradients(gq_mlp *net, int64_t n, const float *x, const float *t,
                           const float *w, float *grads, float *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the same loss; *loss (host, may be NULL)
 * receives the loss before the step (synchronous only when loss is not NULL). */
gq_status gq_mlp_train_step(gq_mlp *net, int64_t n, const float *x, const float *t,
                            const float *w, float lr, float *loss);

const char *gq_mlp_last_error(gq_mlp *net);

/* The HIP stream the network's work is enqueued on (as given to gq_mlp_create). */
void *gq_mlp_stream(const gq_mlp *net);

/* ---- per-center features and order prediction (uses a built gq_ctx) ---------------------- */

#define GQ_N_FEATURES 8

/* Geometry features of every center, from the sources within four expansion radii r of it
 * (tree walk over the leaf boxes that meet that disk). Written as FP32 to the device array feat
 * (n_ctr x GQ_N_FEATURES, the caller's center order):
 *   0: arc length (sum of quadrature weights) within 2 r, over 4 r
 *   1: arc length within 4 r, over 8 r
 *   2: distance to the nearest source node, over r
 *   3: log2(r / mean node spacing within 4 r)
 *   4: |sum of w n| / sum of w within 4 r  (1 for one straight piece of curve)
 *   5: weighted standard deviation of (y - c).n / r within 4 r  (curvature)
 *   6: weighted mean of (y - c).n / r within 4 r  (about +1 interior side, -1 exterior side)
 *   7: distance to the nearest source whose normal faces against that of the nearest node,
 *      over 4 r (1 when there is none inside the disk: no opposite sheet of curve nearby)
 * Needs a successful gq_build on a device context (else GQ_ESTATE). Synchronous. */
gq_status gq_center_features(gq_ctx *ctx, float *feat);

/* Per-center QBX orders from the network: features -> network -> predicted log10 QBX error
 * e_j = out_scale * y_j + out_shift for each candidate order cand[j] (n_cand ascending host
 * values in 0..p_qbx; the network's n_out must equal n_cand). Each center takes the smallest
 * candidate with e_j + margins[j] <= log10_tol (margins: n_cand host values, NULL for zeros),
 * else the largest candidate (the fallback for centers the network cannot place, and for
 * non-finite predictions). Orders go to the device array `orders` (n_ctr int32, caller order);
 * with apply != 0 they are then passed to gq_set_qbx_orders. Temporary device buffers are
 * allocated and freed here. Synchronous. */
gq_status gq_orders_predict(gq_ctx *ctx, gq_mlp *net, const int32_t *cand, int n_cand,
                            double out_scale, double out_shift, double log10_tol,
                            const double *margins, int32_t *orders, int apply);

#ifdef __cplusplus
}
#endif

#endif /* GIGAQBX_MLP_H */
