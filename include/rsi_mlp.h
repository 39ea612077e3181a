/*
 * rsi_mlp.h -- C ABI of the learned surrogate of the RSI field (not part of the paper).
 *
 * A coordinate MLP maps q = (x, z_below, f, depth, tilt) -- a field point in the x-z plane
 * below a planar water/solid interface at z = depth, for a piston tilted by `tilt` about
 * y at frequency f -- to two numbers y = (y0, y1) from which the field is rebuilt around
 * a computed carrier: the refracted plane wave of the beam axis (rsi_surrogate_carrier),
 * or the ray-tracing model of the piston (rsi_ray_field, eq. 12) with the network
 * learning the RSI field's departure from it (rsi_surrogate_ray_frame).  The RSI model
 * (rsi.h) produces the training fields and stays the fallback and judge of the
 * surrogate.
 *
 * Network: u = B v (B fixed [m][5], v = affine image of q on its box in [-1, 1]^5),
 * h0 = [sin 2 pi u, cos 2 pi u] (2m features), h_l = silu(W_l h_{l-1} + b_l) for
 * l = 1..L (width W), y = Wo h_L + bo (2 outputs).  The hidden layers run as bfloat16
 * MFMA GEMMs with FP32 accumulation (operands W_l, h_l in bfloat16; FP32 master weights);
 * features, head, loss and Adam run in FP32.  Loss: sum_b |y_b - t_b|^2 / (2 n).
 *
 * Flat parameter order (FP32): W_1 [W][2m], b_1 [W], W_2 [W][W], b_2, ..., W_L, b_L,
 * Wo [2][W], bo [2].  Limits: 2m and W multiples of 64, 2m <= 1024, W <= 1024,
 * 1 <= L <= 16; batches of up to max_batch rows (padded internally to 64).
 *
 * Conventions as in rsi.h: device pointers unless marked host, asynchronous on
 * `stream`, rsi_status returns, argument errors before any work.  An rsi_mlp object
 * may be used by one stream at a time.
 */
#ifndef RSI_MLP_H
#define RSI_MLP_H

#include <stdint.h>

#include "rsi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsi_mlp rsi_mlp;

/* Create a network and its training workspace on the current device.  B: host float
 * [n_ff][5]; lo, hi: host float[5], the box of q.  Parameters start at zero (set them
 * with rsi_mlp_set_params).  RSI_ERR_ARG for unsupported dimensions.  The workspace,
 * for Mp = max_batch padded to 64: bf16 activations of every layer and FP32
 * pre-activations (Mp (2m + L W) x 2 + Mp L W x 4 bytes), two bf16 gradient buffers, and
 * every layer's FP32 weight-gradient partials over up to 128 batch splits (128 x W x
 * (2m + (L - 1) W) x 4 bytes); about 1.0 GB for L = 7, W = 256, m = 128, max_batch 65536. */
rsi_status rsi_mlp_create(rsi_mlp **net, int n_ff, int width, int depth, const float *B,
                          const float *lo, const float *hi, int64_t max_batch);
rsi_status rsi_mlp_destroy(rsi_mlp *net);

/* Number of FP32 parameters in the flat order above. */
int64_t rsi_mlp_num_params(const rsi_mlp *net);

/* Copy the flat FP32 parameters from / to host memory (synchronous).  set_params also
 * refreshes the bfloat16 copies and resets the Adam state and step counter. */
rsi_status rsi_mlp_set_params(rsi_mlp *net, const float *host_params);
rsi_status rsi_mlp_get_params(const rsi_mlp *net, float *host_params);

/* y [n][2] = network(q [n][5]); n <= max_batch. */
rsi_status rsi_mlp_forward(rsi_mlp *net, int64_t n, const float *q, float *y, void *stream);

/* Loss and gradients (flat order, device float[num_params]) for targets t [n][2];
 * loss: device float[1] or NULL.  Parameters are not changed. */
rsi_status rsi_mlp_gradients(rsi_mlp *net, int64_t n, const float *q, const float *t,
                             float *grad, float *loss, void *stream);

/* One training step: gradients as above, then Adam (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected, step counter advanced) with learning rate lr on the FP32 master
 * parameters, then the bfloat16 copies are refreshed. */
rsi_status rsi_mlp_train_step(rsi_mlp *net, int64_t n, const float *q, const float *t,
                              float lr, float *loss, void *stream);

/* Checkpoint: dimensions, step counter, parameters and both Adam moments in one file
 * (synchronises the device).  load requires a network of the same dimensions. */
rsi_status rsi_mlp_save(const rsi_mlp *net, const char *path);
rsi_status rsi_mlp_load(rsi_mlp *net, const char *path);

/* Carrier of the surrogate for media (c1, rho1) -> (c2, rho2): for each q [n][5]
 *   mode 0 (demodulate): out[i] = in[i] * exp(-i psi(q_i)) / scale   (field -> envelope)
 *   mode 1 (modulate):   out[i] = in[i] * exp(+i psi(q_i)) * scale   (envelope -> field)
 * in/out: complex FP32 [n] (may alias).  psi as above (computed in FP64 and reduced to
 * one revolution).  scale = rho1 c1 (a pressure per unit velocity). */
rsi_status rsi_surrogate_carrier(int64_t n, const float *q, rsi_medium m1, rsi_medium m2,
                                 int mode, const float *in, float *out, void *stream);

/* Ray-model frame of the surrogate.  p_ray: the ray-tracing field (rsi_ray_field) at the
 * same n points; s: the RMS of ref [n_ref], the ray field of the same configuration on a
 * fixed set of points (n_ref >= 1).  For each point i, with u_i = p_ray[i] / |p_ray[i]|
 * (|p_ray[i]| below 1e-30 s counts as 1e-30 s):
 *   mode 0 (field -> frame): out[i] = (in[i] - p_ray[i]) conj(u_i) / (s sigma), its
 *                            magnitude capped at `clip` when clip > 0 (training targets:
 *                            configurations where the ray model fails do not swamp the
 *                            loss; they fail validation and fall back to RSI anyway)
 *   mode 1 (frame -> field): out[i] = p_ray[i] + s sigma in[i] u_i   (clip unused)
 * The network then learns the RSI field's departure from the ray model in the frame of
 * the ray's phase, scaled so that the squared error summed over a configuration's points
 * is its squared rel-L2 (up to a constant).  All arrays complex FP32 (out may alias in).
 * RSI_ERR_ARG for sigma <= 0, a non-finite clip or an unknown mode. */
rsi_status rsi_surrogate_ray_frame(int64_t n, const float *p_ray, int64_t n_ref, const float *ref,
                                   double sigma, double clip, int mode, const float *in,
                                   float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RSI_MLP_H */
