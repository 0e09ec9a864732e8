/* Learned coarse-time surrogate for batches of shock tubes.
 *
 * The paper has no learned component: this is the learned part of the
 * workload built around the lattice BGK method (section "The Gaussian
 * quadrature" for the step, section "Numerical simulations for electrons in
 * metals" for the shock tubes).  A small 1D convolutional network maps the
 * row-averaged profiles (n, u_x) of a tube of length L to the profiles a fixed
 * number of lattice steps later; the lattice method is both its training-data
 * generator and its fallback.
 *
 * Network (parameters one flat float32 vector, 42754 values, in the order
 * W1 b1 W2 b2 W3 b3 W4 b4, each W laid out [tap][c_out][c_in]):
 *   features x = ((n - 1)/0.25, u/0.25, (tau - 0.75)/0.25)
 *   z1 = conv(x,  W1, b1, dilation 1)   3 -> 64, a1 = GELU(z1)
 *   z2 = conv(a1, W2, b2, dilation 3)  64 -> 64, a2 = GELU(z2)
 *   z3 = conv(a2, W3, b3, dilation 9)  64 -> 64, a3 = GELU(z3)
 *   y  = conv(a3, W4, b4, dilation 27) 64 -> 2
 *   n' = n + 0.25 y0, u' = u + 0.25 y1
 * conv(a, W, b, d)[c_out, x] = b[c_out] + sum_{tap, c_in} W[tap][c_out][c_in] a[c_in, x + (tap - 2) d],
 * kernel 5, zero outside [0, L); GELU(z) = z Phi(z) with the normal CDF Phi.
 * Weights and the hidden activations are stored in bfloat16 (round to
 * nearest even of the float32 value), accumulation is float32; the 64 -> 64
 * layers and their gradients run on the bf16 matrix cores.
 *
 * Profiles: float32 device arrays [batch][2][L], field 0 = n, field 1 = u_x,
 * x fastest (the layout lbm_batch_profiles writes).  tau: float32 device
 * array [batch].  L (the context's length) is a multiple of 128.
 *
 * Conventions as in lbm.h: the context borrows its device workspace until
 * srg_free; calls are asynchronous on the context's stream unless marked as
 * synchronizing; LBM_ERR_ARG for invalid arguments, LBM_ERR_HIP for HIP
 * failures, with the text in lbm_last_error().
 */
#ifndef PAPER_1510_07328_SRG_H
#define PAPER_1510_07328_SRG_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct srg_ctx_s *srg_ctx;

/* Number of network parameters (42754). */
lbm_status srg_param_count(int64_t *n);

/* Device workspace for batches of up to max_batch profiles of length `length`
 * (a multiple of 128): parameters, Adam state, bf16 weight copies, the
 * activations of one forward pass, gradient scratch and the hybrid advance's
 * fallback counts. */
lbm_status srg_workspace_bytes(int max_batch, int length, size_t *bytes);

/* Create a context on `stream` over a 256-byte-aligned device workspace of at
 * least srg_workspace_bytes() bytes (borrowed until srg_free).  Parameters are
 * undefined until srg_set_params. */
lbm_status srg_create(int max_batch, int length, void *workspace, size_t bytes, void *stream, srg_ctx *out);

/* Load the float32 parameter vector from device memory and reset the Adam
 * state (moments and step count) to zero.  Synchronizes. */
lbm_status srg_set_params(srg_ctx c, const float *params_dev);

/* Copy the float32 master parameters into a device buffer. */
lbm_status srg_get_params(srg_ctx c, float *params_dev);

/* out = network(profiles, tau) for `batch` profiles (1 <= batch <= max_batch).
 * Keeps the activations for a following srg_backward.  The inputs must stay
 * unchanged until that backward has run. */
lbm_status srg_forward(srg_ctx c, const float *prof_dev, const float *tau_dev, int batch, float *out_dev);

/* Inference: the same out as srg_forward, bit for bit, from one kernel that
 * keeps every activation in LDS (one workgroup per profile, or per two profiles
 * when the batch exceeds the device's compute units and 2 L <= 4096; lengths up
 * to 4096, longer ones run layer by layer); nothing is kept for a backward pass (a
 * following srg_backward needs a new srg_forward).
 * prof_dev [batch][2][L] and tau_dev [batch] float32 on the device, out_dev
 * [batch][2][L], which must not alias prof_dev.  LBM_ERR_ARG for a batch
 * outside [1, max_batch] or null pointers. */
lbm_status srg_infer(srg_ctx c, const float *prof_dev, const float *tau_dev, int batch, float *out_dev);

/* Gradient of a scalar loss with respect to the parameters, given dout = dLoss/d out
 * ([batch][2][L] float32, device) of the latest srg_forward; writes the flat
 * float32 gradient (srg_param_count values) to grad_dev.  LBM_ERR_STATE
 * without a preceding forward. */
lbm_status srg_backward(srg_ctx c, const float *dout_dev, float *grad_dev);

/* Training loss of predictions against targets (both [batch][2][L]):
 * e = (out - target)/0.25 over both fields,
 * loss = mean(e^2) + lambda_mass * mean_b (mean_x e_n)^2;
 * writes dLoss/d out to dout_dev and, if loss_host is not NULL, the loss
 * (then synchronizes). */
lbm_status srg_loss(srg_ctx c, const float *out_dev, const float *target_dev, int batch, float lambda_mass,
                    float *dout_dev, double *loss_host);

/* One Adam step (bias-corrected; the step count is kept by the context) on the
 * float32 master parameters with the gradient grad_dev, then refresh of the
 * bf16 copies. */
lbm_status srg_adam(srg_ctx c, const float *grad_dev, float lr, float b1, float b2, float eps);

/* srg_forward + srg_loss + srg_backward + srg_adam (b1 0.9, b2 0.999, eps 1e-8)
 * on one minibatch.  Synchronizes when loss_host is not NULL. */
lbm_status srg_train_step(srg_ctx c, const float *prof_dev, const float *tau_dev, const float *target_dev, int batch,
                          float lr, float lambda_mass, double *loss_host);

/* Per-profile relative mass residual |sum_x n_out - sum_x n_in| / sum_x n_in
 * into resid_dev[batch] (float32). */
lbm_status srg_mass_residual(srg_ctx c, const float *in_dev, const float *out_dev, int batch, float *resid_dev);

/* Advance a batch of tubes (all of length L, at most max_batch of them, d2v9,
 * created with lbm_batch_init on the same stream as the context) by `jumps`
 * coarse steps of `jump_steps` lattice steps each.  Per jump: the profile of
 * every tube, one network jump and its indicator per tube, which is the
 * relative mass residual, or +inf when a predicted value is not finite or a
 * predicted density is not positive.  A tube whose indicator is <= mass_tol
 * takes the prediction (n', u') as its state; the others are advanced by
 * jump_steps lattice steps from their state before the jump.  A tube's profile
 * is its populations' row-averaged n, u when its last jump ran on the lattice
 * (or there was none), else the prediction itself; its populations are set to
 * f = f_eq(n', (u', 0)) on every row when a later jump falls back to the
 * lattice, and by the end of the call for every tube whose last jump was
 * accepted.  On an error return the populations of accepted tubes may be
 * stale.  fallback_host (may be NULL)
 * receives the number of fallback tubes per jump (`jumps` ints).  A negative
 * mass_tol sends every tube to the lattice method.  The accept/reject decision
 * is taken on the device and every jump is queued without waiting for it: the
 * call synchronizes once at the start and, when fallback_host is not NULL,
 * after every 1024 jumps and at the end to read the counts back; with
 * fallback_host NULL it returns with the work still queued on the stream.
 * jump_steps in [1, 2^30).
 * LBM_ERR_UNSUPPORTED for tubes of unequal length or a length other than the
 * context's. */
lbm_status srg_hybrid_advance(srg_ctx c, lbm_batch b, const float *tau_dev, int ntubes, int jumps, int jump_steps,
                              float mass_tol, int *fallback_host);

/* Release the context (not the workspace).  Synchronizes the stream. */
lbm_status srg_free(srg_ctx c);

/* Inference without a context, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid it): the
 * same out as srg_infer on a context holding the same parameters, bit for bit,
 * with no workspace and no allocation of any kind.
 *   params_dev: the flat float32 parameter vector (srg_param_count values), device;
 *   prof_dev [batch][2][length], tau_dev [batch], out_dev [batch][2][length]:
 *              float32 device arrays as for srg_infer (out must not alias prof);
 *   stream:    hipStream_t to enqueue on (NULL = null stream).  Asynchronous.
 * Its scratch is the bfloat16 copy of the weights (about 85 KB) in a static
 * device array the library holds on each GPU it runs on until the process ends;
 * every call rewrites it from params_dev, so calls on one GPU that overlap in
 * time (on different streams or threads) race and must be serialized by the
 * caller.  length must be a multiple of 128 and at most 4096 (the one-kernel
 * inference; longer profiles need activation buffers): LBM_ERR_ARG otherwise,
 * and for batch < 1 or null pointers.  LBM_ERR_HIP on a HIP failure. */
lbm_status srg_infer_noalloc(const float *params_dev, const float *prof_dev, const float *tau_dev, int batch,
                             int length, float *out_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif
