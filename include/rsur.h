/* rsur.h — C ABI of the learned stress surrogate of the r-cell library (MI355X, gfx950).
 *
 * The coupling of arXiv:1902.09171 obtains each quadrature point's stress from an MD r-cell
 * (Sec. 2.1, Fig. 1).  The surrogate replaces most of those MD runs by a small network trained on
 * r-cell data: an ensemble of K multilayer perceptrons mapping a normalised deformation history
 * (din floats) to the normalised stress (dout floats), depth hidden layers of `width` units with
 * SiLU, linear output.  The spread of the ensemble flags inputs the networks have not learned, and
 * those points fall back to batched MD (rcell.h).
 *
 * Arithmetic: matrix products in BF16 on the matrix cores with FP32 accumulation; FP32 master
 * weights, Adam (beta1 0.9, beta2 0.999, eps 1e-8) in FP32; MSE loss on normalised outputs.
 *
 * Conventions as in rcell.h: int status (0 or a negative RCELL_ERR_* value), no exceptions,
 * host arrays copied at call time, *_dev pointers are caller-owned device memory used on the
 * context's stream.  Parameter layout of one member (host, FP32): for each layer l with fan-in
 * d_l and fan-out d_{l+1} (d_0 = din, hidden widths, d_L = dout): W_l as a d_l x d_{l+1}
 * row-major block (y = x W_l + b_l), then b_l.
 */
#ifndef RSUR_H
#define RSUR_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsur_ctx rsur_ctx;

/* Allocate a K-member ensemble for batches of up to max_batch rows on the current device.
 * Parameters start at zero: load them with rsur_set_params.  Normalisation starts as identity.
 * All device memory is allocated here (parameters, Adam moments, activations for max_batch rows,
 * and the partial sums of the training step's split reductions: 8 x K x the largest layer's
 * weights, in FP32); the forward and training calls allocate nothing. */
int rsur_create(int32_t din, int32_t width, int32_t depth, int32_t dout, int32_t ensemble,
                int32_t max_batch, void* hip_stream, rsur_ctx** out);
int rsur_destroy(rsur_ctx* ctx);
const char* rsur_last_error(const rsur_ctx* ctx);
/* number of parameters of one member (the length of the flat layout) */
int rsur_num_params(rsur_ctx* ctx, int64_t* n);

/* FP32 master parameters of one member from / to the host (flat layout above); setting them
 * also resets that member's Adam moments and step counter. */
int rsur_set_params(rsur_ctx* ctx, int32_t member, const float* w);
int rsur_get_params(rsur_ctx* ctx, int32_t member, float* w);
/* gradient of the last training step (same layout), for checks */
int rsur_get_grads(rsur_ctx* ctx, int32_t member, float* g);

/* input / output normalisation x_n = (x - x_mu) / x_sd, y = y_n * y_sd + y_mu (host arrays of
 * din and dout floats) */
int rsur_set_norm(rsur_ctx* ctx, const float* x_mu, const float* x_sd, const float* y_mu, const float* y_sd);
/* the same statistics computed on the device from n rows of training data (FP32, row-major
 * X_dev n x din, Y_dev n x dout; population standard deviation, floored at 1e-6) */
int rsur_fit_norm(rsur_ctx* ctx, const void* X_dev, const void* Y_dev, int32_t n);

/* Inference for B <= max_batch rows of raw inputs X_dev (B x din FP32): ensemble mean and
 * variance over members of the de-normalised outputs (B x dout FP32 each; var_dev may be NULL).
 * Enqueued only. */
int rsur_forward(rsur_ctx* ctx, const void* X_dev, int32_t B, void* mean_dev, void* var_dev);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same ensemble mean and variance as rsur_forward,
 * bit for bit, computed without any allocation.  The members' outputs go to a fixed device array of
 * 2^21 floats (8 MiB) that the library holds on each device it runs on until the process ends,
 * instead of the context's activation buffers, so B is limited by that array, not by max_batch:
 * 1 <= B and K * pad64(B) * pad64(dout) <= 2^21 (4096 rows for K = 8 and dout <= 64), else
 * RCELL_ERR_ARG.  Needs padded widths <= 256 and at most 8 layers (RCELL_ERR_ARG otherwise).  Every
 * call on one device shares that device's array: calls that overlap on one device (other streams,
 * other contexts, other host threads) race and must be serialised by the caller.  Enqueued only. */
int rsur_forward_static(rsur_ctx* ctx, const void* X_dev, int32_t B, void* mean_dev, void* var_dev);
/* every member's de-normalised output, K x B x dout FP32 (checks and diagnostics) */
int rsur_forward_members(rsur_ctx* ctx, const void* X_dev, int32_t B, void* out_dev);

/* One Adam step of every member on the same minibatch (raw X_dev B x din, raw Y_dev B x dout,
 * FP32), learning rate lr.  loss: host array of K floats receiving each member's MSE on the
 * normalised outputs before the step (synchronises), or NULL (enqueue only).  The reductions over
 * the minibatch (weight and bias gradients, loss) are split over blocks for large B and their
 * partial sums added in a fixed order, so a step is reproducible bit for bit. */
int rsur_train_step(rsur_ctx* ctx, const void* X_dev, const void* Y_dev, int32_t B, float lr, float* loss);

#ifdef __cplusplus
}
#endif
#endif
