/* Learned warm start for altGDmin: a small CNN that maps the zero-filled,
 * coil-combined frames of a sequence to an initial basis (then QR), with
 * hand-written HIP training kernels.  The fallback to the spectral
 * initialisation is altgdmin_init_warm in altgdmin.h.
 *
 * Network: 4 convolutions 3x3, stride 1, zero "same" padding, with bias:
 *   conv(2q -> width) ReLU, conv(width -> width) ReLU,
 *   conv(width -> width) ReLU, conv(width -> 2r);
 * input: the 2q planes of altgdmin_cnn_input; output channel 2j is Re and
 * 2j+1 is Im of column j of M (n x r).  The target is a converged basis
 * U_tgt; the loss is the squared subspace distance of span(M) to
 * span(U_tgt) (the paper's SD, Sec. II-A), L = r - tr(G^-1 C C^H) with
 * G = M^H M, C = M^H U_tgt, which only depends on span(M).
 *
 * Conventions (as in altgdmin.h): device pointers, caller-owned memory,
 * asynchronous on the stream given to wsinit_create, status codes of
 * altgdmin_status; the library never allocates device memory.
 *   parameters  FP32, layer by layer: W[cout][cin][3][3] then b[cout];
 *   d_in        FP32 [batch][2q][ny][nx];
 *   d_M, d_Ut   complex64 [batch][r][n] (each n x r column-major);
 *   d_ws        workspace of wsinit_workspace_bytes, 256-byte aligned.
 * Limits: nx, ny multiples of 8 (<= 512), 1 <= q <= 128, 1 <= r <= 16,
 * 4 <= width <= 32, layers = 4, 1 <= batch <= 64.
 */
#ifndef WSINIT_H
#define WSINIT_H

#include "altgdmin.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wsinit_ctx wsinit_ctx;

/* Shapes and the largest batch a call may use.  stream: hipStream_t (NULL =
 * default stream).  Host only. */
altgdmin_status wsinit_create(int32_t nx, int32_t ny, int32_t q, int32_t r, int32_t width, int32_t layers,
                              int32_t batch, void* stream, wsinit_ctx** out);

/* Number of FP32 parameters (49,644 for q = 48, r = 6, width 32). */
altgdmin_status wsinit_param_count(const wsinit_ctx* ctx, int64_t* count);

/* Workspace bytes for the largest batch (activations kept for the
 * backward pass, packed weights, gradient partials). */
altgdmin_status wsinit_workspace_bytes(const wsinit_ctx* ctx, size_t* bytes);

/* Forward pass of `batch` sequences: d_M[b] = network output as n x r
 * complex. */
altgdmin_status wsinit_forward(wsinit_ctx* ctx, const float* d_params, const float* d_in, int32_t batch, void* d_M,
                               void* d_ws);

/* Forward, loss and backward of `batch` sequences with targets d_Ut:
 * *d_loss (device FP64) = mean loss, d_grads = gradient of the mean loss
 * (parameter layout). */
altgdmin_status wsinit_loss_backward(wsinit_ctx* ctx, const float* d_params, const float* d_in, const void* d_Ut,
                                     int32_t batch, float* d_grads, double* d_loss, void* d_ws);

/* One Adam update (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step
 * counts from 1) of d_params with d_grads; d_m, d_v are the moment buffers
 * (zero before step 1). */
altgdmin_status wsinit_adam_step(wsinit_ctx* ctx, float* d_params, const float* d_grads, float* d_m, float* d_v,
                                 float lr, int32_t step);

void wsinit_destroy(wsinit_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif
