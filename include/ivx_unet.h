/*
 * ivx_unet — the learned warm start of the Classic3D solve: a 4-level U-Net (Ronneberger
 * et al. 2015) mapping the normalised dirty mosaic d = -grad Q(0) / max|d| to an initial
 * sky x0 / 50 K, trained on converged cold-start solutions of the same objective.  All
 * layers run in hand-written gfx950 kernels: 3x3 convolutions as implicit GEMMs on the
 * bf16 matrix cores (v_mfma_f32_16x16x16_bf16) with bf16 weights and activations rounded
 * to bf16 on load, FP32 accumulation and FP32 master weights; pooling, nearest upsampling,
 * concatenation, ReLU, the 1x1 head, MSE and Adam in FP32 vector code.
 *
 * Layouts: activations NHWC float ([n][y][x][c]); 3x3 weights [out][3][3][in] (bf16 bits
 * as uint16 where noted); the network input and output are [batch][height][width] float
 * (one channel).  Device pointers unless stated.  All calls are asynchronous on `stream`
 * (a hipStream_t as void*) unless a host pointer receives a result.  Status codes and
 * ivx_last_error() are those of ivx.h.
 */
#ifndef IVX_UNET_H
#define IVX_UNET_H

#include <stdint.h>

#include "ivx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ivx_unet ivx_unet;

/* levels in [1, 5], base channels multiple of 16, height/width divisible by 2^(levels-1),
 * max_batch >= 1.  Parameters are initialised from `seed` (He-normal weights, zero biases).
 * Allocates all activation, gradient and optimiser buffers up front. */
ivx_status ivx_unet_create(int32_t levels, int32_t base, int32_t max_batch, int32_t height,
                           int32_t width, uint64_t seed, ivx_unet **out);
ivx_status ivx_unet_destroy(ivx_unet *net);

/* Number of FP32 master parameters (order: per 3x3 conv weight [out][3][3][in] then bias,
 * encoder levels top-down, decoder levels bottom-up, then the 1x1 head weight and bias). */
int64_t ivx_unet_param_count(const ivx_unet *net);
/* Copy the FP32 master parameters out / in (host or device pointer, param_count floats);
 * set_params also refreshes the bf16 copies and resets the Adam state. */
ivx_status ivx_unet_get_params(const ivx_unet *net, float *params);
ivx_status ivx_unet_set_params(ivx_unet *net, const float *params);

/* y = net(x), x and y [batch][height][width], batch <= max_batch. */
ivx_status ivx_unet_forward(ivx_unet *net, const float *x, float *y, int32_t batch, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the MSE between net(x) and target;
 * *loss (host or device double, may be NULL) receives the loss before the update. */
ivx_status ivx_unet_train_step(ivx_unet *net, const float *x, const float *target, int32_t batch,
                               float lr, double *loss, void *stream);

/* Loss and gradient without an update: grads (host or device, param_count floats, same
 * order as the parameters) and *loss (host or device double, may be NULL). */
ivx_status ivx_unet_loss_grad(ivx_unet *net, const float *x, const float *target, int32_t batch,
                              float *grads, double *loss, void *stream);

/* ---- single layers, for checking against a reference (each call may allocate) ---- */

/* y = [mask > 0] * (conv3x3(x, W) + bias, ReLU if relu) (+ y if accumulate);
 * x [n][h][w][cin] (cin % 4 == 0), W bf16 bits [cout][3][3][cin] (cout % 16 == 0),
 * bias [cout] or NULL, mask [n][h][w][cout] or NULL. */
ivx_status ivx_nn_conv3x3(const float *x, int32_t n, int32_t h, int32_t w, int32_t cin,
                          const uint16_t *weight, const float *bias, int32_t cout, int32_t relu,
                          const float *mask, int32_t accumulate, float *y, void *stream);
/* Gradient of sum(dy * conv3x3(x, W)) with respect to W and bias (x and dy rounded to bf16
 * for the matrix cores, FP32 sums): dw [cout][3][3][cin], db [cout] (overwritten). */
ivx_status ivx_nn_conv3x3_grad_weight(const float *x, const float *dy, int32_t n, int32_t h,
                                      int32_t w, int32_t cin, int32_t cout, float *dw, float *db,
                                      void *stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving or training loops, harnesses that forbid hipMalloc): the same weight and bias
 * gradient as ivx_nn_conv3x3_grad_weight, same arguments and results, with its split
 * partials in a static device array of ivx_nn_conv3x3_grad_weight_noalloc_capacity()
 * floats (32 MiB, one copy per device, held until the process ends) instead of a buffer
 * allocated per call.  It calls no hipMalloc or hipFree and does not synchronise: the
 * work is queued on `stream`.  IVX_EINVAL (nothing launched) when the shape needs more
 * partials than the array holds (ivx_nn_conv3x3_grad_weight_scratch_floats gives the
 * need).  All calls on one device share its array: calls that overlap on one device
 * (other streams, other threads) race and must be ordered by the caller. */
ivx_status ivx_nn_conv3x3_grad_weight_noalloc(const float *x, const float *dy, int32_t n,
                                              int32_t h, int32_t w, int32_t cin, int32_t cout,
                                              float *dw, float *db, void *stream);
int64_t ivx_nn_conv3x3_grad_weight_noalloc_capacity(void);
/* Floats of split partials the weight gradient needs for this shape (-1 if invalid). */
int64_t ivx_nn_conv3x3_grad_weight_scratch_floats(int32_t n, int32_t h, int32_t w, int32_t cin,
                                                  int32_t cout);

/* Weights of the transposed correlation: wt[c][a][b][o] = W[o][2-a][2-b][c] (bf16 bits). */
ivx_status ivx_nn_conv3x3_flip(const uint16_t *weight, int32_t cin, int32_t cout, uint16_t *flipped,
                               void *stream);
/* Round FP32 to bf16 bits (nearest even). */
ivx_status ivx_nn_to_bf16(const float *x, int64_t count, uint16_t *out, void *stream);
/* 2x2 max pool and its gradient (to the first maximum, (0,0),(0,1),(1,0),(1,1) order;
 * accumulate adds into dx). */
ivx_status ivx_nn_pool2(const float *x, int32_t n, int32_t h, int32_t w, int32_t c, float *y,
                        void *stream);
ivx_status ivx_nn_pool2_grad(const float *x, const float *dy, int32_t n, int32_t h, int32_t w,
                             int32_t c, int32_t accumulate, float *dx, void *stream);
/* Nearest 2x upsampling of [n][h][w][c] and its gradient (sum over each 2x2 block). */
ivx_status ivx_nn_up2(const float *x, int32_t n, int32_t h, int32_t w, int32_t c, float *y,
                      void *stream);
ivx_status ivx_nn_up2_grad(const float *dy, int32_t n, int32_t h, int32_t w, int32_t c, float *dx,
                           void *stream);

#ifdef __cplusplus
}
#endif

#endif /* IVX_UNET_H */
