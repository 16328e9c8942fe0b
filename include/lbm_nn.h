/*
 * lbm_nn.h -- C ABI of the warm-start network kernels (gfx950, BF16 MFMA).
 *
 * The warm-start network maps a cavity's conduction state and its
 * parameters (log Ra, Pr, aspect ratio) to a developed convective state
 * (T, u) from which the lattice Boltzmann step of lbm.h starts.  These
 * entry points are its layers, forward and backward, for training on the
 * GPU; the model, data and optimiser loop live in the Python package.
 *
 * Conventions
 *   - Tensors are device pointers, caller-owned.  Activations and their
 *     gradients are BF16 (raw uint16_t bits), NHWC, with channel counts a
 *     multiple of 16; weights of a 3x3 convolution are BF16 [9][cout][cin]
 *     (tap = 3 ky + kx), biases and all weight gradients FP32.
 *   - Every kernel runs on `stream` (a hipStream_t, NULL = default) and the
 *     calls return without synchronising.  Products accumulate in FP32.
 *   - Return LBM_OK, LBM_E_INVALID for bad shapes or null pointers (message
 *     in lbm_nn_last_error), LBM_E_DEVICE if a launch fails.
 */
#ifndef LBM_NN_H
#define LBM_NN_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* y[n,i,j,o] = act(bias[o] + sum_{tap,k} w[tap][o][k] x[n, i+ky-1, j+kx-1, k]),
 * zero padding, act = ReLU if relu != 0.  bias may be NULL.  cin, cout
 * multiples of 16.                                                      */
lbm_status lbm_nn_conv3x3(const uint16_t* x, int32_t n, int32_t h, int32_t w, int32_t cin,
                          const uint16_t* wt, const float* bias, int32_t cout, int32_t relu,
                          uint16_t* y, void* stream);

/* wf[tap][k][o] = wt[8 - tap][o][k]: with it lbm_nn_conv3x3(dz, wf) gives
 * the input gradient of a convolution with weights wt.                  */
lbm_status lbm_nn_conv3x3_flip(const uint16_t* wt, int32_t cin, int32_t cout, uint16_t* wf,
                               void* stream);

/* Weight and bias gradients of a convolution with input x [n,h,w,cin] and
 * output gradient dz [n,h,w,cout]: dw [9][cout][cin] and db [cout] (FP32;
 * db may be NULL; with db, cout <= 256).  `partial` is scratch of
 * chunks * 9 * cout * cin floats; pixels are split into `chunks` ranges
 * summed in order, so the result does not depend on scheduling.         */
lbm_status lbm_nn_conv3x3_wgrad(const uint16_t* x, const uint16_t* dz, int32_t n, int32_t h,
                                int32_t w, int32_t cin, int32_t cout, float* partial,
                                int32_t chunks, float* dw, float* db, void* stream);

/* dz = dy where y > 0 (y is the ReLU output), else 0.                    */
lbm_status lbm_nn_relu_backward(const uint16_t* y, const uint16_t* dy, uint16_t* dz,
                                int64_t count, void* stream);

/* 2x2 mean pooling of x [n,h,w,c] (h, w even) into y [n,h/2,w/2,c], and its
 * gradient dx [n,h,w,c] from dy [n,h/2,w/2,c].                           */
lbm_status lbm_nn_avgpool2(const uint16_t* x, int32_t n, int32_t h, int32_t w, int32_t c,
                           uint16_t* y, void* stream);
lbm_status lbm_nn_avgpool2_backward(const uint16_t* dy, int32_t n, int32_t h, int32_t w,
                                    int32_t c, uint16_t* dx, void* stream);

/* nearest 2x upsampling of x [n,h,w,c] into y [n,2h,2w,c], and its
 * gradient dx [n,h,w,c] from dy [n,2h,2w,c].                             */
lbm_status lbm_nn_upsample2(const uint16_t* x, int32_t n, int32_t h, int32_t w, int32_t c,
                            uint16_t* y, void* stream);
lbm_status lbm_nn_upsample2_backward(const uint16_t* dy, int32_t n, int32_t h, int32_t w,
                                     int32_t c, uint16_t* dx, void* stream);

/* Channel slice copy for concatenation and its gradient:
 * dst[p][doff + k] = src[p][soff + k] (or += when accumulate != 0), k < cc,
 * p < pixels; cs, cd are the channel counts of src and dst.              */
lbm_status lbm_nn_copy_channels(const uint16_t* src, int32_t cs, int32_t soff, uint16_t* dst,
                                int32_t cd, int32_t doff, int32_t cc, int64_t pixels,
                                int32_t accumulate, void* stream);

/* Masked mean squared error over the first `used` channels of y [P][cy]:
 * loss[0] = sum mask (y - t)^2 / count, count = sum of mask; target and
 * mask are FP32 [P][used].  dy [P][cy] (BF16, nullable) receives the
 * gradient.  `scratch` holds 1024 floats.                               */
lbm_status lbm_nn_mse(const uint16_t* y, int32_t cy, const float* target, const float* mask,
                      int64_t pixels, int32_t used, double count, uint16_t* dy, float* loss,
                      float* scratch, void* stream);

/* One Adam step (Kingma & Ba 2015) on FP32 weights w with gradient g and
 * moments m, v; step >= 1 is the 1-based update count; w_bf16 (nullable)
 * receives the BF16 copy of the new weights.                            */
lbm_status lbm_nn_adam(float* w, const float* g, float* m, float* v, int64_t count, float lr,
                       float beta1, float beta2, float eps, int32_t step, uint16_t* w_bf16,
                       void* stream);

/* FP32 <-> BF16 (round to nearest even).                                */
lbm_status lbm_nn_to_bf16(const float* src, uint16_t* dst, int64_t count, void* stream);
lbm_status lbm_nn_to_f32(const uint16_t* src, float* dst, int64_t count, void* stream);

const char* lbm_nn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_NN_H */
