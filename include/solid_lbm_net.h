/*
 * solid_lbm_net.h -- C ABI of the convolution kernels of the learned warm
 * start (a small 3x3 convolutional network that predicts an initial
 * displacement for the solid-LBM primal solve).
 *
 * The paper's method has no learned part; it starts every primal solve from
 * d_0 = 0.  These kernels only produce a better d_0: the solver, its FP64
 * arithmetic and its convergence test are unchanged, so the converged result
 * is the same fixed point (eq. primal_fixed_point) and the cold start stays
 * available.
 *
 * Conventions: all pointers are device memory on the current HIP device;
 * stream may be NULL (default stream).  Activations are NCHW; "bf16" buffers
 * hold bfloat16 bit patterns (uint16_t, round-to-nearest-even from FP32).
 * Weights of a layer with Cin inputs, Cout <= 32 outputs are packed as
 * bf16 [32][Kp] with K = Cin*9 entries per output channel ordered (ci, ky, kx),
 * Kp = K rounded up to a multiple of 16 (one k-slice of gfx950's
 * v_mfma_f32_32x32x16_bf16), unused rows/columns zero.  The convolutions run on
 * that MFMA (bf16 inputs, FP32 accumulation) with the weights and the input
 * rows a workgroup touches staged in LDS; the weight gradient runs on the
 * FP32 MFMA (FP32 dz times the bf16 input, exact products, FP32 sums in a
 * fixed order).  Every call returns
 * 0 or a negative SLBM_* code (-1 bad arguments, -3 HIP error); the kernels
 * allocate nothing.
 */
#ifndef SOLID_LBM_NET_H
#define SOLID_LBM_NET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* y[b][co][p] = act(bias[co] + sum_{ci,ky,kx} W[co][ci][ky][kx] x[b][ci][p + dil (ky-1, kx-1)])
 * with zero padding at the image border; act = ReLU if relu != 0; dilation dil >= 1.
 * x: bf16 [B][Cin][H][W]; w: packed bf16 (see above); bias: FP32 [Cout] or NULL;
 * y: FP32 [B][Cout][H][W]; y_bf16: bf16 copy of y or NULL. */
int slbm_conv3x3_forward(const uint16_t *x, const uint16_t *w, const float *bias, float *y,
                         uint16_t *y_bf16, int32_t B, int32_t Cin, int32_t Cout, int32_t H, int32_t W,
                         int32_t relu, int32_t dilation, void *stream);

/* Weight gradient: dw[co][ci*9 + tap] = sum_b sum_p dz[b][co][p] x[b][ci][p + dil off(tap)],
 * db[co] = sum_b sum_p dz[b][co][p] (db may be NULL); dz FP32 [B][Cout][H][W]
 * (Cout <= 32), x bf16 [B][Cin][H][W]; dw FP32 [Cout][Cin*9] (unpacked).
 * Deterministic (fixed split of the pixels and fixed summation order). */
int slbm_conv3x3_backward_weight(const float *dz, const uint16_t *x, float *dw, float *db, int32_t B,
                                 int32_t Cin, int32_t Cout, int32_t H, int32_t W, int32_t dilation,
                                 void *stream);

/* dz = dy * (y > 0) (ReLU backward; relu == 0: dz = dy), also as bf16. n elements. */
int slbm_act_backward(const float *dy, const float *y, float *dz, uint16_t *dz_bf16, int64_t n,
                      int32_t relu, void *stream);

/* Packs FP32 weights w32 [Cout][Cin*9] into the bf16 MFMA layout (wp) and the
 * flipped, transposed layout of the data gradient (wt: the weights of the
 * convolution dx = conv(dz) with Cout inputs, Cin outputs and the same
 * dilation). wt may be NULL. */
int slbm_pack_weights(const float *w32, uint16_t *wp, uint16_t *wt, int32_t Cin, int32_t Cout, void *stream);

/* FP32 -> bf16 (round to nearest even), n elements. */
int slbm_to_bf16(const float *x, uint16_t *y, int64_t n, void *stream);

/* Masked mean squared error over nc channels: loss = sum mask (y - t)^2 / (nc * sum mask),
 * dy = d loss / d y.  y, t, dy: FP32 [B][nc][H*W]; mask FP32 [B][H*W];
 * loss: device double (required; also used as scratch for the mask sum).
 * Synchronises the stream once (to read the mask sum). */
int slbm_mse(const float *y, const float *t, const float *mask, float *dy, double *loss, int32_t B,
             int32_t nc, int64_t HW, void *stream);

/* Adam step on n FP32 parameters (first and second moments m, v; step t >= 1). */
int slbm_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
              float eps, int32_t t, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SOLID_LBM_NET_H */
