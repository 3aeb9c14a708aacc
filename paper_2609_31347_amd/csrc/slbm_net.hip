// Convolution kernels of the learned warm start (gfx950): 3x3 convolutions as
// implicit GEMMs on MFMA (bf16 inputs, FP32 accumulation), their backward
// passes, a masked MSE and Adam.  See include/solid_lbm_net.h.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "solid_lbm_net.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// FP32 -> bfloat16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__host__ __device__ inline int kpad(int K) { return (K + 7) / 8 * 8; }

// One wave = 32 output channels x 32 pixels of one image.  The GEMM runs over
// k = (ci, tap) in slices of 8: A (weights, rows = output channels) and B
// (the input gathered at the 3x3 offsets, columns = pixels) feed
// v_mfma_f32_32x32x8bf16_1k.  Operand lanes: A row = lane % 32, k = 4 (lane / 32) + j;
// B column = lane % 32, same k; result register r of lane l holds row
// 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
__global__ __launch_bounds__(64) void k_conv_fwd(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w,
                                                const float* __restrict__ bias, float* __restrict__ y,
                                                uint16_t* __restrict__ yb, int Cin, int Cout, int H, int W,
                                                int Kp, int relu, int dil)
{
    const int HW = H * W;
    const int p0 = blockIdx.x * 32, b = blockIdx.y;
    const int lane = threadIdx.x, col = lane & 31, kq = (lane >> 5) * 4;
    const int p = p0 + col;
    const bool pv = p < HW;
    const int py = pv ? p / W : 0, px = pv ? p - py * W : 0;
    const int K = Cin * 9;
    const uint16_t* xb = x + (int64_t)b * Cin * HW;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    for (int kb = 0; kb < Kp; kb += 8) {
        bf16x4 av, bv;
        const uint16_t* wr = w + (int64_t)col * Kp + kb + kq;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            av[j] = (short)wr[j];
            const int k = kb + kq + j;
            short v = 0;
            if (pv && k < K) {
                const int ci = k / 9, tap = k - ci * 9;
                const int yy = py + (tap / 3 - 1) * dil, xx = px + (tap % 3 - 1) * dil;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = (short)xb[(int64_t)ci * HW + yy * W + xx];
            }
            bv[j] = v;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
    }
    if (!pv) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int co = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (co < Cout) {
            float v = acc[r] + (bias ? bias[co] : 0.0f);
            if (relu) v = v > 0.0f ? v : 0.0f;
            const int64_t o = ((int64_t)b * Cout + co) * HW + p;
            y[o] = v;
            if (yb) yb[o] = f2bf(v);
        }
    }
}

// dw[co][ci][tap] and db[co] (taps at dilation dil): one block per (co, ci); fixed striding and a
// fixed reduction tree (deterministic).
__global__ __launch_bounds__(256) void k_conv_bwd_w(const float* __restrict__ dz, const uint16_t* __restrict__ x,
                                                   float* __restrict__ dw, float* __restrict__ db, int B, int Cin,
                                                   int Cout, int H, int W, int dil)
{
    const int co = blockIdx.x, ci = blockIdx.y;
    const int HW = H * W;
    const int64_t total = (int64_t)B * HW;
    float acc[10];
#pragma unroll
    for (int t = 0; t < 10; ++t) acc[t] = 0.0f;
    for (int64_t i = threadIdx.x; i < total; i += 256) {
        const int b = (int)(i / HW), p = (int)(i - (int64_t)b * HW);
        const float g = dz[((int64_t)b * Cout + co) * HW + p];
        const int py = p / W, px = p - py * W;
        const uint16_t* xc = x + ((int64_t)b * Cin + ci) * HW;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int yy = py + (tap / 3 - 1) * dil, xx = px + (tap % 3 - 1) * dil;
            if (yy >= 0 && yy < H && xx >= 0 && xx < W) acc[tap] += g * bf2f(xc[yy * W + xx]);
        }
        acc[9] += g;
    }
    __shared__ float red[10][256];
#pragma unroll
    for (int t = 0; t < 10; ++t) red[t][threadIdx.x] = acc[t];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int t = 0; t < 10; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 9) dw[(int64_t)co * Cin * 9 + ci * 9 + threadIdx.x] = red[threadIdx.x][0];
    if (threadIdx.x == 9 && ci == 0 && db) db[co] = red[9][0];
}

__global__ void k_act_bwd(const float* __restrict__ dy, const float* __restrict__ y, float* __restrict__ dz,
                          uint16_t* __restrict__ dzb, int64_t n, int relu)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = relu ? (y[i] > 0.0f ? dy[i] : 0.0f) : dy[i];
    if (dz) dz[i] = v;
    if (dzb) dzb[i] = f2bf(v);
}

__global__ void k_pack(const float* __restrict__ w32, uint16_t* __restrict__ wp, uint16_t* __restrict__ wt,
                       int Cin, int Cout)
{
    const int K = Cin * 9, Kp = kpad(K);
    const int Kt = Cout * 9, Ktp = kpad(Kt);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 32 * Kp) {
        const int co = i / Kp, k = i - co * Kp;
        wp[i] = (co < Cout && k < K) ? f2bf(w32[co * K + k]) : (uint16_t)0;
    }
    if (wt && i < 32 * Ktp) {
        // data gradient: conv with Cout inputs and Cin outputs, taps flipped
        const int ci = i / Ktp, k = i - ci * Ktp;
        uint16_t v = 0;
        if (ci < Cin && k < Kt) {
            const int co = k / 9, tp = k - co * 9;
            v = f2bf(w32[co * K + ci * 9 + (8 - tp)]);
        }
        wt[i] = v;
    }
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

__global__ void k_mse_grad(const float* __restrict__ y, const float* __restrict__ t, const float* __restrict__ mask,
                           float* __restrict__ dy, int nc, int64_t HW, int64_t n, double inv_norm)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t b = i / (nc * HW), p = i % HW;
    const float m = mask[b * HW + p];
    dy[i] = (float)(2.0 * inv_norm) * m * (y[i] - t[i]);
}

// loss = sum mask (y - t)^2 * inv_norm, one block, fixed order
__global__ __launch_bounds__(1024) void k_mse_loss(const float* __restrict__ y, const float* __restrict__ t,
                                                  const float* __restrict__ mask, double* __restrict__ loss, int nc,
                                                  int64_t HW, int64_t n, double inv_norm)
{
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const int64_t b = i / (nc * HW), p = i % HW;
        const double d = (double)y[i] - (double)t[i];
        s += (double)mask[b * HW + p] * d * d;
    }
    __shared__ double red[1024];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 512; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] * inv_norm;
}

__global__ __launch_bounds__(1024) void k_mask_sum(const float* __restrict__ mask, int64_t n, double* __restrict__ out)
{
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) s += mask[i];
    __shared__ double red[1024];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 512; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int status(hipError_t e) { return e == hipSuccess ? 0 : -3; }

}  // namespace

extern "C" {

int slbm_conv3x3_forward(const uint16_t* x, const uint16_t* w, const float* bias, float* y, uint16_t* y_bf16,
                         int32_t B, int32_t Cin, int32_t Cout, int32_t H, int32_t W, int32_t relu, int32_t dilation,
                         void* stream)
{
    if (!x || !w || !y || B < 1 || Cin < 1 || Cout < 1 || Cout > 32 || H < 1 || W < 1 || dilation < 1) return -1;
    dim3 grid(blocks((int64_t)H * W, 32), (unsigned)B);
    hipLaunchKernelGGL(k_conv_fwd, grid, dim3(64), 0, (hipStream_t)stream, x, w, bias, y, y_bf16, Cin, Cout, H, W,
                       kpad(Cin * 9), relu, dilation);
    return status(hipGetLastError());
}

int slbm_conv3x3_backward_weight(const float* dz, const uint16_t* x, float* dw, float* db, int32_t B, int32_t Cin,
                                 int32_t Cout, int32_t H, int32_t W, int32_t dilation, void* stream)
{
    if (!dz || !x || !dw || B < 1 || Cin < 1 || Cout < 1 || H < 1 || W < 1 || dilation < 1) return -1;
    hipLaunchKernelGGL(k_conv_bwd_w, dim3((unsigned)Cout, (unsigned)Cin), dim3(256), 0, (hipStream_t)stream, dz, x,
                       dw, db, B, Cin, Cout, H, W, dilation);
    return status(hipGetLastError());
}

int slbm_act_backward(const float* dy, const float* y, float* dz, uint16_t* dz_bf16, int64_t n, int32_t relu,
                      void* stream)
{
    if (!dy || (relu && !y) || n < 0) return -1;
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_act_bwd, dim3(blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, dy, y, dz, dz_bf16, n,
                       relu);
    return status(hipGetLastError());
}

int slbm_pack_weights(const float* w32, uint16_t* wp, uint16_t* wt, int32_t Cin, int32_t Cout, void* stream)
{
    if (!w32 || !wp || Cin < 1 || Cin > 32 || Cout < 1 || Cout > 32) return -1;
    int n = 32 * (kpad(Cin * 9) > kpad(Cout * 9) ? kpad(Cin * 9) : kpad(Cout * 9));
    hipLaunchKernelGGL(k_pack, dim3(blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, w32, wp, wt, Cin, Cout);
    return status(hipGetLastError());
}

int slbm_to_bf16(const float* x, uint16_t* y, int64_t n, void* stream)
{
    if (!x || !y || n < 0) return -1;
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, x, y, n);
    return status(hipGetLastError());
}

int slbm_mse(const float* y, const float* t, const float* mask, float* dy, double* loss, int32_t B, int32_t nc,
             int64_t HW, void* stream)
{
    if (!y || !t || !mask || !dy || B < 1 || nc < 1 || HW < 1) return -1;
    hipStream_t s = (hipStream_t)stream;
    // normalisation: nc * sum(mask), computed on the device into loss[0] first
    double* tmp = loss;
    if (!tmp) return -1;
    hipLaunchKernelGGL(k_mask_sum, dim3(1), dim3(1024), 0, s, mask, (int64_t)B * HW, tmp);
    double msum = 0.0;
    hipError_t e = hipMemcpyAsync(&msum, tmp, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return -3;
    if (!(msum > 0.0)) return -1;
    const double inv = 1.0 / (nc * msum);
    const int64_t n = (int64_t)B * nc * HW;
    hipLaunchKernelGGL(k_mse_grad, dim3(blocks(n, 256)), dim3(256), 0, s, y, t, mask, dy, nc, HW, n, inv);
    hipLaunchKernelGGL(k_mse_loss, dim3(1), dim3(1024), 0, s, y, t, mask, loss, nc, HW, n, inv);
    return status(hipGetLastError());
}

int slbm_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2, float eps,
              int32_t t, void* stream)
{
    if (!w || !g || !m || !v || n < 0 || t < 1) return -1;
    if (n == 0) return 0;
    float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, w, g, m, v, n, lr, beta1,
                       beta2, eps, c1, c2);
    return status(hipGetLastError());
}

}  // extern "C"
