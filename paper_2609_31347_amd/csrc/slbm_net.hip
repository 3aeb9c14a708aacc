// Convolution kernels of the learned warm start (gfx950): 3x3 convolutions as
// implicit GEMMs on MFMA (bf16 inputs, FP32 accumulation), their backward
// passes, a masked MSE and Adam.  See include/solid_lbm_net.h.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "solid_lbm_net.h"

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short shortx8 __attribute__((ext_vector_type(8)));

// FP32 -> bfloat16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// K of the packed weights: rounded up to the 16 of one bf16 MFMA k-slice.
__host__ __device__ inline int kpad(int K) { return (K + 15) / 16 * 16; }

constexpr int kFwdPix = 128;                 // output pixels per workgroup (4 waves of 32)
constexpr int kFwdStage = 64 * 1024;         // LDS bytes for the staged input rows

// Rows of the image that the kFwdPix pixels from p0 (and their 3x3 taps at
// dilation dil) touch: [ylo, ylo + nrows).
__host__ __device__ inline void fwd_rows(int p0, int HW, int H, int W, int dil, int* ylo, int* nrows)
{
    const int p1 = min(p0 + kFwdPix, HW) - 1;
    const int y0 = max(0, p0 / W - dil), y1 = min(H - 1, p1 / W + dil);
    *ylo = y0;
    *nrows = y1 - y0 + 1;
}

// Upper bound of fwd_rows' count over all workgroups of a launch.
inline int fwd_rows_max(int H, int W, int dil) { return std::min(H, (kFwdPix + W - 1) / W + 1 + 2 * dil); }

// 3x3 convolution as an implicit GEMM on gfx950's v_mfma_f32_32x32x16_bf16:
// one wave = 32 output channels x 32 pixels of one image, four waves = 128
// consecutive pixels.  The packed weights (A, rows = output channels) and,
// when they fit (stage != 0), the input rows that the workgroup's taps touch
// are first copied into LDS; the B operand (the input at the 3x3 offsets,
// columns = pixels) is then gathered from LDS.  Operand lanes: row / column =
// lane % 32, k = 8 (lane / 32) + j, j < 8; result register r of lane l holds
// row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w,
                                                 const float* __restrict__ bias, float* __restrict__ y,
                                                 uint16_t* __restrict__ yb, int Cin, int Cout, int H, int W,
                                                 int Kp, int relu, int dil, int stage)
{
    extern __shared__ __align__(16) uint16_t smem[];
    uint16_t* wl = smem;                       // [32][Kp] weights
    uint16_t* xl = smem + 32 * Kp;             // [Cin][nrows][W] input rows (stage != 0)
    const int HW = H * W;
    const int P0 = blockIdx.x * kFwdPix, b = blockIdx.y;
    const uint16_t* xb = x + (int64_t)b * Cin * HW;
    int ylo = 0, nrows = 0;
    fwd_rows(P0, HW, H, W, dil, &ylo, &nrows);
    for (int i = threadIdx.x; i < 32 * Kp; i += 256) wl[i] = w[i];
    if (stage) {
        const int n = Cin * nrows * W;
        for (int i = threadIdx.x; i < n; i += 256) {
            const int ci = i / (nrows * W), r = i - ci * nrows * W;
            xl[i] = xb[(int64_t)ci * HW + (int64_t)ylo * W + r];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, col = lane & 31, kq = (lane >> 5) * 8;
    const int p = P0 + (threadIdx.x >> 6) * 32 + col;
    const bool pv = p < HW;
    const int py = pv ? p / W : 0, px = pv ? p - py * W : 0;
    const int K = Cin * 9;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    for (int kb = 0; kb < Kp; kb += 16) {
        const shortx8 av = *reinterpret_cast<const shortx8*>(wl + col * Kp + kb + kq);
        shortx8 bv;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = kb + kq + j;
            short v = 0;
            if (pv && k < K) {
                const int ci = k / 9, tap = k - ci * 9;
                const int yy = py + (tap / 3 - 1) * dil, xx = px + (tap % 3 - 1) * dil;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    v = (short)(stage ? xl[(ci * nrows + (yy - ylo)) * W + xx] : xb[(int64_t)ci * HW + yy * W + xx]);
            }
            bv[j] = v;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                      acc, 0, 0, 0);
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

// Weight gradient as a GEMM on the FP32 MFMA v_mfma_f32_32x32x2_f32:
// dw[co][k] = sum over pixels of dz[co][pixel] x~[k][pixel], x~ the input at
// tap k's offset (im2col, bf16 values, exact in FP32).  A workgroup of 16
// waves owns 32 columns k; wave v takes the pixel pairs v, v + 16, ... (A:
// rows co = lane % 32, pixel 2 t + lane / 32; B: column k = lane % 32, same
// pixel), and the 16 partial 32 x 32 blocks are summed in a fixed order in
// LDS: deterministic, no scratch memory.  db[co] = sum of dz (workgroup 0).
__global__ __launch_bounds__(1024) void k_conv_bwd_w(const float* __restrict__ dz, const uint16_t* __restrict__ x,
                                                    float* __restrict__ dw, float* __restrict__ db, int B, int Cin,
                                                    int Cout, int H, int W, int dil)
{
    __shared__ float part[16][16][64];        // [wave][register][lane]
    __shared__ float bsum[16][64];
    const int HW = H * W, K = Cin * 9;
    const int kb = blockIdx.x * 32;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, row = lane & 31, half = lane >> 5;
    // this lane's column k: input channel and tap offset (fixed for the loop)
    const int kk = kb + row;
    const bool kval = kk < K;
    const int ci = kval ? kk / 9 : 0, tap = kval ? kk - ci * 9 : 0;
    const int oy = (tap / 3 - 1) * dil, ox = (tap % 3 - 1) * dil;
    const bool cval = row < Cout;
    const int64_t npair = ((int64_t)B * HW + 1) / 2, P = (int64_t)B * HW;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    float s = 0.0f;
    for (int64_t t = wv; t < npair; t += 16) {
        const int64_t pix = 2 * t + half;
        float av = 0.0f, bv = 0.0f;
        if (pix < P) {
            const int bb = (int)(pix / HW), p = (int)(pix - (int64_t)bb * HW);
            if (cval) av = dz[((int64_t)bb * Cout + row) * HW + p];
            if (kval) {
                const int py = p / W, px = p - py * W, yy = py + oy, xx = px + ox;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W) bv = bf2f(x[((int64_t)bb * Cin + ci) * HW + yy * W + xx]);
            }
        }
        s += av;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) part[wv][r][lane] = acc[r];
    bsum[wv][lane] = s;
    __syncthreads();
    {
        const int r = threadIdx.x >> 6, l = threadIdx.x & 63;   // one output element per thread
        float v = 0.0f;
        for (int q = 0; q < 16; ++q) v += part[q][r][l];
        const int co = 8 * (r >> 2) + 4 * (l >> 5) + (r & 3), k = kb + (l & 31);
        if (co < Cout && k < K) dw[(int64_t)co * K + k] = v;
    }
    if (blockIdx.x == 0 && db && threadIdx.x < 32 && threadIdx.x < Cout) {
        float v = 0.0f;
        for (int q = 0; q < 16; ++q) v += bsum[q][threadIdx.x] + bsum[q][threadIdx.x + 32];
        db[threadIdx.x] = v;
    }
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
    const int Kp = kpad(Cin * 9);
    const size_t wbytes = (size_t)32 * Kp * sizeof(uint16_t);
    const size_t xbytes = (size_t)Cin * fwd_rows_max(H, W, dilation) * W * sizeof(uint16_t);
    const int stage = xbytes <= (size_t)kFwdStage ? 1 : 0;
    const size_t lds = wbytes + (stage ? xbytes : 0);
    static bool attr = false;
    if (!attr) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_conv_fwd), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(kFwdStage + 32 * 32 * 9 * sizeof(uint16_t) + 1024)) != hipSuccess)
            return -3;
        attr = true;
    }
    dim3 grid(blocks((int64_t)H * W, kFwdPix), (unsigned)B);
    hipLaunchKernelGGL(k_conv_fwd, grid, dim3(256), lds, (hipStream_t)stream, x, w, bias, y, y_bf16, Cin, Cout, H, W,
                       Kp, relu, dilation, stage);
    return status(hipGetLastError());
}

int slbm_conv3x3_backward_weight(const float* dz, const uint16_t* x, float* dw, float* db, int32_t B, int32_t Cin,
                                 int32_t Cout, int32_t H, int32_t W, int32_t dilation, void* stream)
{
    if (!dz || !x || !dw || B < 1 || Cin < 1 || Cout < 1 || H < 1 || W < 1 || dilation < 1) return -1;
    if (Cout > 32) return -1;
    hipLaunchKernelGGL(k_conv_bwd_w, dim3((unsigned)((Cin * 9 + 31) / 32)), dim3(1024), 0, (hipStream_t)stream, dz, x,
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
