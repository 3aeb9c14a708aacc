// HIP kernels of the solid lattice-Boltzmann primal and adjoint sweeps (gfx950).
//
// Data layout (HBM): populations in two SoA buffers of 8 planes of N = nx*ny
// doubles each, x fastest.  The primal buffer holds post-collision populations
// f^C(t-1) indexed by their source node, so one sweep *pulls* f^S_q(x, t) =
// f^C_q(x - c_q, t-1) (eq. local_stream), collides (eq. local_collide) and
// writes f^C(x, t) at x: every plane is one shifted, contiguous stream, 64 B
// read + 64 B written per node plus the 16 B forcing (144 B/node/step).
// Plate nodes outside the domain are never written by their own thread; the
// slot (x - c_q, q) of a cut link instead receives the closure value computed
// by the boundary node x, so the pull stays branch-free.
// The adjoint buffer holds phi^C(t) indexed like f^S; one adjoint sweep pulls
// phi^S_q(x) = phi^C_q(x + c_q) (eq. adjoint_streaming, S^T = S^{-1}) and applies
// the transposed collision minus the objective source (eq. adjoint_collision).
// Slots of nodes outside the domain stay zero, which makes the transpose of the
// closures' dropped outgoing populations exact.
#pragma once
#include "slbm_device.h"
#include <type_traits>

namespace slbm {

constexpr int kBlock = 256;

// Convergence status shared by the sweeps of one solve (device memory).
constexpr int kMaxCvWindow = 32;
struct Status {
    int32_t stop;      // set once the residual test passed: later sweeps return at once
    int32_t nwin;      // checks recorded in cwin (coefficient-of-variation test; < 2 x window)
    int64_t t_conv;    // step index of the passing test
    int64_t t_last;    // step index of the last test
    double res;        // last residual (or coefficient of variation)
    double cwin[kMaxCvWindow];  // sum |d|^2 of the last checks, slot = check number mod window
};

struct SweepArgs {
    const double* __restrict__ src;   // 8 planes
    double* __restrict__ dst;         // 8 planes
    const double* __restrict__ g;     // 2 planes forcing (primal) or r (adjoint)
    const double* __restrict__ E;     // 1 plane Young's modulus (E field) or null
    const int32_t* __restrict__ code; // masked: -1 outside, 0 bulk, k+1 boundary record k
    const BNode* __restrict__ bnodes;
    double* __restrict__ snap;        // check sweeps: 2 planes, d(t - K)
    double* __restrict__ partial;     // check sweeps: 2 doubles per block
    const Status* __restrict__ status;
    int32_t nx, ny;
    int64_t N;
    double k11, ks, kd;               // uniform material relaxation keep-factors
    double E0, nu;                    // uniform E (boundary records) and Poisson ratio
    double scale;                     // adjoint: s = dx^2 / Cbar
};

__device__ __forceinline__ void block_sum2(double a, double b, double* out)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    __shared__ double sa[kBlock / 64], sb[kBlock / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { sa[w] = a; sb[w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) { x += sa[i]; y += sb[i]; }
        out[0] = x;
        out[1] = y;
    }
}

// Row index of a linear cell index without an integer division.
__device__ __forceinline__ int row_of(int64_t n, int nx, double inv_nx)
{
    int iy = (int)((double)n * inv_nx);
    int64_t base = (int64_t)iy * nx;
    if (base > n) { --iy; base -= nx; }
    if (base + nx <= n) ++iy;
    return iy;
}

// Source index of direction q for a pull from x - s*c_q (s = +1 primal, -1 adjoint).
// ix/iy wrapped periodically (plates never touch the box edge).
__device__ __forceinline__ void neighbours(int ix, int iy, int nx, int ny, int64_t idx[8], int sgn)
{
    int xm = ix == 0 ? nx - 1 : ix - 1, xp = ix == nx - 1 ? 0 : ix + 1;
    int ym = iy == 0 ? ny - 1 : iy - 1, yp = iy == ny - 1 ? 0 : iy + 1;
    int64_t rY = (int64_t)iy * nx, rM = (int64_t)ym * nx, rP = (int64_t)yp * nx;
    if (sgn > 0) {  // x - c_q
        idx[0] = rY + xm; idx[1] = rM + ix; idx[2] = rY + xp; idx[3] = rP + ix;
        idx[4] = rM + xm; idx[5] = rM + xp; idx[6] = rP + xp; idx[7] = rP + xm;
    } else {        // x + c_q
        idx[0] = rY + xp; idx[1] = rP + ix; idx[2] = rY + xm; idx[3] = rM + ix;
        idx[4] = rP + xp; idx[5] = rP + xm; idx[6] = rM + xm; idx[7] = rM + xp;
    }
}

// ---------------------------------------------------------------- primal sweep
// One node of a primal sweep; num/den receive its residual terms on check sweeps.
template <bool MASKED, bool EFIELD, bool CHECK>
__device__ __forceinline__ void primal_node(const SweepArgs& a, int64_t n, double inv_nx, double& num,
                                            double& den)
{
    int code = MASKED ? a.code[n] : 0;
    if (code < 0) return;
    int iy = row_of(n, a.nx, inv_nx);
    int ix = (int)(n - (int64_t)iy * a.nx);
    int64_t idx[8];
    neighbours(ix, iy, a.nx, a.ny, idx, +1);
    const int64_t N = a.N;
    double f[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) f[q] = a.src[q * N + idx[q]];
    double gx = a.g[n], gy = a.g[N + n];
    double d0, d1;
    if (!MASKED || code == 0) {
        double k11 = a.k11, ks = a.ks, kd = a.kd;
        if (EFIELD) {
            Relax<double> r = relax_from_E<double>(a.E[n], a.nu, false);
            k11 = r.k11; ks = r.ks; kd = r.kd;
        }
        collide_bulk(f, 0.25 * gx, 0.25 * gy, k11, ks, kd, d0, d1);
#pragma unroll
        for (int q = 0; q < 8; ++q) a.dst[q * N + n] = f[q];
    } else {
        const BNode* bn = a.bnodes + (code - 1);
        Relax<double> r = relax_from_E<double>(EFIELD ? a.E[n] : a.E0, a.nu, true);
        double gg[2] = {gx, gy}, fC[8], h[8], mb[5];
        node_map<double>(f, gg, r, bn, true, fC, h, mb);
        d0 = mb[0];
        d1 = mb[1];
        uint32_t cut = bn->cut;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            a.dst[q * N + n] = fC[q];
            if ((cut >> q) & 1u) a.dst[q * N + idx[q]] = h[q];   // ghost slot of the cut link
        }
    }
    if (CHECK) {
        double s0 = a.snap[n], s1 = a.snap[N + n];
        num = (d0 - s0) * (d0 - s0) + (d1 - s1) * (d1 - s1);
        den = d0 * d0 + d1 * d1;
        a.snap[n] = d0;
        a.snap[N + n] = d1;
    }
}

template <bool MASKED, bool EFIELD, bool CHECK>
__global__ __launch_bounds__(kBlock) void k_primal(SweepArgs a, double inv_nx)
{
    if (a.status->stop) return;
    int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double num = 0.0, den = 0.0;
    if (n < a.N) primal_node<MASKED, EFIELD, CHECK>(a, n, inv_nx, num, den);
    if (CHECK) block_sum2(num, den, a.partial + 2 * (int64_t)blockIdx.x);
}

// ---------------------------------------------------------------- adjoint sweep
template <bool MASKED, bool EFIELD, bool CHECK>
__device__ __forceinline__ void adjoint_node(const SweepArgs& a, int64_t n, double inv_nx, double& num,
                                             double& den)
{
    int code = MASKED ? a.code[n] : 0;
    if (code < 0) return;
    int iy = row_of(n, a.nx, inv_nx);
    int ix = (int)(n - (int64_t)iy * a.nx);
    int64_t idx[8];
    neighbours(ix, iy, a.nx, a.ny, idx, -1);
    const int64_t N = a.N;
    double p[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) p[q] = a.src[q * N + idx[q]];
    double srx = a.scale * a.g[n], sry = a.scale * a.g[N + n];
    if (CHECK) {
        double d0 = (p[0] - p[2]) + (p[4] - p[5]) + (p[7] - p[6]);
        double d1 = (p[1] - p[3]) + (p[4] + p[5]) - (p[6] + p[7]);
        double s0 = a.snap[n], s1 = a.snap[N + n];
        num = (d0 - s0) * (d0 - s0) + (d1 - s1) * (d1 - s1);
        den = d0 * d0 + d1 * d1;
        a.snap[n] = d0;
        a.snap[N + n] = d1;
    }
    if (!MASKED || code == 0) {
        double k11 = a.k11, ks = a.ks, kd = a.kd;
        if (EFIELD) {
            Relax<double> r = relax_from_E<double>(a.E[n], a.nu, false);
            k11 = r.k11; ks = r.ks; kd = r.kd;
        }
        adj_collide_bulk(p, srx, sry, k11, ks, kd);
#pragma unroll
        for (int q = 0; q < 8; ++q) a.dst[q * N + n] = p[q];
    } else {
        // transposed extended map of the boundary node: inputs are the routed
        // regular slots and the node's own slots of its cut links
        const BNode* bn = a.bnodes + (code - 1);
        const Relax<double> r = relax_from_E<double>(EFIELD ? a.E[n] : a.E0, a.nu, true);
        double yh[8], out[8];
        const uint32_t cut = bn->cut;
#pragma unroll
        for (int q = 0; q < 8; ++q) yh[q] = ((cut >> q) & 1u) ? a.src[q * N + n] : 0.0;
        adj_boundary(p, yh, bn, r, srx, sry, out);
#pragma unroll
        for (int q = 0; q < 8; ++q) a.dst[q * N + n] = out[q];
    }
}

template <bool MASKED, bool EFIELD, bool CHECK>
__global__ __launch_bounds__(kBlock) void k_adjoint(SweepArgs a, double inv_nx)
{
    if (a.status->stop) return;
    int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double num = 0.0, den = 0.0;
    if (n < a.N) adjoint_node<MASKED, EFIELD, CHECK>(a, n, inv_nx, num, den);
    if (CHECK) block_sum2(num, den, a.partial + 2 * (int64_t)blockIdx.x);
}

// ---------------------------------------------------------------- reductions
// Sums nblk pairs of partials in a fixed order (deterministic), tests r < tol.
// Convergence test of a check sweep.  K-lag mode (cv_window = 0): r =
// ||d(t) - d(t-K)|| / ||d(t)|| < tol.  Coefficient-of-variation mode
// (cv_window = W > 0, the paper's eq. convergence_crit): c = sum |d(t)|^2
// (the mean over the domain nodes up to a constant factor, which cancels)
// joins a window of the last W checks; once W are recorded, std / mean over
// them (population std, sums in slot order) < tol.
__global__ __launch_bounds__(kBlock) void k_residual(const double* __restrict__ partial, int64_t nblk,
                                                    Status* st, double tol, int64_t t, int cv_window)
{
    if (st->stop) return;
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < nblk; i += kBlock) {
        a += partial[2 * i];
        b += partial[2 * i + 1];
    }
    __shared__ double out[2];
    block_sum2(a, b, out);
    if (threadIdx.x == 0) {
        double num = out[0], den = out[1];
        double r;
        if (cv_window > 0) {
            const int W = cv_window;
            st->cwin[st->nwin % W] = den;
            // nwin counts checks up to W and then cycles through [W, 2W): the
            // slot sequence continues (2W = W mod W) and the count never overflows
            st->nwin = st->nwin + 1 == 2 * W ? W : st->nwin + 1;
            r = INFINITY;
            if (st->nwin >= W) {
                double sum = 0.0;
                for (int k = 0; k < W; ++k) sum += st->cwin[k];
                const double mean = sum / W;
                double var = 0.0;
                for (int k = 0; k < W; ++k) var += (st->cwin[k] - mean) * (st->cwin[k] - mean);
                var /= W;
                r = mean > 0.0 ? sqrt(var) / mean : 0.0;
            }
        } else {
            r = den > 0.0 ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
        }
        st->res = r;
        st->t_last = t;
        if (r < tol) {
            st->stop = 1;
            st->t_conv = t;
        }
    }
}

__global__ void k_status_reset(Status* st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->stop = 0;
        st->nwin = 0;
        st->t_conv = -1;
        st->t_last = -1;
        st->res = INFINITY;
    }
}

__global__ __launch_bounds__(kBlock) void k_fill(double* __restrict__ a, int64_t n, double v)
{
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = v;
}

// partial[b] = sum over the block of a[i] * w[i] (w may be null: plain sum), ncomp planes of N
__global__ __launch_bounds__(kBlock) void k_dot_partial(const double* __restrict__ a,
                                                       const double* __restrict__ w, int64_t n,
                                                       double* __restrict__ partial)
{
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double s = 0.0;
    if (i < n) s = w ? a[i] * w[i] : a[i];
    block_sum2(s, 0.0, partial + 2 * (int64_t)blockIdx.x);
}

// out[0] = sum of partial[2 i] (fixed order)
__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* __restrict__ partial, int64_t nblk,
                                                        double* __restrict__ out)
{
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < nblk; i += kBlock) a += partial[2 * i];
    __shared__ double o[2];
    block_sum2(a, 0.0, o);
    if (threadIdx.x == 0) out[0] = o[0];
}

// ---------------------------------------------------------------- control -> forcing
// g = dx^2 sum_i alpha_i B_i
__global__ __launch_bounds__(kBlock) void k_force_modes(const double* __restrict__ modes,
                                                       const double* __restrict__ alpha, int k,
                                                       int64_t n2, double dx2, double* __restrict__ g)
{
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n2) return;
    double s = 0.0;
    for (int m = 0; m < k; ++m) s += alpha[m] * modes[m * n2 + i];
    g[i] = dx2 * s;
}

// out[c*N+i] = scale * (a[c*N+i] - mean[c]) for masked-in nodes (mask null = all), else 0
__global__ __launch_bounds__(kBlock) void k_axpb2(const double* __restrict__ a, const double* __restrict__ mean,
                                                 const int32_t* __restrict__ code, int64_t N, double scale,
                                                 double* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= 2 * N) return;
    int64_t n = i % N;
    int c = (int)(i / N);
    bool in = code ? code[n] >= 0 : true;
    double m = mean ? mean[c] : 0.0;
    out[i] = in ? scale * (a[i] - m) : 0.0;
}

// ---------------------------------------------------------------- initial state
// f^S(0) = populations whose moments are N (d0 - g/2) (equilibrium with bared
// displacement d0; d0 = 0 gives the cold start f = 0), stored pulled-from so the
// first sweep gathers it: buf[q][x - c_q] = f^S_q(x, 0).  snap = d(0).
__global__ __launch_bounds__(kBlock) void k_init_state(double* __restrict__ buf, const double* __restrict__ d0,
                                                      const double* __restrict__ g,
                                                      const int32_t* __restrict__ code, int nx, int ny,
                                                      int64_t N, double inv_nx, double* __restrict__ snap)
{
    int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    if (code && code[n] < 0) {
        snap[n] = 0.0;
        snap[N + n] = 0.0;
        return;
    }
    double gx = g[n], gy = g[N + n];
    double ux = (d0 ? d0[n] : 0.0) - (d0 ? 0.5 * gx : 0.0);
    double uy = (d0 ? d0[N + n] : 0.0) - (d0 ? 0.5 * gy : 0.0);
    int iy = row_of(n, nx, inv_nx);
    int ix = (int)(n - (int64_t)iy * nx);
    int64_t idx[8];
    neighbours(ix, iy, nx, ny, idx, +1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        double W = q < 4 ? 1.0 / 3.0 : 1.0 / 12.0;
        buf[q * N + idx[q]] = W * (cx(q) * ux + cy(q) * uy);
    }
    snap[n] = ux + 0.5 * gx;
    snap[N + n] = uy + 0.5 * gy;
}

// ---------------------------------------------------------------- finalize primal
// From X = f^C(t-1) and Y = f^C(t): f^S(t), f^S(t+1) by pulls, the two-step
// averages fbar, dbar, the residual r = dbar - d* on the observation set and
// per-block sums of |r|^2.
template <bool MASKED>
__global__ __launch_bounds__(kBlock) void k_primal_finalize(
    const double* __restrict__ X, const double* __restrict__ Y, const double* __restrict__ g,
    const int32_t* __restrict__ code, const double* __restrict__ target, const uint8_t* __restrict__ obs,
    int nx, int ny, int64_t N, double inv_nx, double* __restrict__ dbar, double* __restrict__ r,
    double* __restrict__ fbar, double* __restrict__ partial)
{
    int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double s = 0.0;
    if (n < N) {
        bool in = MASKED ? code[n] >= 0 : true;
        if (in) {
            int iy = row_of(n, nx, inv_nx);
            int ix = (int)(n - (int64_t)iy * nx);
            int64_t idx[8];
            neighbours(ix, iy, nx, ny, idx, +1);
            double fa[8], fb[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                fa[q] = X[q * N + idx[q]];
                fb[q] = Y[q * N + idx[q]];
                fbar[q * N + n] = 0.5 * (fa[q] + fb[q]);
            }
            double gx = g[n], gy = g[N + n];
            double a0 = (fa[0] - fa[2]) + (fa[4] - fa[5]) + (fa[7] - fa[6]) + 0.5 * gx;
            double a1 = (fa[1] - fa[3]) + (fa[4] + fa[5]) - (fa[6] + fa[7]) + 0.5 * gy;
            double b0 = (fb[0] - fb[2]) + (fb[4] - fb[5]) + (fb[7] - fb[6]) + 0.5 * gx;
            double b1 = (fb[1] - fb[3]) + (fb[4] + fb[5]) - (fb[6] + fb[7]) + 0.5 * gy;
            double d0 = 0.5 * (a0 + b0), d1 = 0.5 * (a1 + b1);
            dbar[n] = d0;
            dbar[N + n] = d1;
            bool o = obs ? obs[n] != 0 : true;
            double r0 = o ? d0 - target[n] : 0.0, r1 = o ? d1 - target[N + n] : 0.0;
            r[n] = r0;
            r[N + n] = r1;
            s = r0 * r0 + r1 * r1;
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) fbar[q * N + n] = 0.0;
            dbar[n] = dbar[N + n] = 0.0;
            r[n] = r[N + n] = 0.0;
        }
    }
    block_sum2(s, 0.0, partial + 2 * (int64_t)blockIdx.x);
}

// ---------------------------------------------------------------- finalize adjoint + gradient
// From X = phi^C(t), Y = phi^C(t+1): averaged routed adjoint, then eq. optimality
// locally:  dJ/dF = dx^2 (s r / 2 - (dC/dg)^T phi^S)   and, for E controls,
//           dJ/dE = -(dC/dE)^T phi^S  (forward-mode dual number through the node map
//           at the averaged primal state fbar).
template <bool MASKED>
__global__ __launch_bounds__(kBlock) void k_adjoint_finalize(
    const double* __restrict__ X, const double* __restrict__ Y, const int32_t* __restrict__ code,
    const BNode* __restrict__ bnodes, const double* __restrict__ fbar, const double* __restrict__ r,
    const double* __restrict__ g, const double* __restrict__ E, double E0, double nu, int want_E,
    int nx, int ny, int64_t N, double inv_nx, double scale, double dx2, double* __restrict__ dJdF,
    double* __restrict__ dJdE, double* __restrict__ adisp)
{
    int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    int c = MASKED ? code[n] : 0;
    if (c < 0) {
        dJdF[n] = dJdF[N + n] = 0.0;
        if (want_E) dJdE[n] = 0.0;
        adisp[n] = adisp[N + n] = 0.0;
        return;
    }
    int iy = row_of(n, nx, inv_nx);
    int ix = (int)(n - (int64_t)iy * nx);
    int64_t idx[8];
    neighbours(ix, iy, nx, ny, idx, -1);
    double ext[16];
#pragma unroll
    for (int q = 0; q < 8; ++q) ext[q] = 0.5 * (X[q * N + idx[q]] + Y[q * N + idx[q]]);
    const BNode* bn = c > 0 ? bnodes + (c - 1) : nullptr;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        ext[8 + q] = (bn && ((bn->cut >> q) & 1u)) ? 0.5 * (X[q * N + n] + Y[q * N + n]) : 0.0;
    adisp[n] = (ext[0] - ext[2]) + (ext[4] - ext[5]) + (ext[7] - ext[6]);
    adisp[N + n] = (ext[1] - ext[3]) + (ext[4] + ext[5]) - (ext[6] + ext[7]);
    double rx = r[n], ry = r[N + n];
    double Eh = E ? E[n] : E0;
    double Btx, Bty;
    if (!bn) {
        double psi[7];
        adj_moments(ext, psi);
        Btx = psi[0] + 0.5 * kTheta * psi[5];
        Bty = psi[1] + 0.5 * kTheta * psi[6];
    } else {
        Relax<double> rl = relax_from_E<double>(Eh, nu, true);
        double z[8] = {0, 0, 0, 0, 0, 0, 0, 0}, fC[8], h[8], mb[5];
        double gx1[2] = {1.0, 0.0}, gy1[2] = {0.0, 1.0};
        node_map<double>(z, gx1, rl, bn, false, fC, h, mb);
        Btx = 0.0;
        for (int q = 0; q < 8; ++q) Btx += ext[q] * fC[q] + ext[8 + q] * h[q];
        node_map<double>(z, gy1, rl, bn, false, fC, h, mb);
        Bty = 0.0;
        for (int q = 0; q < 8; ++q) Bty += ext[q] * fC[q] + ext[8 + q] * h[q];
    }
    dJdF[n] = dx2 * (0.5 * scale * rx - Btx);
    dJdF[N + n] = dx2 * (0.5 * scale * ry - Bty);
    if (want_E) {
        Dual f[8], gd[2], fC[8], h[8], mb[5];
#pragma unroll
        for (int q = 0; q < 8; ++q) f[q] = Dual(fbar[q * N + n]);
        gd[0] = Dual(g[n]);
        gd[1] = Dual(g[N + n]);
        Relax<Dual> rl = relax_from_E<Dual>(Dual(Eh, 1.0), nu, bn != nullptr);
        node_map<Dual>(f, gd, rl, bn, true, fC, h, mb);
        double s = 0.0;
        for (int q = 0; q < 8; ++q) s += ext[q] * fC[q].d + (bn ? ext[8 + q] * h[q].d : 0.0);
        dJdE[n] = -s;
    }
}

// Current populations f^S of the primal state (pull from the buffer) and their
// bared displacement; plain copies for nodes outside (zeros).
template <bool MASKED>
__global__ __launch_bounds__(kBlock) void k_gather_state(const double* __restrict__ X,
                                                        const double* __restrict__ g,
                                                        const int32_t* __restrict__ code, int nx, int ny,
                                                        int64_t N, double inv_nx, double* __restrict__ pops,
                                                        double* __restrict__ disp)
{
    int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    bool in = MASKED ? code[n] >= 0 : true;
    int iy = row_of(n, nx, inv_nx);
    int ix = (int)(n - (int64_t)iy * nx);
    int64_t idx[8];
    neighbours(ix, iy, nx, ny, idx, +1);
    double f[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) f[q] = in ? X[q * N + idx[q]] : 0.0;
    if (pops)
        for (int q = 0; q < 8; ++q) pops[q * N + n] = f[q];
    if (disp) {
        disp[n] = in ? (f[0] - f[2]) + (f[4] - f[5]) + (f[7] - f[6]) + 0.5 * g[n] : 0.0;
        disp[N + n] = in ? (f[1] - f[3]) + (f[4] + f[5]) - (f[6] + f[7]) + 0.5 * g[N + n] : 0.0;
    }
}

// A converged state given as averaged populations fbar: its displacement
// (eq. disp_from_moments), r = d - d* on the observation set, per-block |r|^2.
template <bool MASKED>
__global__ __launch_bounds__(kBlock) void k_restore(const double* __restrict__ fbar, const double* __restrict__ g,
                                                   const int32_t* __restrict__ code,
                                                   const double* __restrict__ target,
                                                   const uint8_t* __restrict__ obs, int64_t N,
                                                   double* __restrict__ dbar, double* __restrict__ r,
                                                   double* __restrict__ partial)
{
    int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double s = 0.0;
    if (n < N) {
        bool in = MASKED ? code[n] >= 0 : true;
        double f[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) f[q] = fbar[q * N + n];
        double d0 = in ? (f[0] - f[2]) + (f[4] - f[5]) + (f[7] - f[6]) + 0.5 * g[n] : 0.0;
        double d1 = in ? (f[1] - f[3]) + (f[4] + f[5]) - (f[6] + f[7]) + 0.5 * g[N + n] : 0.0;
        dbar[n] = d0;
        dbar[N + n] = d1;
        bool o = in && (obs ? obs[n] != 0 : true);
        double r0 = o ? d0 - target[n] : 0.0, r1 = o ? d1 - target[N + n] : 0.0;
        r[n] = r0;
        r[N + n] = r1;
        s = r0 * r0 + r1 * r1;
    }
    block_sum2(s, 0.0, partial + 2 * (int64_t)blockIdx.x);
}

// Bared stress (lattice units) of the averaged state fbar (eq. stress_from_moments).
__global__ __launch_bounds__(kBlock) void k_stress(const double* __restrict__ fbar, const double* __restrict__ g,
                                                  const int32_t* __restrict__ code,
                                                  const BNode* __restrict__ bnodes,
                                                  const double* __restrict__ E, double E0, double nu,
                                                  int64_t N, double* __restrict__ out)
{
    int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    int c = code ? code[n] : 0;
    if (c < 0) {
        out[n] = out[N + n] = out[2 * N + n] = 0.0;
        return;
    }
    double f[8], gg[2] = {g[n], g[N + n]}, fC[8], h[8], mb[5];
    for (int q = 0; q < 8; ++q) f[q] = fbar[q * N + n];
    Relax<double> r = relax_from_E<double>(E ? E[n] : E0, nu, c > 0);
    node_map<double>(f, gg, r, nullptr, false, fC, h, mb);
    out[n] = -0.5 * (mb[3] + mb[4]);
    out[N + n] = -0.5 * (mb[3] - mb[4]);
    out[2 * N + n] = -mb[2];
}

}  // namespace slbm

namespace slbm {

// ---------------------------------------------------------------- tangent (forward-mode) sweeps
// Forward-mode differentiation of the primal iteration (f-AD, Sec. "Forward
// automatic differentiation"): every population carries its derivative with
// respect to a scalar control direction (Dual value + eps derivative), the
// control's derivative enters as g-dot (force controls) or E-dot (modulus
// controls), and the sweep is the primal one evaluated in dual numbers
// through the same node map (collision, gamma, closures).  At the fixed point
// the derivative part is the tangent d-dot = (dd/dalpha) . direction.
struct TangentArgs {
    const double* __restrict__ srcv;   // 8 planes: values
    const double* __restrict__ srcd;   // 8 planes: derivatives
    double* __restrict__ dstv;
    double* __restrict__ dstd;
    const double* __restrict__ g;      // 2 planes
    const double* __restrict__ gdot;   // 2 planes or null
    const double* __restrict__ E;      // E plane (E field) or null
    const double* __restrict__ Edot;   // its derivative plane or null
    const int32_t* __restrict__ code;
    const BNode* __restrict__ bnodes;
    double* __restrict__ snapv;        // check sweeps: 2 planes each
    double* __restrict__ snapd;
    double* __restrict__ partial;      // check sweeps: 4 doubles per block
    const Status* __restrict__ status;
    int32_t nx, ny;
    int64_t N;
    double E0, E0dot, nu;              // uniform modulus and its derivative
};

__device__ __forceinline__ void block_sum4(double a, double b, double c, double d, double* out)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
        c += __shfl_xor(c, o);
        d += __shfl_xor(d, o);
    }
    __shared__ double s4[4][kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { s4[0][w] = a; s4[1][w] = b; s4[2][w] = c; s4[3][w] = d; }
    __syncthreads();
    if (threadIdx.x < 4) {
        double x = 0.0;
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) x += s4[threadIdx.x][i];
        out[threadIdx.x] = x;
    }
}

template <bool MASKED, bool EFIELD, bool CHECK>
__global__ __launch_bounds__(kBlock) void k_tangent(TangentArgs a, double inv_nx)
{
    if (a.status->stop) return;
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double nv = 0.0, dv = 0.0, nd = 0.0, dd = 0.0;
    const int code = (n < a.N) ? (MASKED ? a.code[n] : 0) : -1;
    if (code >= 0) {
        const int iy = row_of(n, a.nx, inv_nx);
        const int ix = (int)(n - (int64_t)iy * a.nx);
        int64_t idx[8];
        neighbours(ix, iy, a.nx, a.ny, idx, +1);
        const int64_t N = a.N;
        Dual f[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) f[q] = Dual(a.srcv[q * N + idx[q]], a.srcd[q * N + idx[q]]);
        Dual gg[2] = {Dual(a.g[n], a.gdot ? a.gdot[n] : 0.0), Dual(a.g[N + n], a.gdot ? a.gdot[N + n] : 0.0)};
        const Dual E = EFIELD ? Dual(a.E[n], a.Edot ? a.Edot[n] : 0.0) : Dual(a.E0, a.E0dot);
        const Relax<Dual> r = relax_from_E<Dual>(E, a.nu, code > 0);
        const BNode* bn = (MASKED && code > 0) ? a.bnodes + (code - 1) : nullptr;
        Dual fC[8], h[8], mb[5];
        node_map<Dual>(f, gg, r, bn, true, fC, h, mb);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            a.dstv[q * N + n] = fC[q].v;
            a.dstd[q * N + n] = fC[q].d;
        }
        if (bn) {
            const uint32_t cut = bn->cut;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if ((cut >> q) & 1u) {
                    a.dstv[q * N + idx[q]] = h[q].v;
                    a.dstd[q * N + idx[q]] = h[q].d;
                }
        }
        if (CHECK) {
            const double v0 = mb[0].v, v1 = mb[1].v, e0 = mb[0].d, e1 = mb[1].d;
            const double s0 = a.snapv[n], s1 = a.snapv[N + n], t0 = a.snapd[n], t1 = a.snapd[N + n];
            nv = (v0 - s0) * (v0 - s0) + (v1 - s1) * (v1 - s1);
            dv = v0 * v0 + v1 * v1;
            nd = (e0 - t0) * (e0 - t0) + (e1 - t1) * (e1 - t1);
            dd = e0 * e0 + e1 * e1;
            a.snapv[n] = v0;
            a.snapv[N + n] = v1;
            a.snapd[n] = e0;
            a.snapd[N + n] = e1;
        }
    }
    if (CHECK) block_sum4(nv, dv, nd, dd, a.partial + 4 * (int64_t)blockIdx.x);
}

// K-lag residual of a tangent sweep: the larger of the value and derivative residuals.
__global__ __launch_bounds__(kBlock) void k_residual2(const double* __restrict__ partial, int64_t nblk,
                                                     Status* st, double tol, int64_t t)
{
    if (st->stop) return;
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
    for (int64_t k = threadIdx.x; k < nblk; k += kBlock) {
        a += partial[4 * k];
        b += partial[4 * k + 1];
        c += partial[4 * k + 2];
        d += partial[4 * k + 3];
    }
    __shared__ double o[4];
    block_sum4(a, b, c, d, o);
    if (threadIdx.x == 0) {
        const double rv = o[1] > 0.0 ? sqrt(o[0] / o[1]) : (o[0] > 0.0 ? INFINITY : 0.0);
        const double rd = o[3] > 0.0 ? sqrt(o[2] / o[3]) : (o[2] > 0.0 ? INFINITY : 0.0);
        const double r = rv > rd ? rv : rd;
        st->res = r;
        st->t_last = t;
        if (r < tol) {
            st->stop = 1;
            st->t_conv = t;
        }
    }
}

// Two-step averages of value and derivative displacements from X (f^C(t-1))
// and Y (f^C(t)); partial sums of |r|^2 and r . d-dot over the observed
// domain nodes (2 doubles per block), r = d - d*.
template <bool MASKED>
__global__ __launch_bounds__(kBlock) void k_tangent_finalize(
    const double* __restrict__ Xv, const double* __restrict__ Xd, const double* __restrict__ Yv,
    const double* __restrict__ Yd, const double* __restrict__ g, const double* __restrict__ gdot,
    const int32_t* __restrict__ code, const double* __restrict__ target, const uint8_t* __restrict__ obs,
    int nx, int ny, int64_t N, double inv_nx, double* __restrict__ partial)
{
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double sj = 0.0, sd = 0.0;
    if (n < N && (!MASKED || code[n] >= 0) && (!obs || obs[n])) {
        const int iy = row_of(n, nx, inv_nx);
        const int ix = (int)(n - (int64_t)iy * nx);
        int64_t idx[8];
        neighbours(ix, iy, nx, ny, idx, +1);
        // bared value and derivative displacement of the pull from one buffer pair
        auto disp = [&](const double* vv, const double* dd, double out[4]) {
            double fv[8], fd[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                fv[q] = vv[q * N + idx[q]];
                fd[q] = dd[q * N + idx[q]];
            }
            out[0] = (fv[0] - fv[2]) + (fv[4] - fv[5]) + (fv[7] - fv[6]) + 0.5 * g[n];
            out[1] = (fv[1] - fv[3]) + (fv[4] + fv[5]) - (fv[6] + fv[7]) + 0.5 * g[N + n];
            out[2] = (fd[0] - fd[2]) + (fd[4] - fd[5]) + (fd[7] - fd[6]) + (gdot ? 0.5 * gdot[n] : 0.0);
            out[3] = (fd[1] - fd[3]) + (fd[4] + fd[5]) - (fd[6] + fd[7]) + (gdot ? 0.5 * gdot[N + n] : 0.0);
        };
        double x[4], y[4], d[2], e[2];
        disp(Xv, Xd, x);
        disp(Yv, Yd, y);
        d[0] = 0.5 * (x[0] + y[0]);
        d[1] = 0.5 * (x[1] + y[1]);
        e[0] = 0.5 * (x[2] + y[2]);
        e[1] = 0.5 * (x[3] + y[3]);
        const double r0 = d[0] - target[n], r1 = d[1] - target[N + n];
        sj = r0 * r0 + r1 * r1;
        sd = r0 * e[0] + r1 * e[1];
    }
    block_sum2(sj, sd, partial + 2 * (int64_t)blockIdx.x);
}

// out[0], out[1] = sums of partial[2 i], partial[2 i + 1] (fixed order)
__global__ __launch_bounds__(kBlock) void k_sum_partials2(const double* __restrict__ partial, int64_t nblk,
                                                         double* __restrict__ out)
{
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < nblk; i += kBlock) {
        a += partial[2 * i];
        b += partial[2 * i + 1];
    }
    __shared__ double o[2];
    block_sum2(a, b, o);
    if (threadIdx.x == 0) {
        out[0] = o[0];
        out[1] = o[1];
    }
}

// ---------------------------------------------------------------- global-memory access
// Loads and stores through pointers that the caller guarantees to address
// global memory (device buffers).  The fused kernels also run inside batch
// kernels that read their pointers from a device table; to the compiler
// such pointers could address LDS or scratch and would take flat
// instructions, so the accesses state the address space themselves.
template <class T>
__device__ __forceinline__ T ldg(const T* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ void stg(T* p, T v)
{
    *(__attribute__((address_space(1))) T*)p = v;
}

// ---------------------------------------------------------------- temporally blocked sweeps
// T fused time steps of the periodic, uniform-material bulk sweep (primal or
// adjoint) per launch.  One 64-lane wave owns a strip of 64 consecutive
// columns (64 - 2T of them written, T halo columns on each side) and H output
// rows, and marches down the rows of the strip with a pipeline of T levels:
// level k computes step t+k-1 for row r-k while level 0 loads row r.  The pull
// of row y at level k reads level k-1 at rows y-1 (two iterations back), y
// (one back) and y+1 (this iteration); these are kept in registers, and the
// x-neighbours come from the adjacent lanes by shuffles.  Every node is read
// once and written once per T steps (plus the halo), instead of once per step.
// The arithmetic per node and step is the single-step kernels' own
// (collide_bulk / adj_collide_bulk), so the result equals T single sweeps.
struct TBArgs {
    const double* __restrict__ src;
    double* __restrict__ dst;
    const double* __restrict__ g;   // primal: forcing; adjoint: r
    const Status* __restrict__ status;
    int32_t nx, ny, H;
    int32_t strips;                 // strips per row block (single-problem launches)
    int64_t N;
    double k11, ks, kd, scale;
};

// Compute dies (XCDs) of the device: the dispatcher hands consecutive
// workgroups of a launch to the XCDs in turn, and each XCD has its own L2.
constexpr int kXcds = 8;

// Workgroup b of a launch of n -> its place in an order that gives every XCD
// one contiguous run of the n work items (so neighbours in that order, which
// read the same halo lines, run on the same XCD at the same time and the
// second read hits that XCD's L2).  A bijection of [0, n).
__device__ __forceinline__ int xcd_order(int b, int n)
{
    const int x = b % kXcds, j = b / kXcds;
    const int q = n / kXcds, rem = n % kXcds;
    return x * q + min(x, rem) + j;
}

// Whole-wave lane shifts of a double: up = value of lane l-1, down = value of
// lane l+1 (the end lanes keep their own value; they are halo lanes).
// DPP wave_shr:1 / wave_shl:1 moves (no LDS crossbar) unless built with
// SLBM_TB_DPP=0 (then ds_bpermute shuffles).
#ifndef SLBM_TB_DPP
#define SLBM_TB_DPP 1
#endif
__device__ __forceinline__ double lane_up(double v)
{
#if SLBM_TB_DPP
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);  // wave_shr:1
    hi = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
#else
    return __shfl_up(v, 1);
#endif
}
__device__ __forceinline__ double lane_down(double v)
{
#if SLBM_TB_DPP
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);  // wave_shl:1
    hi = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
#else
    return __shfl_down(v, 1);
#endif
}

__device__ __forceinline__ int wrapi(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// One pipeline step of a strip: `o` holds row r as loaded (level 0) and
// returns level T's output (row r - T).  Levels above kmax only advance their
// input history (their outputs are not needed yet: see tb_strip).
template <int T, bool ADJ>
__device__ __forceinline__ void tb_row(double (&p2)[T][3], double (&p1a)[T][3], double (&p1b)[T][2],
                                       double (&o)[8], const TBArgs& a, const double (&gh)[T][2], int kmax)
{
    constexpr int A0 = ADJ ? 3 : 1, A1 = ADJ ? 6 : 4, A2 = ADJ ? 7 : 5;   // planes pulled from row y-1
#pragma unroll
    for (int k = 1; k <= T; ++k) {
        const bool on = k <= kmax;
        // pull of row y = r - k from level k-1
        double f[8];
        if (!on) {
        } else if (!ADJ) {
            f[0] = lane_up(p1b[k - 1][0]);     // (1,0)   from x-1, row y
            f[2] = lane_down(p1b[k - 1][1]);   // (-1,0)  from x+1, row y
            f[1] = p2[k - 1][0];               // (0,1)   row y-1
            f[4] = lane_up(p2[k - 1][1]);      // (1,1)   x-1, row y-1
            f[5] = lane_down(p2[k - 1][2]);    // (-1,1)  x+1, row y-1
            f[3] = o[3];                       // (0,-1)  row y+1
            f[6] = lane_down(o[6]);            // (-1,-1) x+1, row y+1
            f[7] = lane_up(o[7]);              // (1,-1)  x-1, row y+1
        } else {
            f[0] = lane_down(p1b[k - 1][0]);   // from x+1, row y
            f[2] = lane_up(p1b[k - 1][1]);     // from x-1, row y
            f[3] = p2[k - 1][0];               // (0,-1)  row y-1
            f[6] = lane_up(p2[k - 1][1]);      // (-1,-1) x-1, row y-1
            f[7] = lane_down(p2[k - 1][2]);    // (1,-1)  x+1, row y-1
            f[1] = o[1];                       // (0,1)   row y+1
            f[4] = lane_down(o[4]);            // (1,1)   x+1, row y+1
            f[5] = lane_up(o[5]);              // (-1,1)  x-1, row y+1
        }
        // level k-1 history advances by one row
        p2[k - 1][0] = p1a[k - 1][0];
        p2[k - 1][1] = p1a[k - 1][1];
        p2[k - 1][2] = p1a[k - 1][2];
        p1a[k - 1][0] = o[A0];
        p1a[k - 1][1] = o[A1];
        p1a[k - 1][2] = o[A2];
        p1b[k - 1][0] = o[0];
        p1b[k - 1][1] = o[2];
        if (!on) continue;
        // quarter forcing (primal) or scaled residual (adjoint) of row r - k from the history
        if (!ADJ) {
            double d0, d1;
            collide_bulk(f, gh[k - 1][0], gh[k - 1][1], a.k11, a.ks, a.kd, d0, d1);
        } else {
            adj_collide_bulk(f, gh[k - 1][0], gh[k - 1][1], a.k11, a.ks, a.kd);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) o[q] = f[q];
    }
}

// One strip (sx, sy) of a fused launch, run by one 64-lane wave.
template <int T, bool ADJ>
__device__ __forceinline__ void tb_strip(const TBArgs& a, int sx, int sy)
{
    constexpr int V = 64 - 2 * T;
    // With V a multiple of 16 (T = 8: 48 columns) the strips are shifted by T
    // columns, so that every wave's 64 columns start on a 128-byte line (when
    // a row is, i.e. nx a multiple of 16) and a row read touches 4 lines, not
    // 5; the wrap keeps each column written by exactly one strip.
    constexpr int XOFF = V % 16 == 0 ? T : 0;
    const int lane = threadIdx.x;
    const int nx = a.nx, ny = a.ny;
    const int64_t N = a.N;
    const int xs = sx * V - T + XOFF + lane;            // unwrapped column of this lane
    const int x = wrapi(xs, nx);
    const bool out_lane = lane >= T && lane < 64 - T && xs < nx + XOFF;
    const int y0 = sy * a.H;
    const int y1 = min(y0 + a.H, ny);
    // histories of level k's outputs (k = 0..T-1): p2 = row two back, p1 = row one back.
    // primal: rows y-1 feed planes {1,4,5}, rows y+1 feed {3,6,7};
    // adjoint: rows y-1 feed {3,6,7}, rows y+1 feed {1,4,5}.
    // gh[j] = forcing / 4 (or scaled residual) of row r - 1 - j: each row's is
    // loaded once, with its populations, and consumed by level j + 1 one row later
    double p2[T][3], p1a[T][3], p1b[T][2], gh[T][2];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        p2[k][0] = p2[k][1] = p2[k][2] = 0.0;
        p1a[k][0] = p1a[k][1] = p1a[k][2] = 0.0;
        p1b[k][0] = p1b[k][1] = 0.0;
        gh[k][0] = gh[k][1] = 0.0;
    }
    const double gsc = ADJ ? a.scale : 0.25;
    const int iters = (y1 - y0) + 2 * T;
    int r = y0 - T;
    int rw = wrapi(r, ny);                              // r wrapped into [0, ny)
    auto next = [&](int v) { return v + 1 == ny ? 0 : v + 1; };
    auto load = [&](int roww, double (&v)[8], double (&gr)[2]) {
        const int64_t base = (int64_t)roww * nx + x;
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = ldg(a.src + q * N + base);
        gr[0] = ldg(a.g + base);
        gr[1] = ldg(a.g + N + base);
    };
    auto shift = [&](const double (&gr)[2]) {
#pragma unroll
        for (int j = T - 1; j > 0; --j) {
            gh[j][0] = gh[j - 1][0];
            gh[j][1] = gh[j - 1][1];
        }
        gh[0][0] = gr[0];
        gh[0][1] = gr[1];
    };
    auto store = [&](int row, const double (&v)[8]) {
        const int yo = row - T;
        if (out_lane && yo >= y0 && yo < y1) {
            const int64_t base = (int64_t)yo * nx + x;
#pragma unroll
            for (int q = 0; q < 8; ++q) stg(a.dst + q * N + base, v[q]);
        }
    };
    // Rows are loaded one trip (two rows) ahead of their use, so a trip's
    // loads are in flight while the previous trip computes (one wave per SIMD:
    // no other wave hides the latency).  The loads are issued on every trip (a
    // branch around them would make the compiler wait for all loads where the
    // paths join); the last trip re-reads its own rows (L2 hits) instead.
    int it = 0;
    double n0[8], n1[8], gn0[2], gn1[2];                // rows it, it + 1
    load(rw, n0, gn0);
    load(next(rw), n1, gn1);
    auto take = [&](double (&o0)[8], double (&o1)[8], double (&g0)[2], double (&g1)[2], bool more) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            o0[q] = n0[q];
            o1[q] = n1[q];
        }
        g0[0] = gsc * gn0[0];
        g0[1] = gsc * gn0[1];
        g1[0] = gsc * gn1[0];
        g1[1] = gsc * gn1[1];
        if (more) rw = next(next(rw));
        load(rw, n0, gn0);
        load(next(rw), n1, gn1);
    };
    // Pipeline fill: level k first produces a row that a later level (or the
    // output) reads at iteration 2k (its row r - k = y0 - T + k lies in the
    // halo of width T - k that level k must cover), so the first T trips of two
    // rows run levels 1..trip only; nothing is stored before iteration 2T.
    // A prefetched row past the strip's last (it + 3 = iters) is a valid,
    // wrapped row that is never used.
    for (int j = 0; j < T; ++j, it += 2, r += 2) {
        double o0[8], o1[8], g0[2], g1[2];
        take(o0, o1, g0, g1, true);
        tb_row<T, ADJ>(p2, p1a, p1b, o0, a, gh, j);
        shift(g0);
        tb_row<T, ADJ>(p2, p1a, p1b, o1, a, gh, j);
        shift(g1);
    }
    // two rows per trip: the second row's early levels overlap the first's late ones
    for (; it + 1 < iters; it += 2, r += 2) {
        double o0[8], o1[8], g0[2], g1[2];
        take(o0, o1, g0, g1, it + 2 < iters);
        tb_row<T, ADJ>(p2, p1a, p1b, o0, a, gh, T);
        store(r, o0);
        shift(g0);
        tb_row<T, ADJ>(p2, p1a, p1b, o1, a, gh, T);
        store(r + 1, o1);
        shift(g1);
    }
    if (it < iters) {
        tb_row<T, ADJ>(p2, p1a, p1b, n0, a, gh, T);
        store(r, n0);
    }
}

// One wave per strip of a row block, in row-major order of (row block, strip)
// handed out XCD by XCD: the strips of a row block, which share their halo
// columns with their neighbours, run together on one XCD.
template <int T, bool ADJ>
__global__ __launch_bounds__(64) void k_sweep_tb(TBArgs a)
{
    if (a.status->stop) return;
    const int t = xcd_order(blockIdx.x, gridDim.x);
    tb_strip<T, ADJ>(a, t % a.strips, t / a.strips);
}

// ---------------------------------------------------------------- fused sweeps, plates and E fields
// Several sweeps of a plate (masked domain with boundary closures) or of a
// per-node modulus field per launch.  A workgroup owns a tile of tw x th
// nodes; it loads the tile plus a halo of `halo` nodes (all 8 planes) into
// LDS, runs `steps` <= halo sweeps there, and writes only the tile's own
// nodes (and the ghost slots of its boundary nodes) back to HBM.  Plates keep
// two LDS copies of the region: sweep s reads copy (s - 1) % 2 and writes
// copy s % 2, as the single-step sweeps read one population buffer and write
// the other, so one barrier per sweep orders them (their slower boundary
// waves made the second barrier costly).  Unmasked problems sweep one copy in
// place: all pulls are read, a barrier, then the writes and a second barrier
// (half the LDS, and measured faster there).  Sweep s computes
// the tile grown by steps - s nodes, so every value it pulls was produced by
// sweep s - 1 inside the region.  The per-node arithmetic is the
// single-step kernels' own, so a launch of k steps equals k single sweeps
// bit for bit.
struct TileArgs {
    const double* __restrict__ src;
    double* __restrict__ dst;
    const double* __restrict__ g;     // primal: forcing; adjoint: r
    const double* __restrict__ E;     // E plane or null
    const int32_t* __restrict__ code;
    const BNode* __restrict__ bnodes;
    const Status* __restrict__ status;
    int32_t nx, ny;
    int64_t N;
    double k11, ks, kd, E0, nu, scale;
    int32_t tw, th, halo, steps, tiles_x;
    int32_t order_by_kind;           // plates: threads take bulk, then boundary, then outside nodes
    int32_t maxb;                    // boundary records staged in LDS (<= kTileMaxB; the rest from HBM)
    // launch plan of the tile shape (null: formed in the kernel), written once
    // by k_tile_plan: per tile and thread (node, code, region node | (staged
    // slot + 1) << 16, rx | ry << 16); per tile the records of its staged
    // slots and their count
    const int4* plan;
    const int32_t* plan_rec;
    const int32_t* plan_nst;
};

constexpr int kTileBlock = 1024;
constexpr int kTileNPT = 1;                          // region nodes per thread (2 with 512 threads measured slower)
constexpr int kTileMaxNodes = kTileBlock * kTileNPT; // region <= 1024 nodes (64 KiB of LDS per copy)
// Boundary records staged in LDS once per launch (plates); records beyond
// the cap are read from HBM / L2 (same values, only slower).
constexpr int kTileMaxB = 96;                        // 96 x 272 B

__host__ __device__ constexpr size_t tile_lds_bytes(int region, bool masked, int maxb = kTileMaxB)
{
    return (size_t)(masked ? 16 : 8) * region * sizeof(double) + (masked ? (size_t)maxb * sizeof(BNode) : 0);
}

// The stable order by kind of a plate tile's region nodes (bulk, boundary,
// outside): ni[j] becomes the region node the thread runs in pass j.  Reads
// the node codes (one round trip); ends with a barrier.
__device__ __forceinline__ void tile_order(const TileArgs& a, int x0, int y0, int RX, int R, int ni[kTileNPT])
{
    const int nx = a.nx, ny = a.ny;
    constexpr int W = kTileBlock / 64;
    __shared__ int wcount[kTileNPT][2][W];      // bulk / boundary nodes per wave
    __shared__ short order[kTileMaxNodes];      // region node of each slot
    const int w = threadIdx.x / 64;
    const uint64_t below = __lanemask_lt();
    uint64_t b0[kTileNPT], b1[kTileNPT];
    int kind[kTileNPT];                         // 0 bulk, 1 boundary, 2 outside or none
#pragma unroll
    for (int j = 0; j < kTileNPT; ++j) {
        const int i = ni[j];
        int c = -1;
        if (i < R) c = ldg(a.code + (int64_t)wrapi(y0 + i / RX, ny) * nx + wrapi(x0 + i % RX, nx));
        kind[j] = c < 0 ? 2 : (c > 0 ? 1 : 0);
        b0[j] = __ballot(kind[j] == 0);
        b1[j] = __ballot(kind[j] == 1);
        if ((threadIdx.x & 63) == 0) {
            wcount[j][0][w] = __popcll(b0[j]);
            wcount[j][1][w] = __popcll(b1[j]);
        }
    }
    __syncthreads();
    // totals and the counts of earlier waves (pass j's waves come after pass j - 1's)
    int tot0 = 0, tot1 = 0;
    int pre0[kTileNPT], pre1[kTileNPT];
#pragma unroll
    for (int j = 0; j < kTileNPT; ++j) {
        pre0[j] = tot0;
        pre1[j] = tot1;
        for (int v = 0; v < W; ++v) {
            const int n0 = wcount[j][0][v], n1 = wcount[j][1][v];
            if (v < w) {
                pre0[j] += n0;
                pre1[j] += n1;
            }
            tot0 += n0;
            tot1 += n1;
        }
    }
#pragma unroll
    for (int j = 0; j < kTileNPT; ++j) {
        const int i = ni[j];
        const int r0 = pre0[j] + __popcll(b0[j] & below), r1 = pre1[j] + __popcll(b1[j] & below);
        const int slot = kind[j] == 0 ? r0 : kind[j] == 1 ? tot0 + r1 : tot0 + tot1 + (i - r0 - r1);
        order[slot] = (short)i;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kTileNPT; ++j) ni[j] = order[threadIdx.x + j * kTileBlock];
}

// One tile (index `tile` of the problem's tiles_x x tiles_y) of a tiled launch;
// lds: the region's 8 planes (two copies for plates), then the staged
// boundary records.  PLAN: the launch has a plan (a.plan non-null).
template <bool MASKED, bool EFIELD, bool ADJ, bool PLAN = false>
__device__ __forceinline__ void tile_body(const TileArgs& a, int tile, double* lds)
{
    const int h = a.halo, RX = a.tw + 2 * h, RY = a.th + 2 * h, R = RX * RY;
    const int bx = tile % a.tiles_x, by = tile / a.tiles_x;
    const int x0 = bx * a.tw - h, y0 = by * a.th - h;   // unwrapped origin of the region
    const int nx = a.nx, ny = a.ny;
    const int64_t N = a.N;
    // per-node constants of the launch, held in registers: position, code,
    // source term (primal: g; adjoint: s r) and relaxation (the same
    // relax_from_E values the single-step kernels form every step)
    int rx[kTileNPT], ry[kTileNPT], cd[kTileNPT];
    int64_t gn[kTileNPT];
    double c0[kTileNPT], c1[kTileNPT];
    Relax<double> rl[kTileNPT];
    // staged boundary records: a node's record is read from LDS (slot bsl) or,
    // past the cap, from HBM (bng).  The two pointers are kept apart, so each
    // use is compiled for its own memory (LDS reads, global loads); a pointer
    // that could be either is a generic one, whose loads are slower.
    __shared__ int nstaged;
    BNode* lbn = reinterpret_cast<BNode*>(lds + (MASKED ? 16 : 8) * R);
    const BNode* bng[kTileNPT];
    int bsl[kTileNPT];
    // The region node a thread runs in pass j: node threadIdx.x + j * kTileBlock, or, with
    // order_by_kind (plates), a stable order by kind -- bulk nodes first, then
    // boundary nodes, then outside nodes -- so that the few boundary nodes
    // (whose node map is several times the bulk work) fill one or two waves
    // instead of diverging in many, and outside nodes leave whole waves idle.
    // Each node's arithmetic is unchanged, only the thread that runs it.
    // Formed here, the order costs a round trip to HBM for the node codes
    // before the other loads (measured: it pays where a launch has no more
    // tiles than the GPU has CUs, not beyond); with a launch plan (PLAN) the
    // thread reads its node, code, position and staged-record slot instead.
    int ni[kTileNPT];
    constexpr bool planned = PLAN;
    int4 pe[kTileNPT];                           // this thread's plan entries
#pragma unroll
    for (int j = 0; j < kTileNPT; ++j) ni[j] = threadIdx.x + j * kTileBlock;
    if (planned) {
#pragma unroll
        for (int j = 0; j < kTileNPT; ++j) {
            pe[j] = a.plan[(int64_t)tile * kTileMaxNodes + threadIdx.x + j * kTileBlock];
            ni[j] = pe[j].z & 0xffff;
        }
    } else if (MASKED) {
        if (threadIdx.x == 0) nstaged = 0;
        if (a.order_by_kind) tile_order(a, x0, y0, RX, R, ni);
        else __syncthreads();
    }
    // planned launches copy the tile's staged records with all threads (each
    // a few words), issued with the node loads: one round trip after the plan
    constexpr int kRecWords = (int)(sizeof(BNode) / 8);
    constexpr int kStageWords = (kTileMaxB * kRecWords + kTileBlock - 1) / kTileBlock;
    double rw[MASKED ? kStageWords : 1];
    int nwords = 0;
    if (MASKED && planned) {
        nwords = a.plan_nst[tile] * kRecWords;
        int rec[kStageWords];
#pragma unroll
        for (int p = 0; p < kStageWords; ++p) {
            const int w = threadIdx.x + p * kTileBlock;
            rec[p] = w < nwords ? a.plan_rec[(int64_t)tile * kTileMaxB + w / kRecWords] : 0;
        }
        const double* words = reinterpret_cast<const double*>(a.bnodes);
#pragma unroll
        for (int p = 0; p < kStageWords; ++p) {
            const int w = threadIdx.x + p * kTileBlock;
            rw[p] = w < nwords ? ldg(words + (int64_t)rec[p] * kRecWords + w % kRecWords) : 0.0;
        }
    }
#pragma unroll
    for (int j = 0; j < kTileNPT; ++j) {
        const int i = ni[j];
        if (planned) {
            rx[j] = pe[j].w & 0xffff;
            ry[j] = pe[j].w >> 16;
        } else {
            rx[j] = i % RX;
            ry[j] = i / RX;
        }
        cd[j] = -1;
        gn[j] = 0;
        c0[j] = c1[j] = 0.0;
        rl[j].k11 = a.k11;
        rl[j].ks = a.ks;
        rl[j].kd = a.kd;
        rl[j].gam = 0.0;
        if (i < R) {
            const int64_t n = planned ? (int64_t)pe[j].x : (int64_t)wrapi(y0 + ry[j], ny) * nx + wrapi(x0 + rx[j], nx);
            gn[j] = n;
            // every load of the node is issued before any of them is used (one
            // round trip; the planes cover the whole box, so outside nodes
            // read defined values, which they do not use)
            const int code = planned ? pe[j].y : (MASKED ? ldg(a.code + n) : 0);
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = ldg(a.src + q * N + n);
            const double g0 = ldg(a.g + n), g1 = ldg(a.g + N + n);
            const double Ev = EFIELD ? ldg(a.E + n) : a.E0;
            cd[j] = code;
            // plates fill both copies: slots that no sweep writes (outside
            // nodes, which adjoint boundary nodes pull from) must read their
            // stored values
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                lds[q * R + i] = v[q];
                if (MASKED) lds[(8 + q) * R + i] = v[q];
            }
            const bool live = code >= 0;
            c0[j] = live ? (ADJ ? a.scale * g0 : g0) : 0.0;
            c1[j] = live ? (ADJ ? a.scale * g1 : g1) : 0.0;
            if (EFIELD) {
                const Relax<double> r = relax_from_E<double>(Ev, a.nu, code > 0);
                if (live) rl[j] = r;
            } else if (code > 0) {
                rl[j] = relax_from_E<double>(a.E0, a.nu, true);
            }
        }
        bng[j] = a.bnodes;
        bsl[j] = -1;
        if (MASKED && i < R && cd[j] > 0) {
            const int k = cd[j] - 1;
            bng[j] = a.bnodes + k;
            if (planned) {
                bsl[j] = (pe[j].z >> 16) - 1;            // -1: past the cap, read from HBM
            } else {
                const int slot = atomicAdd(&nstaged, 1);
                if (slot < a.maxb) {
                    const double* s8 = reinterpret_cast<const double*>(a.bnodes + k);
                    double* d8 = reinterpret_cast<double*>(lbn + slot);
#pragma unroll
                    for (int w = 0; w < kRecWords; ++w) d8[w] = ldg(s8 + w);
                    bsl[j] = slot;
                }
            }
        }
    }
    if (MASKED && planned) {
        double* lw = reinterpret_cast<double*>(lbn);
#pragma unroll
        for (int p = 0; p < kStageWords; ++p) {
            const int w = threadIdx.x + p * kTileBlock;
            if (w < nwords) lw[w] = rw[p];
        }
    }
    __syncthreads();
    for (int s = 1; s <= a.steps; ++s) {
        const bool last = s == a.steps;
        const double* cur = MASKED ? lds + ((s - 1) & 1) * 8 * R : lds;   // written by sweep s - 1
        double* nxt = MASKED ? lds + (s & 1) * 8 * R : lds;
        const int m = h - (a.steps - s);             // this sweep computes [m, RX - m) x [m, RY - m)
        double out[kTileNPT][8];
        bool act[kTileNPT];
#pragma unroll
        for (int j = 0; j < kTileNPT; ++j) {
            const int i = ni[j];
            act[j] = i < R && cd[j] >= 0 && rx[j] >= m && rx[j] < RX - m && ry[j] >= m && ry[j] < RY - m;
            // the last sweep writes HBM: only nodes of the grid proper (no wrapped copies)
            if (last) act[j] = act[j] && x0 + rx[j] < nx && y0 + ry[j] < ny;
            if (!act[j]) continue;
            const int64_t n = gn[j];
            const int code = cd[j];
            double f[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int off = cx(q) + cy(q) * RX;
                f[q] = cur[q * R + (ADJ ? i + off : i - off)];
            }
            if (!ADJ) {
                if (!MASKED || code == 0) {
                    double d0, d1;
                    collide_bulk(f, 0.25 * c0[j], 0.25 * c1[j], rl[j].k11, rl[j].ks, rl[j].kd, d0, d1);
#pragma unroll
                    for (int q = 0; q < 8; ++q) out[j][q] = f[q];
                } else {
                    auto bnode = [&](const BNode* bn, auto sparse) {
                        double gg[2] = {c0[j], c1[j]}, fC[8], hv[8], mb[5];
                        node_map<double, decltype(sparse)::value>(f, gg, rl[j], bn, true, fC, hv, mb);
                        const uint32_t cut = bn->cut;
                        int64_t idx[8];
                        // the last sweep covers nodes of the grid proper only (no wrap)
                        if (last) neighbours(x0 + rx[j], y0 + ry[j], nx, ny, idx, +1);
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            out[j][q] = fC[q];
                            if ((cut >> q) & 1u) {
                                if (last) stg(a.dst + q * N + idx[q], hv[q]);
                                else nxt[q * R + i - (cx(q) + cy(q) * RX)] = hv[q];
                            }
                        }
                    };
                    if (bsl[j] >= 0) bnode(lbn + bsl[j], std::true_type());
                    else bnode(bng[j], std::false_type());
                }
            } else {
                const double srx = c0[j], sry = c1[j];
                if (!MASKED || code == 0) {
                    adj_collide_bulk(f, srx, sry, rl[j].k11, rl[j].ks, rl[j].kd);
#pragma unroll
                    for (int q = 0; q < 8; ++q) out[j][q] = f[q];
                } else {
                    auto bnode = [&](const BNode* bn, auto sparse) {
                        const uint32_t cut = bn->cut;
                        double yh[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) yh[q] = ((cut >> q) & 1u) ? cur[q * R + i] : 0.0;
                        adj_boundary<decltype(sparse)::value>(f, yh, bn, rl[j], srx, sry, out[j]);
                    };
                    if (bsl[j] >= 0) bnode(lbn + bsl[j], std::true_type());
                    else bnode(bng[j], std::false_type());
                }
            }
            if (last) {
#pragma unroll
                for (int q = 0; q < 8; ++q) stg(a.dst + q * N + n, out[j][q]);
            }
        }
        if (last) break;
        if (!MASKED) __syncthreads();               // in place: every pull read before the writes
#pragma unroll
        for (int j = 0; j < kTileNPT; ++j) {
            if (!act[j]) continue;
            const int i = ni[j];
#pragma unroll
            for (int q = 0; q < 8; ++q) nxt[q * R + i] = out[j][q];
        }
        __syncthreads();
    }
}

// Tiles in row-major order, handed out XCD by XCD (xcd_order): neighbouring
// tiles, whose regions overlap by the halo, load them on the same L2.
template <bool MASKED, bool EFIELD, bool ADJ>
__global__ __launch_bounds__(kTileBlock) void k_sweep_tile(TileArgs a)
{
    if (a.status->stop) return;
    extern __shared__ __align__(16) double lds[];    // 8 planes of RX * RY doubles (2 copies for plates), then staged records
    if (a.plan) tile_body<MASKED, EFIELD, ADJ, true>(a, xcd_order(blockIdx.x, gridDim.x), lds);
    else tile_body<MASKED, EFIELD, ADJ, false>(a, xcd_order(blockIdx.x, gridDim.x), lds);
}

// Launch plan of a tile shape (grid: one workgroup per tile, in tile order):
// the node each thread of the sweep kernels runs, its grid index, code and
// position, and the staged boundary records.  Written once per shape; the
// sweeps then need no code load, ordering pass or index arithmetic before
// their single round trip for the node data.
//
// Placement (plates with order_by_kind): a wave's time per sweep is that of
// the costliest node kind among its lanes, and a SIMD's is the sum over its
// waves (wave w of the workgroup runs on SIMD w % 4).  Boundary nodes (whose
// node map is several times the bulk work) fill whole waves of their own, one
// per SIMD from SIMD 0 on, and the waves of outside nodes (idle) share those
// SIMDs, so that no SIMD runs a boundary wave on top of a full share of bulk
// waves.  Where that does not fit (no boundary node, more than 4 boundary
// waves, too many bulk waves), bulk nodes come first, then boundary nodes,
// then outside nodes, in region order within each kind.  Unordered launches
// keep the region order.
template <bool MASKED>
__global__ __launch_bounds__(kTileBlock) void k_tile_plan(TileArgs a, int4* plan, int32_t* plan_rec,
                                                         int32_t* plan_nst)
{
    static_assert(kTileNPT == 1, "the plan places one region node per thread");
    constexpr int W = kTileBlock / 64;
    const int tile = blockIdx.x;
    const int h = a.halo, RX = a.tw + 2 * h, RY = a.th + 2 * h, R = RX * RY;
    const int x0 = (tile % a.tiles_x) * a.tw - h, y0 = (tile / a.tiles_x) * a.th - h;
    const int i = threadIdx.x;                          // region node, region order
    const int rx = i % RX, ry = i / RX;
    int n = 0, code = -1;
    if (i < R) {
        n = wrapi(y0 + ry, a.ny) * a.nx + wrapi(x0 + rx, a.nx);
        code = MASKED ? ldg(a.code + n) : 0;
    }
    const int kind = code < 0 ? 2 : (code > 0 ? 1 : 0);   // bulk, boundary, outside or none
    // rank of the node within its kind (region order) and the totals
    __shared__ int cnt[3][W];
    __shared__ int wave_of[W];                          // placement sequence of the waves
    const int w = threadIdx.x / 64;
    const uint64_t below = __lanemask_lt();
    uint64_t bal[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        bal[k] = __ballot(kind == k);
        if ((threadIdx.x & 63) == 0) cnt[k][w] = __popcll(bal[k]);
    }
    __syncthreads();
    int tot[3] = {0, 0, 0}, pre[3] = {0, 0, 0};
    for (int v = 0; v < W; ++v)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (v < w) pre[k] += cnt[k][v];
            tot[k] += cnt[k][v];
        }
    const int rank = (kind == 0 ? pre[0] : kind == 1 ? pre[1] : pre[2]) +
                     __popcll((kind == 0 ? bal[0] : kind == 1 ? bal[1] : bal[2]) & below);
    const int nb = (tot[1] + 63) / 64, n0w = (tot[0] + 63) / 64;
    const bool ordered = MASKED && a.order_by_kind;
    const bool balanced = ordered && nb >= 1 && nb <= 4 && nb + n0w <= W;
    const int pad = 64 * nb - tot[1];                  // outside nodes completing the boundary waves
    const int nI = balanced ? min(min(3 * nb, W - nb - n0w), max(0, tot[2] - pad) / 64) : 0;
    if (threadIdx.x == 0) {
        bool used[W] = {};
        int k = 0;
        if (balanced) {
            for (int s = 0; s < nb; ++s) used[wave_of[k++] = s] = true;                  // boundary waves
            for (int m = 1; m <= 3 && k < nb + nI; ++m)                                   // idle waves beside them
                for (int s = 0; s < nb && k < nb + nI; ++s) used[wave_of[k++] = s + 4 * m] = true;
        }
        for (int v = 0; v < W; ++v)
            if (!used[v]) wave_of[k++] = v;
    }
    __syncthreads();
    int pos;                                            // place in the sequence of lanes
    if (balanced) {
        if (kind == 1) pos = rank;
        else if (kind == 2) pos = rank < pad ? tot[1] + rank
                                  : rank < pad + 64 * nI ? 64 * nb + (rank - pad)
                                                         : 64 * (nb + nI) + tot[0] + (rank - pad - 64 * nI);
        else pos = 64 * (nb + nI) + rank;
    } else if (ordered) {
        pos = kind == 0 ? rank : kind == 1 ? tot[0] + rank : tot[0] + tot[1] + rank;
    } else {
        pos = i;
    }
    const int slot = wave_of[pos / 64] * 64 + pos % 64;
    // staged boundary records: the first maxb boundary nodes in region order
    int slot1 = 0;
    if (MASKED && kind == 1 && rank < a.maxb) {
        plan_rec[(int64_t)tile * kTileMaxB + rank] = code - 1;
        slot1 = rank + 1;
    }
    plan[(int64_t)tile * kTileMaxNodes + slot] = make_int4(n, code, i | (slot1 << 16), rx | (ry << 16));
    if (threadIdx.x == 0) plan_nst[tile] = MASKED ? min(tot[1], a.maxb) : 0;
}

}  // namespace slbm

namespace slbm {

// ---------------------------------------------------------------- batched sweeps
// Many independent problems advance in one launch.  A block table maps every
// block of the launch to (instance, local block / strip); each instance keeps
// its own buffers, parameters, residual checks and stop flag.  Periodic and
// plate instances keep separate buffer parities (fused launches flip a buffer
// once per T steps, single-step launches once per step).
struct BatchInst {
    SweepArgs prim[2];    // primal args by buffer parity (src = buffer p, dst = buffer p^1)
    SweepArgs adj[2];     // adjoint args by buffer parity
    TBArgs tprim[2], tadj[2];      // wave-strip fused launches
    TileArgs lprim[2], ladj[2];    // LDS-tiled fused launches
    Status* status;
    double inv_nx;
    int32_t masked;
    int32_t efield;       // E plane per node (E control)
    int32_t tiled;        // fused by the LDS-tiled kernel (else by the wave strips)
    int32_t sx;           // strips per row of wave-strip launches
    int64_t nblk;         // blocks of one single-step sweep
};

__device__ __forceinline__ bool mask_bit(uint64_t lo, uint64_t hi, int i)
{
    return i < 64 ? ((lo >> i) & 1ull) : ((hi >> (i - 64)) & 1ull);
}

template <bool ADJ>
__global__ __launch_bounds__(kBlock) void k_sweep_batch(const BatchInst* __restrict__ inst,
                                                       const int2* __restrict__ table, int par_periodic,
                                                       int par_plate, uint64_t check_lo, uint64_t check_hi)
{
    const int2 e = table[blockIdx.x];
    const BatchInst& I = inst[e.x];
    if (I.status->stop) return;
    const int par = I.tiled ? par_plate : par_periodic;   // parity of the tiled / wave-strip class
    const SweepArgs& a = ADJ ? I.adj[par] : I.prim[par];
    const bool check = mask_bit(check_lo, check_hi, e.x);
    const int64_t n = (int64_t)e.y * kBlock + threadIdx.x;
    double num = 0.0, den = 0.0;
    if (n < a.N) {
        const int sel = (I.masked ? 4 : 0) | (I.efield ? 2 : 0) | (check ? 1 : 0);
#define BN_CASE(i, M, EF, CH)                                                       \
    case i:                                                                         \
        if (ADJ) adjoint_node<M, EF, CH>(a, n, I.inv_nx, num, den);                 \
        else primal_node<M, EF, CH>(a, n, I.inv_nx, num, den);                      \
        break;
        switch (sel) {
            BN_CASE(0, false, false, false)
            BN_CASE(1, false, false, true)
            BN_CASE(2, false, true, false)
            BN_CASE(3, false, true, true)
            BN_CASE(4, true, false, false)
            BN_CASE(5, true, false, true)
            BN_CASE(6, true, true, false)
            BN_CASE(7, true, true, true)
        }
#undef BN_CASE
    }
    if (check) block_sum2(num, den, a.partial + 2 * (int64_t)e.y);
}

template <int T, bool ADJ>
__global__ __launch_bounds__(64) void k_sweep_tb_batch(const BatchInst* __restrict__ inst,
                                                      const int2* __restrict__ table, int par_periodic)
{
    const int2 e = table[blockIdx.x];
    const BatchInst& I = inst[e.x];
    if (I.status->stop) return;
    const TBArgs a = ADJ ? I.tadj[par_periodic] : I.tprim[par_periodic];
    tb_strip<T, ADJ>(a, e.y % I.sx, e.y / I.sx);
}

// Tiled instances of a batch: `steps` <= halo sweeps of every listed tile.
template <bool ADJ>
__global__ __launch_bounds__(kTileBlock) void k_sweep_tile_batch(const BatchInst* __restrict__ inst,
                                                                 const int2* __restrict__ table, int par,
                                                                 int steps)
{
    const int2 e = table[blockIdx.x];
    const BatchInst& I = inst[e.x];
    if (I.status->stop) return;
    extern __shared__ __align__(16) double lds[];
    TileArgs a = ADJ ? I.ladj[par] : I.lprim[par];
    a.steps = steps;
    const int sel = (I.masked ? 2 : 0) | (I.efield ? 1 : 0) | (a.plan ? 4 : 0);
    switch (sel) {
        case 0: tile_body<false, false, ADJ>(a, e.y, lds); break;
        case 1: tile_body<false, true, ADJ>(a, e.y, lds); break;
        case 2: tile_body<true, false, ADJ>(a, e.y, lds); break;
        case 3: tile_body<true, true, ADJ>(a, e.y, lds); break;
        case 4: tile_body<false, false, ADJ, true>(a, e.y, lds); break;
        case 5: tile_body<false, true, ADJ, true>(a, e.y, lds); break;
        case 6: tile_body<true, false, ADJ, true>(a, e.y, lds); break;
        default: tile_body<true, true, ADJ, true>(a, e.y, lds); break;
    }
}

// One block per instance: instances flagged in the mask test their residual.
__global__ __launch_bounds__(kBlock) void k_residual_batch(const BatchInst* __restrict__ inst, int adjoint,
                                                          uint64_t check_lo, uint64_t check_hi, double tol,
                                                          int64_t t)
{
    const int i = blockIdx.x;
    if (!mask_bit(check_lo, check_hi, i)) return;
    const BatchInst& I = inst[i];
    Status* st = I.status;
    if (st->stop) return;
    const double* partial = adjoint ? I.adj[0].partial : I.prim[0].partial;
    double a = 0.0, b = 0.0;
    for (int64_t k = threadIdx.x; k < I.nblk; k += kBlock) {
        a += partial[2 * k];
        b += partial[2 * k + 1];
    }
    __shared__ double out[2];
    block_sum2(a, b, out);
    if (threadIdx.x == 0) {
        double num = out[0], den = out[1];
        double r = den > 0.0 ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
        st->res = r;
        st->t_last = t;
        if (r < tol) {
            st->stop = 1;
            st->t_conv = t;
        }
    }
}

__global__ void k_status_reset_all(Status* st, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        st[i].stop = 0;
        st[i].nwin = 0;
        st[i].t_conv = -1;
        st[i].t_last = -1;
        st[i].res = INFINITY;
    }
}

// ---------------------------------------------------------------- persistent batch sweeps
// One launch of kPersistBlock-thread workgroups, one per compute unit, that
// advances every instance of a batch round after round until all of them
// have stopped (or a round budget ends the launch; the next launch resumes).
// Each instance keeps its own step counter, buffer parity and residual-check
// schedule (its own K): in a round it runs one fused launch's worth of steps
// (an LDS tile sweep of up to `halo` steps; periodic instances are tiled
// too), or one single step (a residual-check step, or the plain steps before
// its next check or its last step), or, after a check step, the reduction of
// its residual, which sets its stop flag.  The round's work items (tiles,
// 1024-node blocks, reductions) of all running instances form one list that
// the workgroups take from with an atomic counter; a stopped instance has no
// items (it retires).  A grid barrier ends every round.
//
// The per-instance state machine is replicated: thread i of every workgroup
// holds instance i's state and applies the same update after each barrier,
// from data every workgroup reads identically (the round's decisions and the
// stop flags written before the barrier), so all workgroups agree on every
// round without another barrier.  Every wait is bounded: a barrier that does
// not complete within kPersistSpin polls sets the error flag and the launch
// ends (the host reports an error) instead of hanging.
constexpr int kPersistBlock = 1024;
constexpr int kMaxBatch = 128;
constexpr long kPersistSpin = 1L << 26;     // about 4 s of 64-cycle sleeps
enum { PS_RUN = 0, PS_RESID = 1, PS_DONE = 2 };
enum { PT_NONE = 0, PT_FUSED = 1, PT_SINGLE = 2, PT_CHECK = 3, PT_RESID = 4 };

struct PersistInst {
    int64_t K;          // check interval
    int64_t last;       // final step index (max_steps)
    int32_t ntiles;     // tiles of a fused round (tile of 32 - 2 halo nodes, halo = the batch's tile steps Tt)
    int32_t nnb;        // 1024-node blocks of a single step
    int32_t halo;       // steps a fused round may take (tile halo)
    int32_t pad;
};

struct PersistState {
    int64_t s;          // next step to run
    int64_t t_chk;      // step of the latest check
    int32_t cur;        // buffer parity holding the input of step s
    int32_t phase;      // PS_*
    int32_t x_chk;      // input parity of the latest check step
    int32_t x_last;     // input parity of the final step (runs that end at max_steps)
};

struct PersistCtl {
    uint32_t cnt[2];        // work-item counters of alternate rounds
    uint32_t arrive;        // grid barrier: groups arrived
    uint32_t gen;           // grid barrier: generation
    int32_t error;          // a barrier timed out
    int32_t done;           // every instance has stopped
    int32_t budget;         // rounds per launch
    int32_t pad;
    int64_t rounds;         // rounds run so far (all launches of a solve)
    uint32_t grp[kXcds][32];  // grid barrier: workgroups arrived per group (one 128-byte line each)
};

// Sums (a, b) over the kPersistBlock threads into out[0], out[1] (thread 0 writes).
__device__ __forceinline__ void block_sum2_persist(double a, double b, double* out)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    __shared__ double pa[kPersistBlock / 64], pb[kPersistBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { pa[w] = a; pb[w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
#pragma unroll
        for (int i = 0; i < kPersistBlock / 64; ++i) { x += pa[i]; y += pb[i]; }
        out[0] = x;
        out[1] = y;
    }
}

// Grid barrier over nwg workgroups with device-scope release/acquire; false
// if it timed out or another workgroup reported an error.  Two levels: the
// workgroups of a group (those of one XCD: workgroup b runs on XCD b % 8)
// count on the group's own counter, and the last of each group on the
// global one, so no counter takes more than one XCD's arrivals.
__device__ __forceinline__ bool persist_barrier(PersistCtl* ctl, uint32_t nwg)
{
    __shared__ int ok_s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __threadfence();
        const uint32_t ngrp = nwg < (uint32_t)kXcds ? nwg : (uint32_t)kXcds;
        const uint32_t grp = blockIdx.x % ngrp;
        const uint32_t in_grp = nwg / ngrp + (grp < nwg % ngrp ? 1u : 0u);
        const uint32_t g = __hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool last = false;
        if (__hip_atomic_fetch_add(&ctl->grp[grp][0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == in_grp - 1) {
            __hip_atomic_store(&ctl->grp[grp][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = __hip_atomic_fetch_add(&ctl->arrive, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == ngrp - 1;
        }
        if (last) {
            __hip_atomic_store(&ctl->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&ctl->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long spins = 0;
            while (__hip_atomic_load(&ctl->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kPersistSpin ||
                    ((spins & 1023) == 0 && __hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                    __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
            }
        }
        __threadfence();
        ok_s = ok;
    }
    __syncthreads();
    return ok_s != 0;
}

// Round decision of one running instance (mirrors the single-problem solve
// loop: check steps at s > 0, s % K == 0; the last step and leftovers are
// single steps; plain runs between checks are fused up to `halo` steps).
__device__ __forceinline__ void persist_decide(const PersistInst& P, const PersistState& st, bool use_tol,
                                               int& type, int& k, int& items)
{
    type = PT_NONE;
    k = 0;
    items = 0;
    if (st.phase == PS_DONE) return;
    if (st.phase == PS_RESID) {
        type = PT_RESID;
        items = 1;
        return;
    }
    const int64_t s = st.s;
    if (use_tol && s > 0 && s % P.K == 0) {
        type = PT_CHECK;
        k = 1;
        items = P.nnb;
        return;
    }
    const int64_t end = use_tol ? min(P.last, (s / P.K + 1) * P.K - 1) : P.last;
    const int64_t plain = min(end, P.last - 1) - s + 1;
    if (P.halo > 1 && plain >= 2) {
        type = PT_FUSED;
        k = (int)min(plain, (int64_t)P.halo);
        items = P.ntiles;
        return;
    }
    type = PT_SINGLE;
    k = 1;
    items = P.nnb;
}

// State after a round of the given type (stopped: the instance's stop flag,
// read after the barrier; only used after a reduction).
__device__ __forceinline__ void persist_update(const PersistInst& P, PersistState& st, int type, int k,
                                               bool stopped)
{
    switch (type) {
        case PT_FUSED:
            st.s += k;
            st.cur ^= 1;
            break;
        case PT_SINGLE:
        case PT_CHECK:
            if (type == PT_CHECK) {
                st.t_chk = st.s;
                st.x_chk = st.cur;
                st.phase = PS_RESID;
            }
            if (st.s == P.last) st.x_last = st.cur;
            st.s += 1;
            st.cur ^= 1;
            if (type == PT_SINGLE && st.s > P.last) st.phase = PS_DONE;
            break;
        case PT_RESID:
            st.phase = (stopped || st.s > P.last) ? PS_DONE : PS_RUN;
            break;
        default:
            break;
    }
}

// One 1024-node block of a single step (with the residual terms on check steps).
template <bool ADJ>
__device__ __forceinline__ void persist_nodes(const BatchInst& I, int par, int blk, bool check)
{
    const SweepArgs& a = ADJ ? I.adj[par] : I.prim[par];
    const int64_t n = (int64_t)blk * kPersistBlock + threadIdx.x;
    double num = 0.0, den = 0.0;
    if (n < a.N) {
        const int sel = (I.masked ? 4 : 0) | (I.efield ? 2 : 0) | (check ? 1 : 0);
#define BN_CASE(i, M, EF, CH)                                                       \
    case i:                                                                         \
        if (ADJ) adjoint_node<M, EF, CH>(a, n, I.inv_nx, num, den);                 \
        else primal_node<M, EF, CH>(a, n, I.inv_nx, num, den);                      \
        break;
        switch (sel) {
            BN_CASE(0, false, false, false)
            BN_CASE(1, false, false, true)
            BN_CASE(2, false, true, false)
            BN_CASE(3, false, true, true)
            BN_CASE(4, true, false, false)
            BN_CASE(5, true, false, true)
            BN_CASE(6, true, true, false)
            BN_CASE(7, true, true, true)
        }
#undef BN_CASE
    }
    if (check) block_sum2_persist(num, den, a.partial + 2 * (int64_t)blk);
}

// Residual test of an instance after its check step t: the sum of its nnb
// partial pairs in block order, then stop if below tol.
__device__ __forceinline__ void persist_resid(const BatchInst& I, const PersistInst& P, double tol, int64_t t)
{
    const double* partial = I.prim[0].partial;
    double a = 0.0, b = 0.0;
    for (int64_t k = threadIdx.x; k < P.nnb; k += kPersistBlock) {
        a += partial[2 * k];
        b += partial[2 * k + 1];
    }
    __shared__ double out[2];
    block_sum2_persist(a, b, out);
    if (threadIdx.x == 0) {
        Status* st = I.status;
        const double num = out[0], den = out[1];
        const double r = den > 0.0 ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
        st->res = r;
        st->t_last = t;
        if (r < tol) {
            st->t_conv = t;
            __hip_atomic_store(&st->stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <bool ADJ>
__global__ __launch_bounds__(kPersistBlock) void k_batch_persist(const BatchInst* __restrict__ inst,
                                                                 const PersistInst* __restrict__ pinst, int B,
                                                                 PersistState* prep, PersistCtl* ctl,
                                                                 int use_tol, double tol, int maxb)
{
    extern __shared__ __align__(16) double lds[];
    __shared__ int s_dec[kMaxBatch];              // round decision: type | k << 3 | cur << 8
    __shared__ int s_pre[kMaxBatch + 1];          // work items of instances < i
    __shared__ int s_item[3];
    const int tid = threadIdx.x;
    // this workgroup's replica of the instances' states (all replicas evolve alike)
    PersistState* rep = prep + (int64_t)blockIdx.x * B;
    const int budget = ctl->budget;
    int round = 0;
    bool all_done = false;
    for (;;) {
        if (tid < B) {
            const PersistState st = rep[tid];
            int type, k, items;
            persist_decide(pinst[tid], st, use_tol != 0, type, k, items);
            s_dec[tid] = type | (k << 3) | (st.cur << 8);
            s_pre[tid + 1] = items;
        }
        __syncthreads();
        if (tid == 0) {
            s_pre[0] = 0;
            for (int i = 0; i < B; ++i) s_pre[i + 1] += s_pre[i];
        }
        __syncthreads();
        const int total = s_pre[B];
        if (total == 0) {
            all_done = true;
            break;
        }
        if (round >= budget) break;
        const int slot = round & 1;
        // the other counter was last used a round ago: every workgroup finished
        // taking from it before the barrier that ended that round
        if (blockIdx.x == 0 && tid == 0)
            __hip_atomic_store(&ctl->cnt[slot ^ 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (;;) {
            if (tid == 0) {
                const int it = (int)__hip_atomic_fetch_add(&ctl->cnt[slot], 1u, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                int lo = 0, hi = B;                       // instance: s_pre[lo] <= it < s_pre[lo + 1]
                if (it < total) {
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_pre[mid] <= it) lo = mid;
                        else hi = mid;
                    }
                }
                s_item[0] = it;
                s_item[1] = lo;
                s_item[2] = it - s_pre[lo];
            }
            __syncthreads();
            const int it = s_item[0], i = s_item[1], loc = s_item[2];
            __syncthreads();
            if (it >= total) break;
            const BatchInst& I = inst[i];
            const int dec = s_dec[i], ty = dec & 7, par = (dec >> 8) & 1;
            if (ty == PT_FUSED) {
                TileArgs a = ADJ ? I.ladj[par] : I.lprim[par];
                a.steps = (dec >> 3) & 31;
                a.maxb = min(a.maxb, maxb);
                const int sel = (I.masked ? 2 : 0) | (I.efield ? 1 : 0);
                switch (sel) {
                    case 0: tile_body<false, false, ADJ>(a, loc, lds); break;
                    case 1: tile_body<false, true, ADJ>(a, loc, lds); break;
                    case 2: tile_body<true, false, ADJ>(a, loc, lds); break;
                    default: tile_body<true, true, ADJ>(a, loc, lds); break;
                }
            } else if (ty == PT_SINGLE || ty == PT_CHECK) {
                persist_nodes<ADJ>(I, par, loc, ty == PT_CHECK);
            } else if (ty == PT_RESID) {
                persist_resid(I, pinst[i], tol, rep[i].s - 1);    // the check step was s - 1
            }
            __syncthreads();
        }
        if (!persist_barrier(ctl, gridDim.x)) return;
        if (tid < B) {
            PersistState st = rep[tid];
            const int dec = s_dec[tid], type = dec & 7;
            const bool stopped = type == PT_RESID &&
                                 __hip_atomic_load(&inst[tid].status->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            persist_update(pinst[tid], st, type, (dec >> 3) & 31, stopped);
            rep[tid] = st;
        }
        ++round;
    }
    if (blockIdx.x == 0 && tid == 0) {
        ctl->done = all_done ? 1 : 0;
        ctl->rounds += round;
    }
}

// Start of a persistent launch (a graph node, so no memset node): clears the
// round counters and the barrier, sets the round budget.
__global__ void k_persist_begin(PersistCtl* ctl, int budget)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->cnt[0] = ctl->cnt[1] = 0;
        ctl->arrive = 0;
        for (int k = 0; k < kXcds; ++k) ctl->grp[k][0] = 0;
        ctl->gen = 0;
        ctl->error = 0;
        ctl->done = 0;
        ctl->budget = budget;
    }
}

// Start of a persistent solve: every instance at step 0 from buffer 0, in
// each of the n = workgroups x B replicas.
__global__ void k_persist_init(PersistState* st, PersistCtl* ctl, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        st[i].s = 0;
        st[i].t_chk = -1;
        st[i].cur = 0;
        st[i].phase = PS_RUN;
        st[i].x_chk = 0;
        st[i].x_last = 0;
    }
    if (i == 0) ctl->rounds = 0;
}

}  // namespace slbm
