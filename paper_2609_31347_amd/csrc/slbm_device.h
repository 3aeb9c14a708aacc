// Device-side arithmetic of the solid lattice-Boltzmann scheme for gfx950.
//
// D2Q8 moment-space collision (paper eq. moments, eq. gamma, eq. forcing,
// eq. moments_bar_1/2, eq. moments_eq, eq. moments_c, eq. relaxation,
// eq. moments_c_10/01, eq. bared_moments, eq. local_collide, appendix matrix M
// and relaxation-time table) written out in closed form; the boundary-link
// closures; the transposed bulk collision of the adjoint (eq.
// adjoint_collision); a forward-mode dual number used for derivatives w.r.t.
// Young's modulus in the gradient (eq. optimality).
//
// Direction order Q (eq. direction_order):
//   0:(1,0) 1:(0,1) 2:(-1,0) 3:(0,-1) 4:(1,1) 5:(-1,1) 6:(-1,-1) 7:(1,-1)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slbm {

constexpr double kTheta = 1.0 / 3.0;
constexpr double kTauF = 0.5;  // tau_12 = tau_21 = tau_f = 1/2 (omega = 1)

__host__ __device__ constexpr int cx(int q) { return q == 0 || q == 4 || q == 7 ? 1 : (q == 2 || q == 5 || q == 6 ? -1 : 0); }
__host__ __device__ constexpr int cy(int q) { return q == 1 || q == 4 || q == 5 ? 1 : (q == 3 || q == 6 || q == 7 ? -1 : 0); }
__host__ __device__ constexpr int opp(int q) { return q < 4 ? (q + 2) & 3 : 4 + ((q - 4 + 2) & 3); }

// ---------------------------------------------------------------- dual numbers
// Forward-mode AD value: v + d * eps, eps^2 = 0.
struct Dual {
    double v, d;
    __host__ __device__ Dual() : v(0.0), d(0.0) {}
    __host__ __device__ Dual(double a) : v(a), d(0.0) {}
    __host__ __device__ Dual(double a, double b) : v(a), d(b) {}
};
__host__ __device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__host__ __device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__host__ __device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__host__ __device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__host__ __device__ inline Dual operator/(Dual a, Dual b)
{
    double iv = 1.0 / b.v;
    return Dual(a.v * iv, (a.d - a.v * iv * b.d) * iv);
}
__host__ __device__ inline double val(double a) { return a; }
__host__ __device__ inline double val(Dual a) { return a.v; }
__host__ __device__ inline double der(double) { return 0.0; }
__host__ __device__ inline double der(Dual a) { return a.d; }

// ---------------------------------------------------------------- relaxation
// Relaxation of one node: keep factors k = 1 - omega of the second-order
// moments (m11, m_s, m_d) and the boundary coefficient gamma (0 in the bulk).
template <class T>
struct Relax {
    T k11, ks, kd, gam;
};

// Plane-stress moduli mu = E/(2(1+nu)), K = E/(2(1-nu)) (eq. mu, eq. K);
// tau_11 = mu/theta, tau_s = 2K/(1+theta), tau_d = 2mu/(1-theta); omega =
// 1/(tau + 1/2) (eq. relaxation); gamma of eq. gamma at boundary nodes.
// With theta = 1/3 these reduce to tau_11 = tau_d = 3 mu = E * 3/(2(1+nu)),
// tau_s = 3K/2 = E * 3/(4(1-nu)) and gamma = (theta tau_f/(1+theta)) /
// (tau_s - tau_f) = (1/8)/(tau_s - 1/2): two divisions per node (one more at
// boundary nodes) instead of nine, the same values up to rounding.
template <class T>
__host__ __device__ inline Relax<T> relax_from_E(T E, double nu, bool boundary)
{
    const T t11 = E * T(1.5 / (1.0 + nu));      // tau_11 = tau_d
    const T ts = E * T(0.75 / (1.0 - nu));
    Relax<T> r;
    r.k11 = T(1.0) - T(1.0) / (t11 + T(0.5));
    r.kd = r.k11;
    r.ks = T(1.0) - T(1.0) / (ts + T(0.5));
    r.gam = boundary ? T(kTheta * kTauF / (1.0 + kTheta)) / (ts - T(kTauF)) : T(0.0);
    return r;
}

// ---------------------------------------------------------------- boundary records
// One plate boundary node (a domain node with at least one cut link).
struct BNode {
    int32_t cell;        // linear cell index iy * nx + ix
    uint32_t cut;        // bit q set: x - c_q is outside (f_q needs a closure)
    uint32_t dirichlet;  // bit q set: that closure is Dirichlet, else Neumann
    uint32_t pad;
    // closure of cut link q as an affine form of the node's bared stress:
    // h_q = +-fC_qbar + k[0] sxx + k[1] syy + k[2] sxy + k[3]
    // (+ for Dirichlet, - for Neumann; k[3] carries the wall data d_D or T)
    double coef[8][4];
};

// Closure coefficients of one cut link (host, at set-up).  The closures
// (the paper defers their formulas; this is the library's own first-order
// design, wall point at the link midpoint):
//   Dirichlet  h_q = fC_qbar + 2 W_q c_q . d_D,   W = 1/3 (axis), 1/12 (diagonal)
//              (W_q c_q . d are the populations whose moments are N d)
//   Neumann    h_q = -fC_qbar + 2 fsig_q(sigma_w),  fsig the populations with
//              second moments -sigma_w and no others; sigma_w = the node's bared
//              stress sigma with its traction on the wall normal n replaced by T:
//              sigma_w = sigma + n a^T + a n^T - (a.n) n n^T,  a = T - sigma n.
// sigma_w is linear in (sigma, T), so 2 fsig_q(sigma_w) = u . sigma + v(T);
// u and v are formed by evaluating that map on unit stresses and on T.
inline double neumann_closure(int q, double sxx, double syy, double sxy, double tx, double ty, double nx,
                              double ny)
{
    double ax = tx - (sxx * nx + sxy * ny);
    double ay = ty - (sxy * nx + syy * ny);
    double an = ax * nx + ay * ny;
    double wxx = sxx + 2.0 * nx * ax - an * nx * nx;
    double wyy = syy + 2.0 * ny * ay - an * ny * ny;
    double wxy = sxy + ax * ny + ay * nx - an * nx * ny;
    double fs = q == 0 || q == 2 ? -0.5 * wxx : q == 1 || q == 3 ? -0.5 * wyy : q == 4 || q == 6 ? -0.25 * wxy
                                                                                                  : 0.25 * wxy;
    return 2.0 * fs;
}

inline void closure_coefs(int q, bool dirichlet, double w0, double w1, double nx, double ny, double k[4])
{
    if (dirichlet) {
        const double W = q < 4 ? 1.0 / 3.0 : 1.0 / 12.0;
        k[0] = k[1] = k[2] = 0.0;
        k[3] = 2.0 * W * (cx(q) * w0 + cy(q) * w1);
        return;
    }
    k[0] = neumann_closure(q, 1.0, 0.0, 0.0, 0.0, 0.0, nx, ny);
    k[1] = neumann_closure(q, 0.0, 1.0, 0.0, 0.0, 0.0, nx, ny);
    k[2] = neumann_closure(q, 0.0, 0.0, 1.0, 0.0, 0.0, nx, ny);
    k[3] = neumann_closure(q, 0.0, 0.0, 0.0, w0, w1, nx, ny);
}

// ---------------------------------------------------------------- node map
// Extended node map: populations f^S of one node and its forcing g ->
// post-collision populations fC (streamed to x + c_q) and the closure values
// h_q of the cut links (taken as f^S_q(x) at the next step).  mb holds the
// bared moments (m10, m01, m11, m_s, m_d).
//
// Closures: the affine forms of BNode::coef (see closure_coefs); with_walls
// = false drops the wall terms (the linear part, for the adjoint Jacobian).
// SPARSE reads the coefficients of cut links only, behind a branch per link
// (a wave skips a link none of its nodes has cut); the default forms all
// eight links and selects, so that records in HBM are fetched together.
// Both give the same values.
template <class T, bool SPARSE = false>
__host__ __device__ inline void node_map(const T f[8], const T g[2], const Relax<T>& r,
                                         const BNode* bn, bool with_walls, T fC[8], T h[8],
                                         T mb[5])
{
    // raw moments (rows of M); m_f = m22 + gamma m_s
    T m10 = f[0] - f[2] + f[4] - f[5] - f[6] + f[7];
    T m01 = f[1] - f[3] + f[4] + f[5] - f[6] - f[7];
    T m11 = f[4] - f[5] + f[6] - f[7];
    T ms = (f[0] + f[1] + f[2] + f[3]) + T(2.0) * (f[4] + f[5] + f[6] + f[7]);
    T md = f[0] - f[1] + f[2] - f[3];
    T mb10 = m10 + T(0.5) * g[0];
    T mb01 = m01 + T(0.5) * g[1];
    T c10 = mb10 + T(0.5) * g[0];
    T c01 = mb01 + T(0.5) * g[1];
    T c11 = r.k11 * m11;
    T cs = r.ks * ms;
    T cd = r.kd * md;
    T c12 = T(kTheta) * mb10;       // omega_12 = 1: equilibrium theta * mb10
    T c21 = T(kTheta) * mb01;
    T c22 = -(r.gam * cs);          // m_f relaxed to 0 (omega_f = 1), m22 = m_f - gamma m_s
    // populations = M^{-1} m^C
    T a = c10 - c12, b = c01 - c21, s = cs - T(2.0) * c22;
    fC[0] = T(0.25) * (T(2.0) * a + s + cd);
    fC[2] = T(0.25) * (s + cd - T(2.0) * a);
    fC[1] = T(0.25) * (T(2.0) * b + s - cd);
    fC[3] = T(0.25) * (s - cd - T(2.0) * b);
    fC[4] = T(0.25) * (c11 + c12 + c21 + c22);
    fC[5] = T(0.25) * (c21 + c22 - c11 - c12);
    fC[6] = T(0.25) * (c11 + c22 - c12 - c21);
    fC[7] = T(0.25) * (c12 + c22 - c11 - c21);
    // bared moments (eq. bared_moments)
    mb[0] = mb10;
    mb[1] = mb01;
    mb[2] = T(0.5) * (m11 + c11);
    mb[3] = T(0.5) * (ms + cs);
    mb[4] = T(0.5) * (md + cd);
    if (!bn) return;
    // bared stress sigma = -[[m20, m11], [m11, m02]]
    T sxx = -T(0.5) * (mb[3] + mb[4]);
    T syy = -T(0.5) * (mb[3] - mb[4]);
    T sxy = -mb[2];
    // branch-free: all eight links are formed and the cut bits select, so the
    // record's loads go out together
    const uint32_t cut = bn->cut, dir = bn->dirichlet;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (SPARSE) {
            h[q] = T(0.0);
            if (!((cut >> q) & 1u)) continue;
        }
        const double* k = bn->coef[q];
        T lin = T(k[0]) * sxx + T(k[1]) * syy + T(k[2]) * sxy;
        if (with_walls) lin = lin + T(k[3]);
        T hq = (((dir >> q) & 1u) ? fC[opp(q)] : -fC[opp(q)]) + lin;
        h[q] = ((cut >> q) & 1u) ? hq : T(0.0);
    }
}

// ---------------------------------------------------------------- bulk fast paths
// Bulk collision (gamma = 0) in double: f (in) -> fC (out, may alias f).
// hx, hy are a quarter of the forcing (g / 4, exact in binary).  Returns the
// bared displacement in d0, d1.  The same map as node_map without boundary
// terms, with shared sums and differences of the populations and the constant
// factors folded into multiply-adds:
//   mb10 = m10 + g_x / 2,  fC_0,2 = Sp +- ha,  fC_1,3 = Sm +- hb,
//   Sp = (ks + kd)/4 (f0 + f2) + (ks - kd)/4 (f1 + f3) + ks/2 (f4 + f5 + f6 + f7),
//   Sm likewise with (ks + kd) and (ks - kd) swapped,  ha = (1 - theta)/2 mb10 + g_x/4,
//   fC_4 = U + t mb10, fC_5 = -(V + t mb10), fC_6 = V - t mb10, fC_7 = t mb10 - U,
//   U, V = k11/4 m11 +- t mb01,  t = theta/4.
__device__ __forceinline__ void collide_bulk(double f[8], double hx, double hy, double k11, double ks,
                                             double kd, double& d0, double& d1)
{
    const double d02 = f[0] - f[2], d13 = f[1] - f[3];
    const double d45 = f[4] - f[5], d67 = f[6] - f[7];
    const double p45 = f[4] + f[5], p67 = f[6] + f[7];
    const double p02 = f[0] + f[2], p13 = f[1] + f[3];
    const double mb10 = fma(2.0, hx, d02 + (d45 - d67));
    const double mb01 = fma(2.0, hy, d13 + (p45 - p67));
    d0 = mb10;
    d1 = mb01;
    const double ha = fma(0.5 * (1.0 - kTheta), mb10, hx);
    const double hb = fma(0.5 * (1.0 - kTheta), mb01, hy);
    const double u = (0.5 * ks) * (p45 + p67);
    const double A = 0.25 * (ks + kd), B = 0.25 * (ks - kd);
    const double Sp = fma(A, p02, fma(B, p13, u));
    const double Sm = fma(B, p02, fma(A, p13, u));
    f[0] = Sp + ha;
    f[2] = Sp - ha;
    f[1] = Sm + hb;
    f[3] = Sm - hb;
    constexpr double t = 0.25 * kTheta;
    const double R = (0.25 * k11) * (d45 + d67);
    const double U = fma(t, mb01, R), V = fma(-t, mb01, R);
    f[4] = fma(t, mb10, U);
    f[5] = fma(-t, mb10, -V);
    f[6] = fma(-t, mb10, V);
    f[7] = fma(t, mb10, -U);
}

// psi = M^{-T} phi (adjoint in moment space): (psi10, psi01, psi11, psi_s, psi_d, psi12, psi21)
__host__ __device__ inline void adj_moments(const double p[8], double psi[7])
{
    psi[0] = 0.5 * (p[0] - p[2]);
    psi[1] = 0.5 * (p[1] - p[3]);
    psi[2] = 0.25 * ((p[4] - p[5]) + (p[6] - p[7]));
    psi[3] = 0.25 * ((p[0] + p[1]) + (p[2] + p[3]));
    psi[4] = 0.25 * ((p[0] - p[1]) + (p[2] - p[3]));
    psi[5] = 0.25 * (2.0 * (p[2] - p[0]) + (p[4] - p[5]) + (p[7] - p[6]));
    psi[6] = 0.25 * (2.0 * (p[3] - p[1]) + (p[4] + p[5]) - (p[6] + p[7]));
}

// Transposed bulk collision: phi (= phi^S, in) -> phi^C = C^T phi^S - s (r . c_q) (out, may alias).
// C = M^{-1} A M, so C^T = M^T A^T M^{-T}; A^T maps psi = M^{-T} phi to
//   chi10 = psi10 + theta psi12, chi01 = psi01 + theta psi21,
//   chi11 = k11 psi11, chi_s = ks psi_s, chi_d = kd psi_d   (others 0),
// and M^T chi gives the populations.  The source -(dJ/df)^T = -s (r_x c_x + r_y c_y)
// enters as chi10 -= s r_x, chi01 -= s r_y.  Written out with shared sums and
// differences:  chi10 = (1 - theta)/2 (p0 - p2) + theta/4 ((p4 - p5) - (p6 - p7)) - s r_x,
// chi01 = (1 - theta)/2 (p1 - p3) + theta/4 ((p4 + p5) - (p6 + p7)) - s r_y,
// chi11 = k11/4 ((p4 - p5) + (p6 - p7)), chi_s = ks/4 ((p0 + p2) + (p1 + p3)),
// chi_d = kd/4 ((p0 + p2) - (p1 + p3)).
__device__ __forceinline__ void adj_collide_bulk(double p[8], double srx, double sry, double k11,
                                                 double ks, double kd)
{
    const double d02 = p[0] - p[2], d13 = p[1] - p[3];
    const double d45 = p[4] - p[5], d67 = p[6] - p[7];
    const double p45 = p[4] + p[5], p67 = p[6] + p[7];
    const double s02 = p[0] + p[2], s13 = p[1] + p[3];
    const double x10 = 0.5 * (1.0 - kTheta) * d02 + (0.25 * kTheta) * (d45 - d67) - srx;
    const double x01 = 0.5 * (1.0 - kTheta) * d13 + (0.25 * kTheta) * (p45 - p67) - sry;
    const double x11 = (0.25 * k11) * (d45 + d67);
    const double xs = (0.25 * ks) * (s02 + s13);
    const double xd = (0.25 * kd) * (s02 - s13);
    const double Ep = xs + xd, Em = xs - xd;
    p[0] = Ep + x10;
    p[2] = Ep - x10;
    p[1] = Em + x01;
    p[3] = Em - x01;
    const double G = x10 + x01, H = x10 - x01;
    const double T4 = 2.0 * xs + x11, T5 = 2.0 * xs - x11;
    p[4] = T4 + G;
    p[6] = T4 - G;
    p[5] = T5 - H;
    p[7] = T5 + H;
}

// Transposed map of a boundary node (eq. adjoint_collision at nodes with cut
// links): the adjoint of the linear part of node_map (with_walls = false),
//   fC = C_b f,  h_q = s_q fC_qbar + u_q . sigma(f)   (s_q = +1 Dirichlet, -1 Neumann),
// applied to yf (adjoint of fC, pulled from x + c_q) and yh (adjoint of the
// closure values, the node's own slots of its cut links, 0 elsewhere):
//   out = C_b^T (yf + sum_q s_q yh_q e_qbar) + (d sigma / d f)^T (sum_q yh_q u_q) - s (r . c_q).
// C_b = M^{-1} A_b M differs from the bulk collision by m_f = 0 after the
// collision, m22 = -gamma k_s m_s; the transpose runs through the moments as
// adj_collide_bulk does and equals it for gamma = 0 and no cut links.
// SPARSE: as in node_map, only cut links (yh is 0 on the others) are read.
template <bool SPARSE = false>
__host__ __device__ inline void adj_boundary(const double yf[8], const double yh[8], const BNode* bn,
                                             const Relax<double>& r, double srx, double sry, double out[8])
{
    const uint32_t dir = bn->dirichlet;
    double z[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) z[q] = yf[q];
    double w0 = 0.0, w1 = 0.0, w2 = 0.0;
    const uint32_t cut = SPARSE ? bn->cut : 0xffu;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (!((cut >> q) & 1u)) continue;
        const double y = yh[q];
        z[opp(q)] += ((dir >> q) & 1u) ? y : -y;
        w0 += y * bn->coef[q][0];
        w1 += y * bn->coef[q][1];
        w2 += y * bn->coef[q][2];
    }
    // gradients w.r.t. the post-collision moments (M^{-T} z)
    const double pa = 0.5 * (z[0] - z[2]), pb = 0.5 * (z[1] - z[3]);
    const double ps = 0.25 * ((z[0] + z[1]) + (z[2] + z[3]));
    const double pd = 0.25 * ((z[0] - z[1]) + (z[2] - z[3]));
    const double p11 = 0.25 * ((z[4] - z[5]) + (z[6] - z[7]));
    const double p12 = 0.25 * ((z[4] - z[5]) - (z[6] - z[7]));
    const double p21 = 0.25 * ((z[4] + z[5]) - (z[6] + z[7]));
    const double p22 = 0.25 * ((z[4] + z[5]) + (z[6] + z[7]));
    // gradients w.r.t. the pre-collision moments; stress term: sxx = -(mb_s + mb_d)/2,
    // syy = -(mb_s - mb_d)/2, sxy = -mb_11 with mb = (1 + k) m / 2
    const double g10 = (1.0 - kTheta) * pa + kTheta * p12 - srx;
    const double g01 = (1.0 - kTheta) * pb + kTheta * p21 - sry;
    const double g11 = r.k11 * p11 - 0.5 * (1.0 + r.k11) * w2;
    const double gs = r.ks * ((1.0 + 2.0 * r.gam) * ps - r.gam * p22) - 0.25 * (1.0 + r.ks) * (w0 + w1);
    const double gd = r.kd * pd - 0.25 * (1.0 + r.kd) * (w0 - w1);
    // M^T g
    out[0] = g10 + gs + gd;
    out[1] = g01 + gs - gd;
    out[2] = gs + gd - g10;
    out[3] = gs - gd - g01;
    const double t = 2.0 * gs;
    out[4] = t + g11 + (g10 + g01);
    out[5] = t - g11 + (g01 - g10);
    out[6] = t + g11 - (g10 + g01);
    out[7] = t - g11 + (g10 - g01);
}

}  // namespace slbm
