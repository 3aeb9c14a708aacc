/*
 * slbm_oracle.c -- CPU oracle of the solid lattice-Boltzmann primal sweep,
 * its discrete adjoint (ALBM) and the objective gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded FP64 C written from
 * the paper's equations, built with -O2 -ffp-contract=off.  It shares no code
 * with the HIP library; only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  The product path never does.
 *
 * What it computes (paper: "Benchmark cases for gradient-based optimization in
 * linear elastic solid mechanics using lattice Boltzmann methods"):
 *  - D2Q8 moment-space MRT collision with half-force forcing
 *    (Sec. "LBM scheme for solids": eq. moments, eq. gamma, eq. forcing,
 *    eq. moments_bar_1/2, eq. moments_eq, eq. moments_c, eq. relaxation,
 *    eq. moments_c_10/01, eq. bared_moments, eq. local_collide; appendix
 *    matrix M and the relaxation-time table), pure index-shift streaming
 *    (eq. local_stream) on a periodic box.
 *  - Boundary closures for a plate in a box (reading C13; the paper defers the
 *    closure formulas to other work): per cut link, Dirichlet bounce-back with
 *    wall displacement, Neumann anti-bounce-back with wall stress whose normal
 *    traction is T; the gamma-modified moment m_f at boundary nodes.
 *    Parity unpinned against the paper's own closures (their formulas are not
 *    given); pinned instead by first-order convergence on the paper's elliptic
 *    plate, the sparse direct fixed point and finite differences.
 *  - The steady state by pseudo-time marching with the K-lag residual and a
 *    two-step average (readings C6, C7).
 *  - The adjoint fixed-point iteration (eq. adjoint_streaming,
 *    eq. adjoint_collision, eq. adjoint_iteration, eq. adjoint_init): the node
 *    Jacobian is obtained by applying the (affine) node map to unit vectors and
 *    is then transposed -- no hand-derived transpose.
 *  - The local pieces of the optimality condition (eq. optimality): the
 *    derivative of the node map w.r.t. the forcing (unit-vector probes) and
 *    w.r.t. Young's modulus (complex step).
 *  - A complex-step instance of the whole primal solve: the forward-mode
 *    (f-AD, eq. fAD) derivative of the state along one control direction.
 *
 * Layouts: every field is SoA, component-major, x fastest:
 *   a[c * nx * ny + iy * nx + ix].  Per-link arrays use (c * 8 + q) as the
 *   component index.  Directions q follow the order Q of eq. direction_order.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_THETA (1.0 / 3.0)
#define ORC_TAU_F 0.5
#define ORC_BC_DIRICHLET 1
#define ORC_BC_NEUMANN 2

/* Direction order Q, eq. direction_order */
static const int orc_cx[8] = {1, 0, -1, 0, 1, -1, -1, 1};
static const int orc_cy[8] = {0, 1, 0, -1, 1, 1, -1, -1};
static const int orc_opp[8] = {2, 3, 0, 1, 6, 7, 4, 5};

/* Transformation matrix M (appendix "MRT transformation matrices"); rows give
 * (m10, m01, m11, m_s, m_d, m12, m21, m22) */
static const double orc_M[8][8] = {
    {1, 0, -1, 0, 1, -1, -1, 1},
    {0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, 0, 0, 1, -1, 1, -1},
    {1, 1, 1, 1, 2, 2, 2, 2},
    {1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 1, 1, -1, -1},
    {0, 0, 0, 0, 1, 1, 1, 1},
};
/* N of eq. moments_eq (transposed: row b = moment, columns = (m10bar, m01bar)) */
static const double orc_N[8][2] = {
    {1, 0}, {0, 1}, {0, 0}, {0, 0}, {0, 0}, {ORC_THETA, 0}, {0, ORC_THETA}, {0, 0},
};
static double orc_Minv[8][8];
static int orc_ready = 0;

/* Gauss-Jordan elimination with partial pivoting: orc_Minv = M^{-1}. */
static void orc_init(void)
{
    if (orc_ready) return;
    double a[8][16];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 16; ++j) a[i][j] = (j < 8) ? orc_M[i][j] : (j - 8 == i ? 1.0 : 0.0);
    for (int c = 0; c < 8; ++c) {
        int piv = c;
        for (int r = c + 1; r < 8; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        for (int j = 0; j < 16; ++j) { double t = a[c][j]; a[c][j] = a[piv][j]; a[piv][j] = t; }
        double d = a[c][c];
        for (int j = 0; j < 16; ++j) a[c][j] /= d;
        for (int r = 0; r < 8; ++r) {
            if (r == c) continue;
            double f = a[r][c];
            for (int j = 0; j < 16; ++j) a[r][j] -= f * a[c][j];
        }
    }
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) orc_Minv[i][j] = a[i][j + 8];
    orc_ready = 1;
}

/* Problem description (all arrays owned by the caller). */
typedef struct {
    int nx, ny;
    double dx;                 /* lattice spacing; dt = dx^2 */
    double nu;                 /* Poisson ratio */
    const double *E;           /* nx*ny Young's modulus per node (lattice units) */
    const unsigned char *active; /* nx*ny: 1 = node of the domain; NULL = all */
    const unsigned char *bc;   /* 8*nx*ny [q*N+n]: 0 interior link, 1 Dirichlet, 2 Neumann */
    const double *wall;        /* 2*8*nx*ny [(c*8+q)*N+n]: d_D or T (lattice units) */
    const double *normal;      /* 2*8*nx*ny: outward unit normal of Neumann links */
    const double *g;           /* 2*nx*ny forcing (lattice units) */
    int gamma_at_boundary;     /* 1: m_f = m_22 + gamma m_s at boundary nodes */
} orc_problem;

static int orc_is_active(const orc_problem *p, long n) { return p->active ? p->active[n] != 0 : 1; }
static int orc_is_boundary(const orc_problem *p, long n)
{
    if (!p->bc) return 0;
    long N = (long)p->nx * p->ny;
    for (int q = 0; q < 8; ++q)
        if (p->bc[(long)q * N + n]) return 1;
    return 0;
}
static double orc_re_r(double x) { return x; }
static double orc_re_c(double complex x) { return creal(x); }

/* ---- real instance ---- */
#define ORC_T double
#define ORC_SFX _r
#define orc_re orc_re_r
#include "slbm_oracle_body.h"
#undef ORC_T
#undef ORC_SFX
#undef orc_re
/* ---- complex instance ---- */
#define ORC_T double complex
#define ORC_SFX _c
#define ORC_IS_COMPLEX 1
#define orc_re orc_re_c
#include "slbm_oracle_body.h"
#undef ORC_T
#undef ORC_SFX
#undef ORC_IS_COMPLEX
#undef orc_re

/* ========================= exported entry points ========================= */

/* One primal step; disp (2N) / stress (3N, lattice units) of the input state. */
int orc_step(const orc_problem *p, const double *fS, double *fSn, double *disp, double *stress)
{
    orc_init();
    step_r(p, NULL, NULL, fS, fSn, disp, stress);
    return 0;
}

/* n primal steps in place. */
int orc_run(const orc_problem *p, double *fS, long nsteps)
{
    orc_init();
    long N = (long)p->nx * p->ny;
    double *tmp = (double *)malloc(sizeof(double) * 8 * N);
    for (long t = 0; t < nsteps; ++t) {
        step_r(p, NULL, NULL, fS, tmp, NULL, NULL);
        memcpy(fS, tmp, sizeof(double) * 8 * N);
    }
    free(tmp);
    return 0;
}

int orc_solve(const orc_problem *p, double *fS, double tol, long K, long max_steps,
              double *dbar, double *fbar, double *sbar, long *steps, double *res)
{
    orc_init();
    return solve_r(p, NULL, NULL, fS, tol, K, max_steps, dbar, fbar, sbar, steps, res);
}

/*
 * Complex-step primal solve: E + i*E_im, g + i*g_im.  State arrays are split
 * into real and imaginary parts (fS_re/fS_im in/out; outputs may be NULL).
 */
int orc_solve_cs(const orc_problem *p, const double *E_im, const double *g_im,
                 double *fS_re, double *fS_im, double tol, long K, long max_steps,
                 double *dbar_re, double *dbar_im, double *fbar_re, double *fbar_im,
                 long *steps, double *res)
{
    orc_init();
    long N = (long)p->nx * p->ny;
    double complex *f = (double complex *)malloc(sizeof(double complex) * 8 * N);
    double complex *db = (double complex *)malloc(sizeof(double complex) * 2 * N);
    double complex *fb = (double complex *)malloc(sizeof(double complex) * 8 * N);
    for (long k = 0; k < 8 * N; ++k) f[k] = fS_re[k] + I * fS_im[k];
    int rc = solve_c(p, E_im, g_im, f, tol, K, max_steps, db, fb, NULL, steps, res);
    for (long k = 0; k < 8 * N; ++k) { fS_re[k] = creal(f[k]); fS_im[k] = cimag(f[k]); }
    for (long k = 0; k < 2 * N; ++k) {
        if (dbar_re) dbar_re[k] = creal(db[k]);
        if (dbar_im) dbar_im[k] = cimag(db[k]);
    }
    for (long k = 0; k < 8 * N; ++k) {
        if (fbar_re) fbar_re[k] = creal(fb[k]);
        if (fbar_im) fbar_im[k] = cimag(fb[k]);
    }
    free(f); free(db); free(fb);
    return rc;
}

/*
 * Jacobian of the extended node map of node n w.r.t. its 8 input populations:
 * jac[r][p] = d out_r / d fS_p, out = (fC[0..7], h[0..7]).  The map is affine
 * in fS, so probing its linear part (zero forcing, zero wall data) with the
 * unit vectors e_p gives the exact Jacobian.
 */
static void node_jacobian(const orc_problem *p, long n, double jac[16][8])
{
    double zero2[2] = {0.0, 0.0};
    for (int pp = 0; pp < 8; ++pp) {
        double e[8] = {0}, fC[8], h[8], mbar[8];
        e[pp] = 1.0;
        node_map_r(p, n, p->E[n], e, zero2, 0, fC, h, mbar);
        for (int q = 0; q < 8; ++q) { jac[q][pp] = fC[q]; jac[8 + q][pp] = h[q]; }
    }
}

/*
 * Adjoint routing (transpose of the streaming incl. the closure slots),
 * eq. adjoint_streaming:  for node x
 *   phi_ext[q]     = phiC_q(x + c_q)  if x + c_q is in the domain, else 0
 *   phi_ext[8 + q] = phiC_q(x)        for cut links q (closure outputs), else 0
 */
static void adj_route(const orc_problem *p, long ix, long iy, const double *phiC, double out[16])
{
    long nx = p->nx, ny = p->ny, N = nx * ny, n = iy * nx + ix;
    for (int q = 0; q < 8; ++q) {
        long jx = (ix + orc_cx[q] + nx) % nx, jy = (iy + orc_cy[q] + ny) % ny;
        long m = jy * nx + jx;
        out[q] = orc_is_active(p, m) ? phiC[(long)q * N + m] : 0.0;
        out[8 + q] = (p->bc && p->bc[(long)q * N + n]) ? phiC[(long)q * N + n] : 0.0;
    }
}

/*
 * One adjoint iteration, eq. adjoint_iteration:
 *   phi^S = S^T phi^C (routing above),  phi^C_new(x) = jac_x^T phi^S_ext(x) - src(x).
 * src = (dJ/df^S)^T (8N).  dphi (2N, optional): adjoint displacement of the
 * input, (sum_q c_q phi^S_q) over the routed regular slots (reading C18).
 * phi_ext (16N, optional): the routed adjoint of the input.
 */
int orc_adj_step(const orc_problem *p, const double *phiC, double *phiCn, const double *src,
                 double *dphi, double *phi_ext)
{
    orc_init();
    long nx = p->nx, ny = p->ny, N = nx * ny;
    double jac[16][8];
    int have_bulk = 0;
    double jac_bulk[16][8];
    int uniformE = 1;
    for (long n = 1; n < N; ++n)
        if (p->E[n] != p->E[0]) { uniformE = 0; break; }
    for (long iy = 0; iy < ny; ++iy)
        for (long ix = 0; ix < nx; ++ix) {
            long n = iy * nx + ix;
            double ph[16];
            adj_route(p, ix, iy, phiC, ph);
            if (dphi) {
                double ax = 0.0, ay = 0.0;
                for (int q = 0; q < 8; ++q) { ax += orc_cx[q] * ph[q]; ay += orc_cy[q] * ph[q]; }
                dphi[n] = orc_is_active(p, n) ? ax : 0.0;
                dphi[N + n] = orc_is_active(p, n) ? ay : 0.0;
            }
            if (phi_ext)
                for (int r = 0; r < 16; ++r) phi_ext[(long)r * N + n] = orc_is_active(p, n) ? ph[r] : 0.0;
            if (!orc_is_active(p, n)) {
                for (int q = 0; q < 8; ++q) phiCn[(long)q * N + n] = 0.0;
                continue;
            }
            double (*J)[8] = jac;
            if (uniformE && !orc_is_boundary(p, n)) {
                if (!have_bulk) { node_jacobian(p, n, jac_bulk); have_bulk = 1; }
                J = jac_bulk;
            } else {
                node_jacobian(p, n, jac);
            }
            for (int pp = 0; pp < 8; ++pp) {
                double s = 0.0;
                for (int r = 0; r < 16; ++r) s += J[r][pp] * ph[r];
                phiCn[(long)pp * N + n] = s - src[(long)pp * N + n];
            }
        }
    return 0;
}

/*
 * Adjoint solve from phiC (in/out; eq. adjoint_init: zeros for a cold start),
 * stopping rule as the primal on the adjoint displacement, then the two-step
 * average of the routed adjoint phi_ext (16N).  Returns 0/1 like orc_solve.
 */
int orc_adj_solve(const orc_problem *p, double *phiC, const double *src, double tol, long K,
                  long max_steps, double *phi_ext_bar, long *steps, double *res)
{
    orc_init();
    long N = (long)p->nx * p->ny;
    double *tmp = (double *)malloc(sizeof(double) * 8 * N);
    double *dprev = (double *)malloc(sizeof(double) * 2 * N);
    double *dnow = (double *)malloc(sizeof(double) * 2 * N);
    double *e0 = (double *)malloc(sizeof(double) * 16 * N);
    double *e1 = (double *)malloc(sizeof(double) * 16 * N);
    long t = 0;
    double r = INFINITY;
    int converged = 0;
    if (K < 1) K = 1;
    orc_adj_step(p, phiC, tmp, src, dprev, NULL);
    for (;;) {
        if (tol > 0.0 && t > 0 && t % K == 0) {
            orc_adj_step(p, phiC, tmp, src, dnow, NULL);
            double num = 0.0, den = 0.0;
            for (long k = 0; k < 2 * N; ++k) {
                num += (dnow[k] - dprev[k]) * (dnow[k] - dprev[k]);
                den += dnow[k] * dnow[k];
            }
            r = (den > 0.0) ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
            memcpy(dprev, dnow, sizeof(double) * 2 * N);
            if (r < tol) { converged = 1; break; }
        }
        if (t >= max_steps) break;
        orc_adj_step(p, phiC, tmp, src, NULL, NULL);
        memcpy(phiC, tmp, sizeof(double) * 8 * N);
        ++t;
    }
    orc_adj_step(p, phiC, tmp, src, NULL, e0);
    {
        double *tmp2 = (double *)malloc(sizeof(double) * 8 * N);
        orc_adj_step(p, tmp, tmp2, src, NULL, e1);
        free(tmp2);
    }
    if (phi_ext_bar)
        for (long k = 0; k < 16 * N; ++k) phi_ext_bar[k] = (e0[k] + e1[k]) / 2.0;
    if (steps) *steps = t;
    if (res) *res = r;
    free(tmp); free(dprev); free(dnow); free(e0); free(e1);
    return (tol > 0.0 && !converged) ? 1 : 0;
}

/*
 * Adjoint source (dJ/df^S)^T of the node-wise objective eq. node_J summed as in
 * eq. discrete_J: J = sum_obs 1/2 |d - d*|^2 dx^2 / Cbar with d = (m10 + gx/2,
 * m01 + gy/2), so dJ/df_q(x) = scale * (r_x M[0][q] + r_y M[1][q]),
 * scale = dx^2 / Cbar, r = d - d* on the observation set (zero elsewhere).
 */
int orc_source(const orc_problem *p, const double *r, double scale, double *src)
{
    orc_init();
    long N = (long)p->nx * p->ny;
    for (long n = 0; n < N; ++n)
        for (int q = 0; q < 8; ++q)
            src[(long)q * N + n] = scale * (r[n] * orc_M[0][q] + r[N + n] * orc_M[1][q]);
    return 0;
}

/*
 * Local part of eq. optimality: -(dC/d alpha)^T phi^S at every domain node,
 * for the two inputs through which the controls enter:
 *   dg (2N): -sum_r phi_ext[r] d out_r / d g_c   (forcing; unit-vector probes)
 *   dE (N) : -sum_r phi_ext[r] d out_r / d E     (Young's modulus; complex step
 *            at the averaged primal state fbar), only if dE != NULL.
 */
int orc_grad_local(const orc_problem *p, const double *fbar, const double *phi_ext,
                   double *dg, double *dE)
{
    orc_init();
    long N = (long)p->nx * p->ny;
    const double hcs = 1e-30;
    for (long n = 0; n < N; ++n) {
        if (dg) { dg[n] = 0.0; dg[N + n] = 0.0; }
        if (dE) dE[n] = 0.0;
        if (!orc_is_active(p, n)) continue;
        double ph[16];
        for (int r = 0; r < 16; ++r) ph[r] = phi_ext[(long)r * N + n];
        if (dg) {
            for (int c = 0; c < 2; ++c) {
                double z8[8] = {0}, gg[2] = {0.0, 0.0}, fC[8], h[8], mbar[8];
                gg[c] = 1.0;
                node_map_r(p, n, p->E[n], z8, gg, 0, fC, h, mbar);
                double s = 0.0;
                for (int q = 0; q < 8; ++q) s += ph[q] * fC[q] + ph[8 + q] * h[q];
                dg[(long)c * N + n] = -s;
            }
        }
        if (dE) {
            double complex f[8], g[2], fC[8], h[8], mbar[8];
            for (int q = 0; q < 8; ++q) f[q] = fbar[(long)q * N + n];
            g[0] = p->g[n];
            g[1] = p->g[N + n];
            node_map_c(p, n, p->E[n] + I * hcs, f, g, 1, fC, h, mbar);
            double s = 0.0;
            for (int q = 0; q < 8; ++q) s += ph[q] * cimag(fC[q]) / hcs + ph[8 + q] * cimag(h[q]) / hcs;
            dE[n] = -s;
        }
    }
    return 0;
}

/* The inverse moment matrix as computed here (for the pins in the tests). */
void orc_minv(double out[64])
{
    orc_init();
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) out[i * 8 + j] = orc_Minv[i][j];
}
