/*
 * Type-generic body of the CPU oracle.  Included twice by slbm_oracle.c:
 *   ORC_T = double          ORC_SFX = _r   (the plain FP64 oracle)
 *   ORC_T = double complex  ORC_SFX = _c   (complex-step differentiation)
 * Only the arithmetic operators + - * / are used on ORC_T values, so the
 * complex instance is the analytic continuation of the real one and
 * Im(f(x + i h)) / h is the exact derivative (complex-step method,
 * Squire & Trapp 1998) up to round-off for any tiny h.
 *
 * TEST INFRASTRUCTURE ONLY (see slbm_oracle.c).
 */

#define ORC_CAT2(a, b) a##b
#define ORC_CAT(a, b) ORC_CAT2(a, b)
#define ORC_FN(name) ORC_CAT(name, ORC_SFX)

/* Relaxation parameters of one node (Table "relaxation times", eq. relaxation,
 * eq. gamma).  mu and K are the plane-stress moduli of eq. mu / eq. K. */
typedef struct {
    ORC_T omega[8];   /* omega_beta indexed like the moment vector m */
    ORC_T gamma;      /* coefficient of m_f = m_22 + gamma m_s (0 in the bulk) */
} ORC_FN(orc_relax);

static void ORC_FN(relax_params)(ORC_T E, double nu, int boundary,
                                 ORC_FN(orc_relax) *rp)
{
    ORC_T mu = E / (2.0 * (1.0 + nu));        /* eq. mu */
    ORC_T K = E / (2.0 * (1.0 - nu));         /* eq. K  */
    ORC_T tau11 = mu / ORC_THETA;             /* tau_11 = mu / theta        */
    ORC_T taus = 2.0 * K / (1.0 + ORC_THETA); /* tau_s  = 2K / (1 + theta)  */
    ORC_T taud = 2.0 * mu / (1.0 - ORC_THETA);/* tau_d  = 2mu / (1 - theta) */
    double tau3 = ORC_TAU_F;                  /* tau_12 = tau_21 = tau_f = 1/2 */
    /* eq. relaxation: tau = 1/omega - 1/2  <=>  omega = 1 / (tau + 1/2) */
    rp->omega[0] = 0.0;                       /* first-order moments: not relaxed */
    rp->omega[1] = 0.0;
    rp->omega[2] = 1.0 / (tau11 + 0.5);
    rp->omega[3] = 1.0 / (taus + 0.5);
    rp->omega[4] = 1.0 / (taud + 0.5);
    rp->omega[5] = 1.0 / (tau3 + 0.5);
    rp->omega[6] = 1.0 / (tau3 + 0.5);
    rp->omega[7] = 1.0 / (tau3 + 0.5);
    /* eq. gamma, active only in boundary collisions */
    rp->gamma = boundary
        ? ORC_THETA * ORC_TAU_F / ((1.0 + ORC_THETA) * (taus - ORC_TAU_F))
        : 0.0;
}

/*
 * Collision of one node (eq. moments ... eq. local_collide).
 *   fS   : post-streaming populations of the node (in Q order)
 *   g    : forcing of the node, eq. forcing
 * out:
 *   fC   : post-collision populations
 *   mbar : bared moments (eq. moments_bar_1/2 and eq. bared_moments)
 */
static void ORC_FN(collide_node)(const ORC_FN(orc_relax) *rp, const ORC_T fS[8],
                                 const ORC_T g[2], ORC_T fC[8], ORC_T mbar[8])
{
    ORC_T m[8], meq[8], mc[8];
    /* m = M fS (eq. moments); with gamma != 0 the last row of M is
     * replaced by row(m_22) + gamma * row(m_s) (appendix, transformation matrices) */
    for (int b = 0; b < 8; ++b) {
        ORC_T s = 0.0;
        for (int q = 0; q < 8; ++q) s += orc_M[b][q] * fS[q];
        m[b] = s;
    }
    m[7] = m[7] + rp->gamma * m[3];
    /* bared first-order moments, eq. moments_bar_1/2 */
    ORC_T mb10 = m[0] + g[0] / 2.0;
    ORC_T mb01 = m[1] + g[1] / 2.0;
    /* equilibrium moments m_eq = N (mb10, mb01), eq. moments_eq */
    for (int b = 0; b < 8; ++b) meq[b] = orc_N[b][0] * mb10 + orc_N[b][1] * mb01;
    /* first-order moments: second half of the forcing, eq. moments_c_10/01 */
    mc[0] = mb10 + g[0] / 2.0;
    mc[1] = mb01 + g[1] / 2.0;
    /* moment-wise relaxation, eq. moments_c */
    for (int b = 2; b < 8; ++b) mc[b] = m[b] + rp->omega[b] * (meq[b] - m[b]);
    /* bared moments, eq. bared_moments */
    mbar[0] = mb10;
    mbar[1] = mb01;
    for (int b = 2; b < 8; ++b) mbar[b] = (m[b] + mc[b]) / 2.0;
    /* back to populations: m_22 = m_f - gamma m_s, then the raw inverse of M */
    ORC_T mraw[8];
    for (int b = 0; b < 8; ++b) mraw[b] = mc[b];
    mraw[7] = mc[7] - rp->gamma * mc[3];
    for (int q = 0; q < 8; ++q) {
        ORC_T s = 0.0;
        for (int b = 0; b < 8; ++b) s += orc_Minv[q][b] * mraw[b];
        fC[q] = s;
    }
}

/* Cauchy stress (lattice units) from the bared moments, eq. stress_from_moments:
 * sigma = -[[m20, m11], [m11, m02]] with m20 = (ms + md)/2, m02 = (ms - md)/2.
 * out: (sxx, syy, sxy) */
static void ORC_FN(stress_from_mbar)(const ORC_T mbar[8], ORC_T s[3])
{
    s[0] = -(mbar[3] + mbar[4]) / 2.0;
    s[1] = -(mbar[3] - mbar[4]) / 2.0;
    s[2] = -mbar[2];
}

/*
 * Boundary closure of one cut link (reading C13, see the oracle header):
 * node x is in the domain, x - c_q is not, so f^S_q(x, t+1) has no source.
 *  Dirichlet: h = f^C_qbar(x) + 2 feq_q(d_D)      (odd part reflected about d_D)
 *  Neumann  : h = -f^C_qbar(x) + 2 fsig_q(sigma_w) (even part reflected about sigma_w)
 * feq(d) = Minv N d; fsig(sigma) = Minv * (0,0,-sxy,-(sxx+syy),-(sxx-syy),0,0,0);
 * sigma_w is the node's bared stress with its normal traction replaced by T:
 *   a = T - sigma_b n,  sigma_w = sigma_b + a n^T + n a^T - (a.n) n n^T.
 */
static ORC_T ORC_FN(closure_link)(int q, int kind, const ORC_T fC[8], const ORC_T mbar[8],
                                  const ORC_T wall[2], const double nrm[2])
{
    int qb = orc_opp[q];
    if (kind == ORC_BC_DIRICHLET) {
        ORC_T feq = 0.0;
        for (int b = 0; b < 8; ++b)
            feq += orc_Minv[q][b] * (orc_N[b][0] * wall[0] + orc_N[b][1] * wall[1]);
        return fC[qb] + 2.0 * feq;
    } else {
        ORC_T sb[3];
        ORC_FN(stress_from_mbar)(mbar, sb);
        double nx = nrm[0], ny = nrm[1];
        ORC_T ax = wall[0] - (sb[0] * nx + sb[2] * ny);
        ORC_T ay = wall[1] - (sb[2] * nx + sb[1] * ny);
        ORC_T an = ax * nx + ay * ny;
        ORC_T wxx = sb[0] + 2.0 * ax * nx - an * nx * nx;
        ORC_T wyy = sb[1] + 2.0 * ay * ny - an * ny * ny;
        ORC_T wxy = sb[2] + ax * ny + ay * nx - an * nx * ny;
        ORC_T msig[8] = {0.0, 0.0, -wxy, -(wxx + wyy), -(wxx - wyy), 0.0, 0.0, 0.0};
        ORC_T fsig = 0.0;
        for (int b = 0; b < 8; ++b) fsig += orc_Minv[q][b] * msig[b];
        return -fC[qb] + 2.0 * fsig;
    }
}

/*
 * Extended node map: the collision outputs fC[0..7] (streamed to x + c_q) and
 * the closure outputs h[0..7] (written to f^S_q(x) for cut links, 0 otherwise).
 */
static void ORC_FN(node_map)(const orc_problem *p, long n, ORC_T E, const ORC_T fS[8],
                             const ORC_T g[2], int with_walls, ORC_T fC[8], ORC_T h[8],
                             ORC_T mbar[8])
{
    long N = (long)p->nx * p->ny;
    int boundary = orc_is_boundary(p, n);
    ORC_FN(orc_relax) rp;
    ORC_FN(relax_params)(E, p->nu, boundary && p->gamma_at_boundary, &rp);
    ORC_FN(collide_node)(&rp, fS, g, fC, mbar);
    for (int q = 0; q < 8; ++q) {
        h[q] = 0.0;
        int kind = p->bc ? p->bc[(long)q * N + n] : 0;
        if (!kind) continue;
        ORC_T wall[2] = {0.0, 0.0};
        double nrm[2] = {0.0, 0.0};
        if (with_walls && p->wall) {
            wall[0] = p->wall[(0L * 8 + q) * N + n];
            wall[1] = p->wall[(1L * 8 + q) * N + n];
        }
        if (p->normal) {
            nrm[0] = p->normal[(0L * 8 + q) * N + n];
            nrm[1] = p->normal[(1L * 8 + q) * N + n];
        }
        h[q] = ORC_FN(closure_link)(q, kind, fC, mbar, wall, nrm);
    }
}

/*
 * One primal time step (eq. local_collide then eq. local_stream):
 *   f^C(x) = C_x[f^S(x)],  f^S(x + c_q, t+1) = f^C_q(x)   (periodic index wrap),
 * cut links take the closure value.  Nodes outside the domain carry zeros.
 * Eg / gg: imaginary parts of E and g for the complex instance (NULL = 0).
 * disp (2N) / stress (3N), if given, receive the bared displacement
 * (eq. disp_from_moments) and stress of the INPUT state.
 */
static void ORC_FN(step)(const orc_problem *p, const double *E_im, const double *g_im,
                         const ORC_T *fS, ORC_T *fSn, ORC_T *disp, ORC_T *stress)
{
    long nx = p->nx, ny = p->ny, N = nx * ny;
    for (long k = 0; k < 8 * N; ++k) fSn[k] = 0.0;
    for (long iy = 0; iy < ny; ++iy)
        for (long ix = 0; ix < nx; ++ix) {
            long n = iy * nx + ix;
            if (!orc_is_active(p, n)) {
                if (disp) { disp[n] = 0.0; disp[N + n] = 0.0; }
                if (stress) { stress[n] = 0.0; stress[N + n] = 0.0; stress[2 * N + n] = 0.0; }
                continue;
            }
            ORC_T f[8], fC[8], h[8], mbar[8], g[2];
            for (int q = 0; q < 8; ++q) f[q] = fS[(long)q * N + n];
            g[0] = p->g[n];
            g[1] = p->g[N + n];
            ORC_T E = p->E[n];
#ifdef ORC_IS_COMPLEX
            if (g_im) { g[0] += I * g_im[n]; g[1] += I * g_im[N + n]; }
            if (E_im) E += I * E_im[n];
#else
            (void)E_im; (void)g_im;
#endif
            ORC_FN(node_map)(p, n, E, f, g, 1, fC, h, mbar);
            if (disp) { disp[n] = mbar[0]; disp[N + n] = mbar[1]; }
            if (stress) {
                ORC_T s[3];
                ORC_FN(stress_from_mbar)(mbar, s);
                stress[n] = s[0]; stress[N + n] = s[1]; stress[2 * N + n] = s[2];
            }
            for (int q = 0; q < 8; ++q) {
                long jx = (ix + orc_cx[q] + nx) % nx, jy = (iy + orc_cy[q] + ny) % ny;
                long m = jy * nx + jx;
                if (orc_is_active(p, m)) fSn[(long)q * N + m] = fC[q];
            }
            if (p->bc)
                for (int q = 0; q < 8; ++q)
                    if (p->bc[(long)q * N + n]) fSn[(long)q * N + n] = h[q];
        }
}

/* Displacement of a state (bared first moments of every node, eq. disp_from_moments). */
static void ORC_FN(disp_of)(const orc_problem *p, const double *g_im, const ORC_T *fS, ORC_T *disp)
{
    long N = (long)p->nx * p->ny;
    for (long n = 0; n < N; ++n) {
        if (!orc_is_active(p, n)) { disp[n] = 0.0; disp[N + n] = 0.0; continue; }
        ORC_T m10 = 0.0, m01 = 0.0;
        for (int q = 0; q < 8; ++q) {
            m10 += orc_M[0][q] * fS[(long)q * N + n];
            m01 += orc_M[1][q] * fS[(long)q * N + n];
        }
        ORC_T gx = p->g[n], gy = p->g[N + n];
#ifdef ORC_IS_COMPLEX
        if (g_im) { gx += I * g_im[n]; gy += I * g_im[N + n]; }
#else
        (void)g_im;
#endif
        disp[n] = m10 + gx / 2.0;
        disp[N + n] = m01 + gy / 2.0;
    }
}

/*
 * Pseudo-time march to steady state (section "Gradient-based optimization
 * algorithm" with reading C6/C7 for the stopping rule):
 *   every K steps r = ||d(t) - d(t-K)||_2 / ||d(t)||_2 over the domain nodes
 *   (real parts), stop when r < tol or t >= max_steps; then one more step and
 *   the two-step average  d = (d(t) + d(t+1))/2,  f = (f^S(t) + f^S(t+1))/2.
 * tol <= 0 runs exactly max_steps steps (fixed-step mode, no averaging is
 * skipped: the average is still formed).
 * Returns 0 if converged, 1 if max_steps was hit.
 */
static int ORC_FN(solve)(const orc_problem *p, const double *E_im, const double *g_im,
                         ORC_T *fS, double tol, long K, long max_steps,
                         ORC_T *dbar, ORC_T *fbar, ORC_T *sbar,
                         long *steps_out, double *res_out)
{
    long N = (long)p->nx * p->ny;
    ORC_T *tmp = (ORC_T *)malloc(sizeof(ORC_T) * 8 * N);
    ORC_T *dprev = (ORC_T *)malloc(sizeof(ORC_T) * 2 * N);
    ORC_T *dnow = (ORC_T *)malloc(sizeof(ORC_T) * 2 * N);
    ORC_T *s0 = (ORC_T *)malloc(sizeof(ORC_T) * 3 * N);
    ORC_T *s1 = (ORC_T *)malloc(sizeof(ORC_T) * 3 * N);
    ORC_T *d1 = (ORC_T *)malloc(sizeof(ORC_T) * 2 * N);
    long t = 0;
    double res = INFINITY;
    int converged = 0;
    if (K < 1) K = 1;
    ORC_FN(disp_of)(p, g_im, fS, dprev);
    for (;;) {
        if (tol > 0.0 && t > 0 && t % K == 0) {
            ORC_FN(disp_of)(p, g_im, fS, dnow);
            double num = 0.0, den = 0.0;
            for (long k = 0; k < 2 * N; ++k) {
                double a = orc_re(dnow[k]), b = orc_re(dprev[k]);
                num += (a - b) * (a - b);
                den += a * a;
            }
            res = (den > 0.0) ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
            for (long k = 0; k < 2 * N; ++k) dprev[k] = dnow[k];
            if (res < tol) { converged = 1; break; }
        }
        if (t >= max_steps) break;
        ORC_FN(step)(p, E_im, g_im, fS, tmp, NULL, NULL);
        for (long k = 0; k < 8 * N; ++k) fS[k] = tmp[k];
        ++t;
    }
    /* two-step average (reading C7): the state at t and at t+1 */
    ORC_FN(step)(p, E_im, g_im, fS, tmp, dnow, s0);
    ORC_FN(disp_of)(p, g_im, tmp, d1);
    {
        ORC_T *tmp2 = (ORC_T *)malloc(sizeof(ORC_T) * 8 * N);
        ORC_FN(step)(p, E_im, g_im, tmp, tmp2, NULL, s1);
        free(tmp2);
    }
    if (dbar) for (long k = 0; k < 2 * N; ++k) dbar[k] = (dnow[k] + d1[k]) / 2.0;
    if (sbar) for (long k = 0; k < 3 * N; ++k) sbar[k] = (s0[k] + s1[k]) / 2.0;
    if (fbar) for (long k = 0; k < 8 * N; ++k) fbar[k] = (fS[k] + tmp[k]) / 2.0;
    if (steps_out) *steps_out = t;
    if (res_out) *res_out = res;
    free(tmp); free(dprev); free(dnow); free(s0); free(s1); free(d1);
    return (tol > 0.0 && !converged) ? 1 : 0;
}
