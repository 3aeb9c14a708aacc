"""Python side of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Thin ctypes wrapper around liboracle.so plus the plain-numpy glue that the
paper states in closed form: the objective (eq. node_J, eq. discrete_J), its
normalisation, the chain rule from the local optimality pieces to each control
kind (eq. optimality, eq. zero_mean_projection, eq. E_substitution), the
complex-step forward-mode gradient (eq. fAD), central finite differences, and
the paper's coefficient-of-variation convergence test (eq. convergence, eq.
convergence_crit) as an alternative stopping rule of the primal and adjoint
solves.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It does not import the HIP package and the HIP package never
imports it.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

NONE, DIRICHLET, NEUMANN = 0, 1, 2
CX = np.array([1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 1, 0, -1, 1, 1, -1, -1])


def _lib():
    global _LIB
    if _LIB is None:
        path = os.environ.get("SLBM_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        _LIB = ctypes.CDLL(path)
        _setup(_LIB)
    return _LIB


class _CProblem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("dx", ctypes.c_double), ("nu", ctypes.c_double),
        ("E", ctypes.c_void_p), ("active", ctypes.c_void_p), ("bc", ctypes.c_void_p),
        ("wall", ctypes.c_void_p), ("normal", ctypes.c_void_p), ("g", ctypes.c_void_p),
        ("gamma_at_boundary", ctypes.c_int),
    ]


_P = ctypes.c_void_p
_L = ctypes.c_long
_D = ctypes.c_double


def _setup(lib):
    pp = ctypes.POINTER(_CProblem)
    lib.orc_step.argtypes = [pp, _P, _P, _P, _P]
    lib.orc_run.argtypes = [pp, _P, _L]
    lib.orc_solve.argtypes = [pp, _P, _D, _L, _L, _P, _P, _P, _P, _P]
    lib.orc_solve_cs.argtypes = [pp, _P, _P, _P, _P, _D, _L, _L, _P, _P, _P, _P, _P, _P]
    lib.orc_adj_step.argtypes = [pp, _P, _P, _P, _P, _P]
    lib.orc_adj_solve.argtypes = [pp, _P, _P, _D, _L, _L, _P, _P, _P]
    lib.orc_source.argtypes = [pp, _P, _D, _P]
    lib.orc_grad_local.argtypes = [pp, _P, _P, _P, _P]
    lib.orc_minv.argtypes = [_P]
    for f in ("orc_step", "orc_run", "orc_solve", "orc_solve_cs", "orc_adj_step", "orc_adj_solve",
              "orc_source", "orc_grad_local"):
        getattr(lib, f).restype = ctypes.c_int


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Problem:
    """A lattice problem for the oracle.

    nx, ny   grid (x fastest);  dx spacing (dt = dx^2, kappa = 1)
    E        scalar or (ny, nx) Young's modulus;  nu Poisson ratio
    g        (2, ny, nx) forcing in lattice units (g = dx^2 F)
    active   (ny, nx) bool/uint8 domain mask (None = periodic torus, all nodes)
    bc       (8, ny, nx) uint8 link kinds (incoming population f_q at x whose
             source x - c_q lies outside): 0, DIRICHLET, NEUMANN
    wall     (2, 8, ny, nx) wall data per link: d_D (Dirichlet) or T in lattice
             units (Neumann)
    normal   (2, 8, ny, nx) outward unit normal per Neumann link
    """

    def __init__(self, nx, ny, dx, E, nu, g, active=None, bc=None, wall=None, normal=None,
                 gamma_at_boundary=True):
        self.nx, self.ny, self.dx, self.nu = int(nx), int(ny), float(dx), float(nu)
        N = self.nx * self.ny
        self.E = _f64(np.broadcast_to(np.asarray(E, dtype=np.float64), (self.ny, self.nx)))
        self.g = _f64(g).reshape(2, self.ny, self.nx)
        self.active = None if active is None else np.ascontiguousarray(active, dtype=np.uint8).reshape(self.ny, self.nx)
        self.bc = None if bc is None else np.ascontiguousarray(bc, dtype=np.uint8).reshape(8, self.ny, self.nx)
        self.wall = None if wall is None else _f64(wall).reshape(2, 8, self.ny, self.nx)
        self.normal = None if normal is None else _f64(normal).reshape(2, 8, self.ny, self.nx)
        self.gamma_at_boundary = bool(gamma_at_boundary)
        self.N = N
        self._c = _CProblem(self.nx, self.ny, self.dx, self.nu, _ptr(self.E), _ptr(self.active),
                            _ptr(self.bc), _ptr(self.wall), _ptr(self.normal), _ptr(self.g),
                            int(self.gamma_at_boundary))

    def with_(self, **kw):
        args = dict(nx=self.nx, ny=self.ny, dx=self.dx, E=self.E, nu=self.nu, g=self.g,
                    active=self.active, bc=self.bc, wall=self.wall, normal=self.normal,
                    gamma_at_boundary=self.gamma_at_boundary)
        args.update(kw)
        return Problem(**args)

    @property
    def mask(self):
        if self.active is None:
            return np.ones((self.ny, self.nx), dtype=bool)
        return self.active.astype(bool)

    def zeros(self, comps=8, dtype=np.float64):
        return np.zeros((comps, self.ny, self.nx), dtype=dtype)

    def cref(self):
        return ctypes.byref(self._c)


# ----------------------------------------------------------------- primal

def step(p, fS):
    """One primal step (eq. local_collide, then eq. local_stream); returns
    (fS(t+1), d(t), sigma(t) in lattice units)."""
    fS = _f64(fS)
    out, d, s = p.zeros(8), p.zeros(2), p.zeros(3)
    _lib().orc_step(p.cref(), _ptr(fS), _ptr(out), _ptr(d), _ptr(s))
    return out, d, s


def run(p, fS, nsteps):
    """nsteps steps of the primal (collision eq. local_collide, then streaming
    eq. local_stream) from the post-streaming populations fS; returns f^S."""
    f = _f64(fS).copy()
    _lib().orc_run(p.cref(), _ptr(f), int(nsteps))
    return f


def check_interval(dx):
    """K = 2 ceil(0.005 / dx^2): pseudo-time window 0.01 (reading C6)."""
    return 2 * int(np.ceil(0.005 / (dx * dx) - 1e-9))


class Solve:
    """Result record of a primal or adjoint solve (fields set by the solver)."""


def solve(p, fS0=None, tol=1e-10, K=None, max_steps=10_000_000):
    """Steady state (reading C6/C7); tol <= 0 means exactly max_steps steps."""
    f = p.zeros(8) if fS0 is None else _f64(fS0).copy()
    K = check_interval(p.dx) if K is None else int(K)
    dbar, fbar, sbar = p.zeros(2), p.zeros(8), p.zeros(3)
    steps, res = ctypes.c_long(0), ctypes.c_double(0)
    rc = _lib().orc_solve(p.cref(), _ptr(f), float(tol), K, int(max_steps), _ptr(dbar), _ptr(fbar),
                          _ptr(sbar), ctypes.byref(steps), ctypes.byref(res))
    s = Solve()
    s.rc, s.f, s.dbar, s.fbar, s.sbar = rc, f, dbar, fbar, sbar
    s.steps, s.residual, s.K = steps.value, res.value, K
    return s


def solve_cs(p, E_im=None, g_im=None, tol=1e-10, K=None, max_steps=10_000_000):
    """Complex-step primal solve, the forward mode of eq. fAD: returns (dbar,
    dbar_im) for inputs E + i E_im, g + i g_im."""
    fr, fi = p.zeros(8), p.zeros(8)
    K = check_interval(p.dx) if K is None else int(K)
    E_im = None if E_im is None else _f64(np.broadcast_to(E_im, (p.ny, p.nx)))
    g_im = None if g_im is None else _f64(g_im).reshape(2, p.ny, p.nx)
    dr, di = p.zeros(2), p.zeros(2)
    steps, res = ctypes.c_long(0), ctypes.c_double(0)
    rc = _lib().orc_solve_cs(p.cref(), _ptr(E_im), _ptr(g_im), _ptr(fr), _ptr(fi), float(tol), K,
                             int(max_steps), _ptr(dr), _ptr(di), None, None, ctypes.byref(steps),
                             ctypes.byref(res))
    return dr, di, rc, steps.value


# ----------------------------------------------------------------- objective

def cbar(p, target, obs=None):
    """Normalisation constant of eq. node_J: sum_obs |d*|^2 dx^2."""
    m = p.mask if obs is None else (np.asarray(obs, bool) & p.mask)
    return float(((target ** 2).sum(0) * m).sum() * p.dx * p.dx)


def objective(p, d, target, obs=None, normalize=True):
    """eq. discrete_J: sum_obs 1/2 |d - d*|^2 dx^2 / Cbar."""
    m = p.mask if obs is None else (np.asarray(obs, bool) & p.mask)
    c = cbar(p, target, obs) if normalize else 1.0
    r = (d - target) * m
    return 0.5 * float((r ** 2).sum()) * p.dx * p.dx / c


# ----------------------------------------------------------------- adjoint

def source(p, r, scale):
    """Adjoint source (dJ/df^S)^T of eq. discrete_J: scale * (r_x M[0][q] +
    r_y M[1][q]) per node and direction, r = d - d* on the observation set
    (d from the first moments, eq. disp_from_moments), scale = dx^2 / Cbar."""
    src = p.zeros(8)
    _lib().orc_source(p.cref(), _ptr(_f64(r)), float(scale), _ptr(src))
    return src


def adj_step(p, phiC, src):
    """One adjoint iteration (eq. adjoint_iteration): transposed streaming
    (eq. adjoint_streaming), then the transposed node Jacobian minus the
    source (eq. adjoint_collision).  Returns (phi^C, adjoint displacement of
    the input (reading C18), routed adjoint of the input)."""
    out, dphi, ext = p.zeros(8), p.zeros(2), p.zeros(16)
    _lib().orc_adj_step(p.cref(), _ptr(_f64(phiC)), _ptr(out), _ptr(_f64(src)), _ptr(dphi), _ptr(ext))
    return out, dphi, ext


def adj_solve(p, src, tol=1e-10, K=None, max_steps=10_000_000, phiC0=None):
    """Adjoint fixed point from phi^C = 0 (eq. adjoint_init) with the primal's
    stopping rule on the adjoint displacement, then the two-step average of the
    routed adjoint (readings C6, C7, C18)."""
    phiC = p.zeros(8) if phiC0 is None else _f64(phiC0).copy()
    K = check_interval(p.dx) if K is None else int(K)
    ext = p.zeros(16)
    steps, res = ctypes.c_long(0), ctypes.c_double(0)
    rc = _lib().orc_adj_solve(p.cref(), _ptr(phiC), _ptr(_f64(src)), float(tol), K, int(max_steps),
                              _ptr(ext), ctypes.byref(steps), ctypes.byref(res))
    s = Solve()
    s.rc, s.phiC, s.ext, s.steps, s.residual = rc, phiC, ext, steps.value, res.value
    return s


def grad_local(p, fbar, ext, want_E=False):
    """Local part of eq. optimality at every domain node: minus the transposed
    derivative of the node map with respect to the forcing (and, if want_E,
    to Young's modulus, by complex step at the averaged state fbar), applied to
    the averaged routed adjoint `ext`."""
    dg = p.zeros(2)
    dE = p.zeros(1)[0] if want_E else None
    _lib().orc_grad_local(p.cref(), _ptr(_f64(fbar)), _ptr(_f64(ext)), _ptr(dg), _ptr(dE))
    return dg, dE


def zero_mean(a, mask=None):
    """eq. zero_mean_projection, per component."""
    a = np.array(a, dtype=np.float64)
    if mask is None:
        return a - a.reshape(a.shape[0], -1).mean(1)[:, None, None]
    m = np.asarray(mask, bool)
    out = a.copy()
    for c in range(a.shape[0]):
        out[c][m] -= a[c][m].mean()
    return out


class Gradient:
    """Result record of objective_and_grad: J, grad, and the primal / adjoint solves."""


# ------------------------------------------------- the paper's convergence test

def cv_of(window_c):
    """eq. convergence_crit: std(c) / mean(c) of the samples (population
    standard deviation; a window of zeros counts as converged)."""
    w = np.asarray(window_c, dtype=np.float64)
    m = w.mean()
    if m <= 0.0:
        return 0.0
    return float(np.sqrt(((w - m) ** 2).mean()) / m)


def solve_cv(p, tol, window=10, K=None, max_steps=10_000_000):
    """Steady state by the paper's test (Sec. "Gradient-based optimization
    algorithm", eq. convergence, eq. convergence_crit): c(t) = mean over the
    domain nodes of |d(t)|^2, sampled every K steps (the K-lag check spacing,
    reading C6); stop at the first check at which the coefficient of variation
    of the last `window` samples is below tol; then the two-step average
    (reading C7).  The 1/N of the mean cancels in the ratio and is left out."""
    K = check_interval(p.dx) if K is None else int(K)
    m = p.mask
    f = p.zeros(8)
    t, cs, cv, converged = 0, [], np.inf, False
    while True:
        if t > 0:
            fn, d, _ = step(p, f)
            cs.append(float(((d ** 2) * m).sum()))
            if len(cs) >= window:
                cv = cv_of(cs[-window:])
                if cv < tol:
                    converged = True
                    break
            if t >= max_steps:
                break
            f = run(p, fn, K - 1)
        else:
            f = run(p, f, K)
        t += K
    f1, d0, _ = step(p, f)
    d1 = step(p, f1)[1]
    s = Solve()
    s.rc = 0 if converged else 1
    s.fS, s.steps, s.residual = f, t, cv
    s.dbar, s.fbar = (d0 + d1) / 2.0, (f + f1) / 2.0
    return s


def adj_solve_cv(p, src, tol, window=10, K=None, max_steps=10_000_000):
    """Adjoint solve from zero with the same test on the adjoint displacement
    (reading C18), then the two-step average of the routed adjoint."""
    K = check_interval(p.dx) if K is None else int(K)
    m = p.mask
    ph = p.zeros(8)
    t, cs, cv, converged = 0, [], np.inf, False
    while True:
        if t > 0 and t % K == 0:
            dphi = adj_step(p, ph, src)[1]
            cs.append(float(((dphi ** 2) * m).sum()))
            if len(cs) >= window:
                cv = cv_of(cs[-window:])
                if cv < tol:
                    converged = True
                    break
        if t >= max_steps:
            break
        ph = adj_step(p, ph, src)[0]
        t += 1
    ph1, _, e0 = adj_step(p, ph, src)
    e1 = adj_step(p, ph1, src)[2]
    s = Solve()
    s.rc = 0 if converged else 1
    s.phiC, s.ext, s.steps, s.residual = ph, (e0 + e1) / 2.0, t, cv
    return s


def objective_and_grad(p, target, kind, control, modes=None, fixed_force=None, obs=None,
                       normalize=True, tol=1e-10, K=None, max_steps=10_000_000, project=None,
                       cv_window=0):
    """Primal solve, J, adjoint solve and eq. optimality for one control kind.

    kind: 'modes'  (F = sum_i a_i B_i, control a (k,), modes (k, 2, ny, nx))
          'nodal'  (F = P(alpha), control (2, ny, nx))
          'E_nodal' (E = control (ny, nx), forcing dx^2 * fixed_force)
          'E_sq'   (E = alpha^2, control (1,))
    project: zero-mean projection of nodal force control and gradient
             (default: on for 'nodal' on periodic problems).
    cv_window: > 0 solves with the paper's coefficient-of-variation test over
             that many checks (solve_cv / adj_solve_cv), else the K-lag residual.
    """
    dx2 = p.dx * p.dx
    if kind == "modes":
        a = np.asarray(control, dtype=np.float64)
        F = np.tensordot(a, modes, 1)
        q = p.with_(g=dx2 * F)
    elif kind == "nodal":
        if project is None:
            project = p.active is None
        F = zero_mean(control) if project else np.asarray(control, dtype=np.float64)
        q = p.with_(g=dx2 * F)
    elif kind == "E_nodal":
        q = p.with_(E=np.asarray(control, dtype=np.float64), g=dx2 * fixed_force)
    elif kind == "E_sq":
        a = float(np.asarray(control).reshape(-1)[0])
        q = p.with_(E=a * a, g=dx2 * fixed_force)
    else:
        raise ValueError(kind)
    if cv_window > 0:
        prim = solve_cv(q, tol, window=cv_window, K=K, max_steps=max_steps)
    else:
        prim = solve(q, tol=tol, K=K, max_steps=max_steps)
    m = q.mask if obs is None else (np.asarray(obs, bool) & q.mask)
    c = cbar(q, target, obs) if normalize else 1.0
    r = (prim.dbar - target) * m
    J = 0.5 * float((r ** 2).sum()) * dx2 / c
    if q.active is None:
        # periodic (reading C21): d has zero mean (the translations are the
        # kernel of the torus problem, Sec. "Problem formulation"), so the mean
        # of r does not depend on the control; the source takes the zero-mean
        # part of r, the compatibility condition that eq. zero_mean_projection
        # states for the control.  With the mean kept the source excites the
        # adjoint's translation mode (eigenvalue 1) and there is no fixed point.
        r = zero_mean(r)
    src = source(q, r, dx2 / c)
    if cv_window > 0:
        adj = adj_solve_cv(q, src, tol, window=cv_window, K=K, max_steps=max_steps)
    else:
        adj = adj_solve(q, src, tol=tol, K=K, max_steps=max_steps)
    dg_adj, dE = grad_local(q, prim.fbar, adj.ext, want_E=kind in ("E_nodal", "E_sq"))
    # explicit dependence of d on g (half forcing): dJ/dg = r/2 * dx^2/Cbar
    dJdg = 0.5 * r * dx2 / c + dg_adj
    dJdF = dx2 * dJdg
    out = Gradient()
    out.J, out.prim, out.adj, out.r, out.cbar, out.problem = J, prim, adj, r, c, q
    if kind == "modes":
        out.grad = np.array([float((dJdF * b).sum()) for b in modes])
    elif kind == "nodal":
        out.grad = zero_mean(dJdF) if project else dJdF
    elif kind == "E_nodal":
        out.grad = dE * q.mask
    else:
        out.grad = np.array([float((dE * q.mask).sum()) * 2.0 * a])
    return out


def fad_grad_modes(p, target, control, modes, obs=None, normalize=True, tol=1e-10, K=None,
                   max_steps=10_000_000, h=1e-30):
    """Forward-mode (eq. fAD) gradient for mode controls: one complex-step primal
    per control direction; dJ/da_i = Im J(a + i h e_i) / h."""
    dx2 = p.dx * p.dx
    a = np.asarray(control, dtype=np.float64)
    q = p.with_(g=dx2 * np.tensordot(a, modes, 1))
    m = q.mask if obs is None else (np.asarray(obs, bool) & q.mask)
    c = cbar(q, target, obs) if normalize else 1.0
    out = []
    for i in range(len(a)):
        dr, di, rc, _ = solve_cs(q, g_im=h * dx2 * modes[i], tol=tol, K=K, max_steps=max_steps)
        # J(a + i h e_i) = 1/2 sum (r + i h dd)^2 dx^2 / c  ->  Im / h = sum r * dd dx^2 / c
        out.append(float((((dr - target) * di / h) * m).sum()) * dx2 / c)
    return np.array(out)


def fad_grad_E_sq(p, target, alpha, fixed_force, obs=None, normalize=True, tol=1e-10, K=None,
                  max_steps=10_000_000, h=1e-30):
    """Forward-mode gradient (eq. fAD) for the scalar control E = alpha^2
    (eq. E_substitution), by a complex-step primal solve."""
    dx2 = p.dx * p.dx
    q = p.with_(E=alpha * alpha, g=dx2 * fixed_force)
    m = q.mask if obs is None else (np.asarray(obs, bool) & q.mask)
    c = cbar(q, target, obs) if normalize else 1.0
    dr, di, rc, _ = solve_cs(q, E_im=np.full((p.ny, p.nx), 2.0 * alpha * h), tol=tol, K=K,
                             max_steps=max_steps)
    return float((((dr - target) * di / h) * m).sum()) * dx2 / c


def minv():
    """The inverse of the moment matrix M of the appendix, as the C oracle forms
    it (checked against M in the pins)."""
    out = np.zeros(64)
    _lib().orc_minv(_ptr(out))
    return out.reshape(8, 8)
