"""Gradient-based optimisation driver (Algorithm "GBO", Sec. "Gradient-based
optimization algorithm").

Each optimisation step solves the primal to steady state, evaluates J and its
gradient (ALBM on the GPU through `objective_and_grad`, or any callable with
the same contract), forms the L-BFGS descent direction (eq. control_update,
eq. descent_direction) and finds a step size satisfying the strong Wolfe
conditions by an inner line-search loop.  Termination (Algorithm "GBO"):
gradient norm below eps, or every component's relative change
|2 dalpha_i / (alpha_i^(m+1) + alpha_i^(m))| below eps_alpha, or m_max steps.

Reading of the parameters the paper leaves open: strong Wolfe with c1 = 1e-4,
c2 = 0.9 (Nocedal & Wright, Alg. 3.5/3.6 with cubic interpolation in the
zoom); the initial inverse-Hessian is gamma0 * I for the first step and the
usual s.y / y.y scaling afterwards; l = number of stored pairs.
"""
import math
import time

import numpy as np

# Table "parameter" (benchmark 1) of the paper
PAPER_BENCH1 = dict(eps=1e-10, eps_alpha=2.2e-16, lam0=1.0, m_max=50, k_max=100, memory=20, gamma0=1e-4)
# Table "distributed" (benchmark 2)
PAPER_BENCH2 = dict(eps=1e-10, eps_alpha=2.2e-16, lam0=1.0, m_max=100, k_max=100, memory=20, gamma0=1e-4)


class OptResult:
    def __init__(self):
        self.x = None
        self.J = None
        self.grad = None
        self.steps = 0
        self.evals = 0
        self.reason = ""
        self.history = []        # per step: dict(m, J, gnorm, lam, evals, x)
        self.wall_s = 0.0


def _two_loop(g, S, Y, gamma):
    """L-BFGS two-loop recursion: returns H g."""
    q = g.copy()
    alphas = []
    for s, y in zip(reversed(S), reversed(Y)):
        rho = 1.0 / float(y @ s)
        a = rho * float(s @ q)
        alphas.append((a, rho, s, y))
        q -= a * y
    r = gamma * q
    for a, rho, s, y in reversed(alphas):
        b = rho * float(y @ r)
        r += (a - b) * s
    return r


def _cubic_min(a, fa, ga, b, fb, gb):
    """Minimiser of the cubic through (a, fa, ga), (b, fb, gb), or None."""
    d1 = ga + gb - 3.0 * (fa - fb) / (a - b)
    disc = d1 * d1 - ga * gb
    if disc < 0:
        return None
    d2 = math.copysign(math.sqrt(disc), b - a)
    den = gb - ga + 2.0 * d2
    if den == 0:
        return None
    return b - (b - a) * (gb + d2 - d1) / den


def strong_wolfe(phi, phi0, dphi0, lam0=1.0, c1=1e-4, c2=0.9, k_max=100, lam_max=1e20):
    """Step size satisfying the strong Wolfe conditions (Nocedal & Wright,
    Alg. 3.5 / 3.6).  phi(lam) -> (value, derivative, payload).  Returns
    (lam, payload, evaluations, best) where lam is None if k_max evaluations
    did not find one; best = (value, payload) of the lowest value seen."""
    state = {"evals": 0, "best": None}

    def ev(lam):
        f, g, pay = phi(lam)
        state["evals"] += 1
        if state["best"] is None or f < state["best"][0]:
            state["best"] = (f, pay)
        return f, g, pay

    def zoom(lo, flo, glo, hi, fhi, ghi):
        while state["evals"] < k_max:
            lj = _cubic_min(lo, flo, glo, hi, fhi, ghi)
            lmin, lmax = min(lo, hi), max(lo, hi)
            if lj is None or not (lmin + 0.1 * (lmax - lmin) <= lj <= lmax - 0.1 * (lmax - lmin)):
                lj = 0.5 * (lo + hi)
            fj, gj, pj = ev(lj)
            if fj > phi0 + c1 * lj * dphi0 or fj >= flo:
                hi, fhi, ghi = lj, fj, gj
            else:
                if abs(gj) <= -c2 * dphi0:
                    return lj, pj
                if gj * (hi - lo) >= 0:
                    hi, fhi, ghi = lo, flo, glo
                lo, flo, glo = lj, fj, gj
        return None, None

    lam_prev, f_prev, g_prev = 0.0, phi0, dphi0
    lam = lam0
    while state["evals"] < k_max:
        f, g, pay = ev(lam)
        if f > phi0 + c1 * lam * dphi0 or (state["evals"] > 1 and f >= f_prev):
            lam_w, pay_w = zoom(lam_prev, f_prev, g_prev, lam, f, g)
            return lam_w, pay_w, state["evals"], state["best"]
        if abs(g) <= -c2 * dphi0:
            return lam, pay, state["evals"], state["best"]
        if g >= 0:
            lam_w, pay_w = zoom(lam, f, g, lam_prev, f_prev, g_prev)
            return lam_w, pay_w, state["evals"], state["best"]
        lam_prev, f_prev, g_prev = lam, f, g
        lam = min(2.0 * lam, lam_max)
    return None, None, state["evals"], state["best"]


def lbfgs(fun, x0, eps=1e-10, eps_alpha=2.2e-16, lam0=1.0, m_max=50, k_max=100, memory=20, gamma0=1e-4,
          c1=1e-4, c2=0.9, callback=None):
    """Algorithm GBO with L-BFGS.  fun(x) -> (J, grad) with grad shaped like x.
    Returns an OptResult."""
    t0 = time.perf_counter()
    res = OptResult()
    shape = np.shape(x0)
    x = np.asarray(x0, dtype=np.float64).ravel().copy()
    J, g = fun(x.reshape(shape))
    g = np.asarray(g, dtype=np.float64).ravel()
    res.evals = 1
    S, Y = [], []
    gamma = gamma0
    res.history.append(dict(m=0, J=J, gnorm=float(np.linalg.norm(g)), lam=0.0, evals=1, x=x.copy()))
    reason = "m_max"
    for m in range(m_max):
        if np.linalg.norm(g) < eps:
            reason = "gradient"
            break
        p = -_two_loop(g, S, Y, gamma)
        dphi0 = float(g @ p)
        if dphi0 >= 0:                       # not a descent direction: restart from steepest descent
            S, Y = [], []
            p = -gamma0 * g
            dphi0 = float(g @ p)

        def phi(lam):
            xt = x + lam * p
            Jt, gt = fun(xt.reshape(shape))
            gt = np.asarray(gt, dtype=np.float64).ravel()
            return Jt, float(gt @ p), (xt, Jt, gt)

        lam, pay, nev, best = strong_wolfe(phi, J, dphi0, lam0=lam0, c1=c1, c2=c2, k_max=k_max)
        res.evals += nev
        if lam is None:
            # line search failed (Algorithm GBO stops); keep a strict decrease if one was seen
            if best is not None and best[0] < J:
                xn, Jn, gn = best[1]
                x, J, g = xn, Jn, gn
                res.history.append(dict(m=m + 1, J=J, gnorm=float(np.linalg.norm(g)), lam=0.0,
                                        evals=res.evals, x=x.copy()))
            reason = "line search"
            break
        xn, Jn, gn = pay
        s = xn - x
        y = gn - g
        if float(s @ y) > 1e-300:
            S.append(s)
            Y.append(y)
            if len(S) > memory:
                S.pop(0)
                Y.pop(0)
            gamma = float(s @ y) / float(y @ y)
        den = xn + x
        with np.errstate(divide="ignore", invalid="ignore"):
            relchg = np.where(den != 0, np.abs(2.0 * s / den), np.where(s == 0, 0.0, np.inf))
        x, J, g = xn, Jn, gn
        res.history.append(dict(m=m + 1, J=J, gnorm=float(np.linalg.norm(g)), lam=lam if lam else 0.0,
                                evals=res.evals, x=x.copy()))
        if callback:
            callback(res.history[-1])
        if np.linalg.norm(g) < eps:
            reason = "gradient"
            break
        if np.all(relchg < eps_alpha):
            reason = "control change"
            break
    res.x, res.J, res.grad = x.reshape(shape), J, g.reshape(shape)
    res.steps = len(res.history) - 1
    res.reason = reason
    res.wall_s = time.perf_counter() - t0
    return res


def gpu_objective(ctx):
    """fun(x) -> (J, grad) through the HIP library's objective_and_grad.  A
    solve that stops at max_steps before tol raises slbm.NotConverged: a
    non-steady J or gradient would mislead the line search."""
    from . import slbm as S

    def fun(x):
        rc, J, grad, pi, ai = S.objective_and_grad(ctx, np.ascontiguousarray(x, dtype=np.float64))
        S.require_converged(rc, "objective_and_grad", pi if not pi.converged else ai)
        fun.sweeps += pi.sweeps + ai.sweeps
        fun.device_ms += pi.device_ms + ai.device_ms
        return J, np.asarray(grad).reshape(np.shape(x))

    fun.sweeps = 0
    fun.device_ms = 0.0
    return fun
