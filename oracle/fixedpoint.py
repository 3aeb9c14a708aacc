"""Exact fixed point of the oracle's affine step map by a sparse direct solve.

TEST INFRASTRUCTURE ONLY.  One primal step is affine, f^S(t+1) = A f^S(t) + b,
so its fixed point (eq. primal_fixed_point) solves (I - A) f = b and the
adjoint fixed point (eq. adjoint_streaming / eq. adjoint_collision) solves
(I - A^T) lam = (dJ/df)^T.  A is assembled column-wise by applying the oracle's
own step (zero forcing, zero wall data) to unit inputs; nodes whose outputs
cannot overlap (coordinates equal modulo m >= 3 on both axes) are probed
together.  This pins the time marching, the convergence test and the two-step
average (the solve must land on the same fixed point), and -- through the
transposed system -- the adjoint of any boundary closure.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from . import oracle as O


def _modulus(n):
    for m in range(3, n + 1):
        if n % m == 0:
            return m
    return n


def step_matrix(p):
    """(A, idx): sparse linear part of one step (eq. local_collide, eq. local_stream,
    closures of reading C13) restricted to domain slots."""
    nx, ny, N = p.nx, p.ny, p.N
    q0 = p.with_(g=np.zeros((2, ny, nx)), wall=None if p.wall is None else np.zeros_like(p.wall))
    mx, my = _modulus(nx), _modulus(ny)
    act = p.mask
    rows, cols, vals = [], [], []
    for ox in range(mx):
        for oy in range(my):
            col = np.zeros((ny, nx), bool)
            col[oy::my, ox::mx] = True
            col &= act
            if not col.any():
                continue
            for pp in range(8):
                e = np.zeros((8, ny, nx))
                e[pp][col] = 1.0
                out = O.step(q0, e)[0]
                qq, yy, xx = np.nonzero(out)
                rx, ry = (xx - ox) % mx, (yy - oy) % my
                sx = np.where(rx == mx - 1, xx + 1, xx - rx) % nx
                sy = np.where(ry == my - 1, yy + 1, yy - ry) % ny
                rows.append(qq * N + yy * nx + xx)
                cols.append(pp * N + sy * nx + sx)
                vals.append(out[qq, yy, xx])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(8 * N, 8 * N))
    idx = np.flatnonzero(np.broadcast_to(act, (8, ny, nx)).ravel())
    return A[idx][:, idx].tocsc(), idx


def forcing_matrix(p):
    """Sparse map g (2N) -> constant part of one step (8N, domain slots): the
    forcing of eq. local_collide after eq. local_stream."""
    nx, ny, N = p.nx, p.ny, p.N
    mx, my = _modulus(nx), _modulus(ny)
    act = p.mask
    rows, cols, vals = [], [], []
    for ox in range(mx):
        for oy in range(my):
            col = np.zeros((ny, nx), bool)
            col[oy::my, ox::mx] = True
            col &= act
            if not col.any():
                continue
            for c in range(2):
                g = np.zeros((2, ny, nx))
                g[c][col] = 1.0
                q = p.with_(g=g, wall=None if p.wall is None else np.zeros_like(p.wall))
                out = O.step(q, np.zeros((8, ny, nx)))[0]
                qq, yy, xx = np.nonzero(out)
                rx, ry = (xx - ox) % mx, (yy - oy) % my
                sx = np.where(rx == mx - 1, xx + 1, xx - rx) % nx
                sy = np.where(ry == my - 1, yy + 1, yy - ry) % ny
                rows.append(qq * N + yy * nx + xx)
                cols.append(c * N + sy * nx + sx)
                vals.append(out[qq, yy, xx])
    G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(8 * N, 2 * N))
    idx = np.flatnonzero(np.broadcast_to(act, (8, ny, nx)).ravel())
    return G[idx].tocsc()


def fixed_point(p, A=None, idx=None):
    """Exact steady populations f^S (8, ny, nx) and displacement d (2, ny, nx):
    eq. primal_fixed_point solved directly."""
    if A is None:
        A, idx = step_matrix(p)
    b = O.step(p, np.zeros((8, p.ny, p.nx)))[0].ravel()[idx]
    I = sp.identity(A.shape[0], format="csc")
    x = spl.spsolve((I - A).tocsc(), b)
    f = np.zeros(8 * p.N)
    f[idx] = x
    f = f.reshape(8, p.ny, p.nx)
    d = _disp(p, f)
    return f, d


def _disp(p, f):
    m10 = (O.CX[:, None, None] * f).sum(0)
    m01 = (O.CY[:, None, None] * f).sum(0)
    return np.stack([m10 + p.g[0] / 2, m01 + p.g[1] / 2]) * p.mask


def nodal_force_gradient(p, r, scale, A=None, idx=None):
    """Exact dJ/dg (2, ny, nx) of eq. optimality for a force control, through
    the transposed fixed-point system, for J = 1/2 sum |d - d*|^2 * scale with
    r = d - d* (zero off the observation set):  dJ/dg = G^T (I - A)^-T M12^T r s + r s / 2."""
    if A is None:
        A, idx = step_matrix(p)
    G = forcing_matrix(p)
    nx, ny, N = p.nx, p.ny, p.N
    w = np.zeros(8 * N)
    for q in range(8):
        w[q * N:(q + 1) * N] = (O.CX[q] * r[0] + O.CY[q] * r[1]).ravel() * scale
    rhs = w[idx]
    I = sp.identity(A.shape[0], format="csc")
    lam = spl.spsolve((I - A).T.tocsc(), rhs)
    out = (G.T @ lam).reshape(2, ny, nx)
    return (out + 0.5 * r * scale) * p.mask
