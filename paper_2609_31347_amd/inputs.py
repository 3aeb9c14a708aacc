"""Seeded synthetic inputs: manufactured fields, random fields and plate geometry.

This module holds problem data only (manufactured solutions, their body forces
and stresses from the continuum equations, Gaussian random fields, the plate
masks and per-link wall data).  It contains none of the lattice-Boltzmann
arithmetic, so both the HIP path and the CPU oracle can take their inputs from
here.  Every random draw is seeded (numpy PCG64).

Unit conventions (diffusive scaling dt = dx^2, kappa = 1): lattice moduli equal
the physical ones; forcing g = dx^2 F; stress and traction in lattice units are
dx times the physical ones; displacements are the same in both.
"""
import math

import numpy as np

CX = np.array([1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 1, 0, -1, 1, 1, -1, -1])
DIRICHLET, NEUMANN = 1, 2


def lame(E, nu):
    """Plane-stress moduli (eq. lambda, eq. mu, eq. K): returns (lam, mu, K)."""
    lam = E * nu / (1.0 - nu * nu)
    mu = E / (2.0 * (1.0 + nu))
    K = E / (2.0 * (1.0 - nu))
    return lam, mu, K


def grid(nx, ny, dx, x0=0.0, y0=0.0):
    """Node coordinates X, Y of shape (ny, nx): x = x0 + i dx, y = y0 + j dx."""
    x = x0 + np.arange(nx) * dx
    y = y0 + np.arange(ny) * dx
    return np.meshgrid(x, y)


# --------------------------------------------------------------- periodic

def two_mode_basis(n):
    """Body-force modes on the periodic unit square (n x n nodes, dx = 1/n):
    b1 = (sin 2pi x cos 2pi y, cos 2pi x sin 2pi y), b2 = (sin 4pi x, sin 4pi y).
    Returns (2, 2, n, n)."""
    X, Y = grid(n, n, 1.0 / n)
    t = 2.0 * np.pi
    b1 = np.stack([np.sin(t * X) * np.cos(t * Y), np.cos(t * X) * np.sin(t * Y)])
    b2 = np.stack([np.sin(2 * t * X), np.sin(2 * t * Y)])
    return np.stack([b1, b2])


def two_mode_target(n, E=1.0, nu=0.3, A=(0.7, 0.3)):
    """Continuum steady displacement for F = A1 b1 + A2 b2 (reading C10).
    Both modes are gradient fields, so mu lap d + K grad div d = (mu + K) lap d
    and d = A1 b1 / (8 pi^2 (mu + K)) + A2 b2 / (16 pi^2 (mu + K))."""
    _, mu, K = lame(E, nu)
    b = two_mode_basis(n)
    s = mu + K
    return A[0] * b[0] / (8 * np.pi ** 2 * s) + A[1] * b[1] / (16 * np.pi ** 2 * s)


def paper_periodic(n, E=0.11, nu=0.8, delta=(9e-4, 7e-4)):
    """Manufactured periodic solution of the paper (eq. disp_man_periodic,
    eq. force_man_periodic, stress by eq. stress).  Returns dict with d (2,n,n),
    sigma (3,n,n) = (sxx, syy, sxy) physical units, F (2,n,n)."""
    X, Y = grid(n, n, 1.0 / n)
    _, mu, K = lame(E, nu)
    d1, d2 = delta
    t = 2.0 * np.pi
    cx, sx, cy, sy = np.cos(t * X), np.sin(t * X), np.cos(t * Y), np.sin(t * Y)
    d = np.stack([d1 * cx * sy, d2 * sx * cy])
    # gradients
    d1x = -t * d1 * sx * sy
    d1y = t * d1 * cx * cy
    d2x = t * d2 * cx * cy
    d2y = -t * d2 * sx * sy
    sig = _stress(d1x, d1y, d2x, d2y, mu, K)
    F = 4 * np.pi ** 2 * np.stack([(K * (d1 + d2) + 2 * mu * d1) * cx * sy,
                                   (K * (d1 + d2) + 2 * mu * d2) * sx * cy])
    return dict(d=d, sigma=sig, F=F, mu=mu, K=K)


def _stress(d1x, d1y, d2x, d2y, mu, K):
    """eq. stress: sigma = K div I + mu (grad d + grad d^T - div I)."""
    div = d1x + d2y
    return np.stack([K * div + mu * (2 * d1x - div), K * div + mu * (2 * d2y - div), mu * (d1y + d2x)])


def grf(nx, ny, dx, var, ell, seed, comps=1):
    """Periodic Gaussian random field, squared-exponential covariance
    var * exp(-r^2 / (2 ell^2)) by spectral synthesis of PCG64 white noise
    (reading C16).  The mean and the Nyquist rows/columns are removed and the
    sample is rescaled to the exact variance.  Returns (comps, ny, nx)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=dx)
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=dx)
    KX, KY = np.meshgrid(kx, ky)
    amp = np.exp(-(KX ** 2 + KY ** 2) * ell * ell / 4.0)   # sqrt of the Gaussian spectrum
    amp[0, 0] = 0.0
    if nx % 2 == 0:
        amp[:, nx // 2] = 0.0
    if ny % 2 == 0:
        amp[ny // 2, :] = 0.0
    out = np.empty((comps, ny, nx))
    for c in range(comps):
        w = rng.standard_normal((ny, nx))
        f = np.real(np.fft.ifft2(np.fft.fft2(w) * amp))
        f -= f.mean()
        s = f.std()
        out[c] = f * (math.sqrt(var) / s if s > 0 else 0.0)
    return out


def grf_force_control(n, seed, var=0.05, ell=0.1, A=(0.7, 0.3)):
    """Reference nodal force: two-mode manufactured field plus a GRF
    perturbation (variance var, correlation length ell).  Returns (2, n, n)."""
    b = two_mode_basis(n)
    return A[0] * b[0] + A[1] * b[1] + grf(n, n, 1.0 / n, var, ell, seed, comps=2)


# --------------------------------------------------------------- plates

def _ell_local(X, Y, e):
    a2, b2, xc, yc, phi = e
    c, s = math.cos(phi), math.sin(phi)
    xr = c * (X - xc) + s * (Y - yc)
    yr = -s * (X - xc) + c * (Y - yc)
    return xr, yr, a2, b2, c, s


def ellipse_inside(X, Y, e):
    """Inside test of an ellipse (a^2, b^2, xc, yc, phi): the semi-axis a lies
    along x before the rotation by phi (reading C14)."""
    xr, yr, a2, b2, _, _ = _ell_local(X, Y, e)
    return xr * xr / a2 + yr * yr / b2 <= 1.0


def ellipse_normal(X, Y, e):
    """Unit gradient of the ellipse level set (outward from the ellipse)."""
    xr, yr, a2, b2, c, s = _ell_local(X, Y, e)
    gxr, gyr = 2 * xr / a2, 2 * yr / b2
    gx, gy = c * gxr - s * gyr, s * gxr + c * gyr
    nrm = np.hypot(gx, gy)
    nrm = np.where(nrm > 0, nrm, 1.0)
    return gx / nrm, gy / nrm


# Table "ellipseparameter" (L = 1): outer ellipse 1, holes 2 and 3
PAPER_ELLIPSES = (
    (0.48, 0.30, 0.75, 0.75, -math.pi / 9),
    (0.010, 0.018, 0.95, 0.60, 0.0),
    (0.035, 0.010, 0.50, 0.90, 0.0),
)


def paper_plate_solution(X, Y, E=0.1, nu=0.7, delta=(9e-4, 7e-4)):
    """Manufactured plate solution (eq. disp_man_ellipse) with its stress
    (eq. stress) and body force F = -mu lap d - K grad div d."""
    _, mu, K = lame(E, nu)
    d1c, d2c = delta
    p = 2 * np.pi
    sxy, cxy = np.sin(p * X * Y), np.cos(p * X * Y)
    s2, c2 = np.sin(p * Y), np.cos(p * Y)
    d = np.stack([d1c * sxy, d2c * c2 * (1 + X * X)])
    d1x, d1y = d1c * p * Y * cxy, d1c * p * X * cxy
    d2x, d2y = d2c * c2 * 2 * X, -d2c * p * s2 * (1 + X * X)
    sig = _stress(d1x, d1y, d2x, d2y, mu, K)
    lap1 = -d1c * p * p * (X * X + Y * Y) * sxy
    lap2 = d2c * c2 * (2 - p * p * (1 + X * X))
    divx = -d1c * p * p * Y * Y * sxy - 2 * p * d2c * X * s2
    divy = d1c * p * (cxy - p * X * Y * sxy) - d2c * p * p * c2 * (1 + X * X)
    F = np.stack([-mu * lap1 - K * divx, -mu * lap2 - K * divy])
    return dict(d=d, sigma=sig, F=F, mu=mu, K=K)


def _links(active, X, Y, dx, classify, wall_fn):
    """Per-link boundary data of a masked domain.  For a domain node x and
    direction q with x - c_q outside the domain: kind = classify(xo, yo) at the
    outside node, wall point at the link midpoint x - c_q dx / 2, wall value
    and outward normal from wall_fn(kind, xw, yw).  Returns bc (8,ny,nx) uint8,
    wall (2,8,ny,nx), normal (2,8,ny,nx)."""
    ny, nx = active.shape
    bc = np.zeros((8, ny, nx), np.uint8)
    wall = np.zeros((2, 8, ny, nx))
    nrm = np.zeros((2, 8, ny, nx))
    for q in range(8):
        src = np.roll(active, shift=(CY[q], CX[q]), axis=(0, 1))
        cut = active & ~src
        if not cut.any():
            continue
        iy, ix = np.nonzero(cut)
        xo, yo = X[iy, ix] - CX[q] * dx, Y[iy, ix] - CY[q] * dx
        xw, yw = X[iy, ix] - CX[q] * dx / 2, Y[iy, ix] - CY[q] * dx / 2
        kind = classify(xo, yo)
        val, nn = wall_fn(kind, xw, yw)
        bc[q, iy, ix] = kind
        wall[:, q, iy, ix] = val
        nrm[:, q, iy, ix] = nn
    return bc, wall, nrm


def paper_plate(nx_cells, E=0.1, nu=0.7, delta=(9e-4, 7e-4)):
    """Elliptic plate of the bounded-domain benchmark: box [0, 1.5]^2 with
    nx_cells + 1 nodes per direction (dx = 1.5 / nx_cells), Dirichlet d_D = d*
    on the two holes, Neumann T = sigma* n on the outer ellipse, all data from
    the manufactured solution at the reference moduli.  Returns a dict with the
    problem arrays (lattice units) and the manufactured fields."""
    L = 1.5
    n = nx_cells + 1
    dx = L / nx_cells
    X, Y = grid(n, n, dx)
    e1, e2, e3 = PAPER_ELLIPSES
    active = ellipse_inside(X, Y, e1) & ~ellipse_inside(X, Y, e2) & ~ellipse_inside(X, Y, e3)
    if active[0, :].any() or active[-1, :].any() or active[:, 0].any() or active[:, -1].any():
        raise ValueError("plate touches the box edge")

    def classify(xo, yo):
        inner = ellipse_inside(xo, yo, e2) | ellipse_inside(xo, yo, e3)
        return np.where(inner, DIRICHLET, NEUMANN).astype(np.uint8)

    def wall_fn(kind, xw, yw):
        sol = paper_plate_solution(xw, yw, E, nu, delta)
        nxo, nyo = ellipse_normal(xw, yw, e1)
        sxx, syy, sxy = sol["sigma"]
        T = np.stack([sxx * nxo + sxy * nyo, sxy * nxo + syy * nyo]) * dx
        val = np.where(kind == DIRICHLET, sol["d"], T)
        return val, np.stack([nxo, nyo])

    bc, wall, nrm = _links(active, X, Y, dx, classify, wall_fn)
    sol = paper_plate_solution(X, Y, E, nu, delta)
    return dict(nx=n, ny=n, dx=dx, E=E, nu=nu, active=active, bc=bc, wall=wall, normal=nrm,
                F=sol["F"] * active, target=sol["d"] * active, sigma=sol["sigma"] * active, X=X, Y=Y)


def clamped_plate(nx, ny, a=1.0, b=0.6, traction=(0.0, -1e-3), clamp_cos=math.cos(math.pi / 4)):
    """Elliptic plate with semi-axes a x b centred in an nx x ny box of nodes:
    clamped (Dirichlet, d_D = 0) on the left arc x - xc <= -a cos(45 deg) and
    loaded by a uniform traction T on the rest of the rim (Neumann), reading C14.
    dx = 2 a / (nx - 4) keeps a margin of two nodes in x.  Returns a dict."""
    dx = 2.0 * a / (nx - 4)
    xc, yc = 0.5 * (nx - 1) * dx, 0.5 * (ny - 1) * dx
    X, Y = grid(nx, ny, dx)
    e = (a * a, b * b, xc, yc, 0.0)
    active = ellipse_inside(X, Y, e)
    if active[0, :].any() or active[-1, :].any() or active[:, 0].any() or active[:, -1].any():
        raise ValueError("plate touches the box edge")

    def classify(xo, yo):
        return np.where(xo - xc <= -a * clamp_cos, DIRICHLET, NEUMANN).astype(np.uint8)

    def wall_fn(kind, xw, yw):
        nxo, nyo = ellipse_normal(xw, yw, e)
        T = np.stack([np.full_like(xw, traction[0]), np.full_like(xw, traction[1])]) * dx
        val = np.where(kind == DIRICHLET, 0.0, T)
        return val, np.stack([nxo, nyo])

    bc, wall, nrm = _links(active, X, Y, dx, classify, wall_fn)
    return dict(nx=nx, ny=ny, dx=dx, active=active, bc=bc, wall=wall, normal=nrm, X=X, Y=Y,
                center=(xc, yc))
