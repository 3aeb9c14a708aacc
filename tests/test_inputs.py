"""The seeded input generators hold the properties their readings state
(no GPU).  They carry no method arithmetic: these are checks of the problem
data that the oracle and the HIP path both receive."""
import math

import numpy as np

from paper_2609_31347_amd import inputs as I


def test_grf_mean_variance_spectrum_and_seed():
    """Reading C16: zero mean, the exact variance, no mean or Nyquist content,
    reproducible by seed; a longer correlation length gives a smoother field."""
    n, dx = 64, 1 / 64
    f = I.grf(n, n, dx, 0.05, 0.1, 7, comps=2)
    assert f.shape == (2, n, n)
    for c in range(2):
        assert abs(f[c].mean()) < 1e-15
        assert abs(f[c].var() - 0.05) < 1e-14
        F = np.fft.fft2(f[c])
        assert np.abs(F[:, n // 2]).max() < 1e-12 and np.abs(F[n // 2, :]).max() < 1e-12
    assert np.array_equal(f, I.grf(n, n, dx, 0.05, 0.1, 7, comps=2))
    assert not np.allclose(f, I.grf(n, n, dx, 0.05, 0.1, 8, comps=2))
    lag1 = lambda g: float((g * np.roll(g, 1, axis=1)).mean() / g.var())
    smooth, rough = I.grf(n, n, dx, 1.0, 0.2, 3)[0], I.grf(n, n, dx, 1.0, 0.03, 3)[0]
    assert lag1(smooth) > lag1(rough)


def test_two_mode_target_solves_the_navier_lame_equations():
    """Reading C10: with F = A1 b1 + A2 b2 the target d* satisfies
    mu lap d + K grad div d + F = 0 on the unit torus (plane-stress mu, K).
    The derivatives are taken spectrally, exact for these trigonometric fields."""
    n, E, nu = 32, 1.0, 0.3
    _, mu, K = I.lame(E, nu)
    d = I.two_mode_target(n, E, nu)
    b = I.two_mode_basis(n)
    F = 0.7 * b[0] + 0.3 * b[1]
    k = 2 * np.pi * np.fft.fftfreq(n, d=1 / n)
    KX, KY = np.meshgrid(k, k)
    dh = np.fft.fft2(d, axes=(1, 2))
    lap = -(KX ** 2 + KY ** 2) * dh
    div = 1j * KX * dh[0] + 1j * KY * dh[1]
    Ld = np.real(np.fft.ifft2(np.stack([mu * lap[0] + K * 1j * KX * div, mu * lap[1] + K * 1j * KY * div]),
                              axes=(1, 2)))
    assert np.abs(Ld + F).max() < 1e-12 * np.abs(F).max()


def test_clamped_plate_links_kinds_and_normals():
    """Reading C14: link kinds exactly on links from outside nodes, Dirichlet
    (clamped, d_D = 0) on the left arc x - xc <= -a cos 45 deg, the uniform
    traction elsewhere (lattice units: times dx), unit outward normals."""
    cp = I.clamped_plate(64, 39)
    act, bc, X = cp["active"], cp["bc"], cp["X"]
    xc, dx = cp["center"][0], cp["dx"]
    for q in range(8):
        src = np.roll(act, shift=(int(I.CY[q]), int(I.CX[q])), axis=(0, 1))
        assert np.array_equal(bc[q] != 0, act & ~src), q
        iy, ix = np.nonzero(bc[q])
        xo = X[iy, ix] - I.CX[q] * dx
        left = xo - xc <= -math.cos(math.pi / 4)
        assert np.array_equal(bc[q][iy, ix] == I.DIRICHLET, left), q
        w = cp["wall"][:, q, iy, ix]
        assert np.all(w[:, left] == 0.0)
        assert np.allclose(w[0, ~left], 0.0) and np.allclose(w[1, ~left], -1e-3 * dx)
        nrm = cp["normal"][:, q, iy, ix]
        assert np.allclose(np.hypot(nrm[0], nrm[1]), 1.0)
        # the normal points away from the centre
        assert np.all(nrm[0] * (X[iy, ix] - xc) + nrm[1] * (cp["Y"][iy, ix] - cp["center"][1]) > 0)
