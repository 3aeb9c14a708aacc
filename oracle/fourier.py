"""Closed-form steady state of the periodic, uniform-material scheme (test infrastructure).

On a periodic lattice with one material every node shares the affine collision
f^C = C f^S + B g, and streaming f^S_q(x) = f^C_q(x - c_q) is diagonal in
Fourier space with phase exp(-i k.c_q).  The fixed point of eq.
primal_fixed_point is therefore, per wavevector k != 0,

    (I - P(k) C) f^ = P(k) B g^,     d^ = M_12 f^ + g^ / 2,

where P(k) = diag(exp(-i k.c_q)) and M_12 are the first two rows of M
(eq. disp_from_moments).  k = 0 carries the rigid translation and is set to
zero (zero-mean forcing, zero-mean initial state).  The exact nodal gradient of
J for a forcing control follows from the adjoint of this convolution.

C and B are built here from the paper's moment-space description with numpy
(matrix M of the appendix, equilibrium N of eq. moments_eq, relaxation of
eq. moments_c with the relaxation-time table) -- a second, matrix-form
encoding of the collision, independent of the C oracle's node loop.
"""
import numpy as np

THETA = 1.0 / 3.0
CX = np.array([1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 1, 0, -1, 1, 1, -1, -1])
M = np.array([
    [1, 0, -1, 0, 1, -1, -1, 1],
    [0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, 0, 0, 1, -1, 1, -1],
    [1, 1, 1, 1, 2, 2, 2, 2],
    [1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 1, -1, -1, 1],
    [0, 0, 0, 0, 1, 1, -1, -1],
    [0, 0, 0, 0, 1, 1, 1, 1]], dtype=np.float64)


def collision_matrices(E, nu):
    """(C, B): f^C = C f^S + B g for a bulk node (gamma = 0), from eq. moments_c,
    the relaxation-time table and the appendix matrix M."""
    mu = E / (2 * (1 + nu))
    K = E / (2 * (1 - nu))
    taus = {2: mu / THETA, 3: 2 * K / (1 + THETA), 4: 2 * mu / (1 - THETA), 5: 0.5, 6: 0.5, 7: 0.5}
    Nm = np.zeros((8, 2))
    Nm[0, 0] = Nm[1, 1] = 1.0
    Nm[5, 0] = Nm[6, 1] = THETA
    # moment map: m^C = A m + b g with the bared first moments mbar = m_1 + g/2
    A = np.zeros((8, 8))
    b = np.zeros((8, 2))
    A[0, 0] = A[1, 1] = 1.0          # m^C_10 = m10 + g/2 + g/2
    b[0, 0] = b[1, 1] = 1.0
    for beta, tau in taus.items():
        w = 1.0 / (tau + 0.5)
        A[beta, beta] += 1.0 - w
        A[beta, 0] += w * Nm[beta, 0]
        A[beta, 1] += w * Nm[beta, 1]
        b[beta, 0] += w * Nm[beta, 0] / 2
        b[beta, 1] += w * Nm[beta, 1] / 2
    Minv = np.linalg.inv(M)
    return Minv @ A @ M, Minv @ b


def transfer(nx, ny, E, nu):
    """H(k) (ny, nx, 2, 2) with d^ = H g^, and H(0) = 0: eq. primal_fixed_point
    per wavevector, read out by eq. disp_from_moments."""
    C, B = collision_matrices(E, nu)
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    KX, KY = np.meshgrid(kx, ky)
    ph = np.exp(-1j * (KX[..., None] * CX + KY[..., None] * CY))      # (ny, nx, 8)
    PC = ph[..., :, None] * C                                          # (ny, nx, 8, 8)
    lhs = np.eye(8) - PC
    rhs = ph[..., :, None] * B                                         # (ny, nx, 8, 2)
    lhs[0, 0] = np.eye(8)
    rhs[0, 0] = 0.0
    fhat = np.linalg.solve(lhs.reshape(-1, 8, 8), rhs.reshape(-1, 8, 2)).reshape(ny, nx, 8, 2)
    H = np.einsum("aq,yxqc->yxac", M[:2], fhat) + 0.5 * np.eye(2)
    H[0, 0] = 0.0
    return H


def steady_disp(g, E, nu, H=None):
    """Exact fixed-point displacement (2, ny, nx) of eq. primal_fixed_point for
    forcing g (2, ny, nx)."""
    ny, nx = g.shape[1:]
    H = transfer(nx, ny, E, nu) if H is None else H
    gh = np.fft.fft2(g, axes=(1, 2))
    dh = np.einsum("yxac,cyx->ayx", H, gh)
    return np.real(np.fft.ifft2(dh, axes=(1, 2)))


def grad_g(r, E, nu, H=None):
    """Adjoint of the map g -> d of eq. primal_fixed_point applied to r:
    (dd/dg)^T r, shape (2, ny, nx) (the force part of eq. optimality)."""
    ny, nx = r.shape[1:]
    H = transfer(nx, ny, E, nu) if H is None else H
    rh = np.fft.fft2(r, axes=(1, 2))
    gh = np.einsum("yxca,cyx->ayx", np.conj(H), rh)
    return np.real(np.fft.ifft2(gh, axes=(1, 2)))


def mode_decay(nx, ny, E, nu, k):
    """Moduli of the eigenvalues of P(k) C, one step (eq. local_collide, then
    eq. local_stream) of the Fourier mode k = (kx, ky)."""
    C, _ = collision_matrices(E, nu)
    kap = (2 * np.pi * k[0] / nx, 2 * np.pi * k[1] / ny)
    P = np.exp(-1j * (kap[0] * CX + kap[1] * CY))
    return np.abs(np.linalg.eigvals(P[:, None] * C))


def steady_pops(g, E, nu):
    """Exact fixed-point populations f^S (8, ny, nx) of eq. primal_fixed_point for
    forcing g (2, ny, nx)."""
    ny, nx = g.shape[1:]
    C, B = collision_matrices(E, nu)
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    KX, KY = np.meshgrid(kx, ky)
    ph = np.exp(-1j * (KX[..., None] * CX + KY[..., None] * CY))
    lhs = np.eye(8) - ph[..., :, None] * C
    rhs = ph[..., :, None] * B
    lhs[0, 0] = np.eye(8)
    rhs[0, 0] = 0.0
    T = np.linalg.solve(lhs.reshape(-1, 8, 8), rhs.reshape(-1, 8, 2)).reshape(ny, nx, 8, 2)
    gh = np.fft.fft2(g, axes=(1, 2))
    fh = np.einsum("yxqc,cyx->qyx", T, gh)
    return np.real(np.fft.ifft2(fh, axes=(1, 2)))
