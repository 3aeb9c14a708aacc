"""Forward-mode (tangent) solves on the GPU: the directional derivative of J
equals the oracle's complex-step forward mode and the adjoint gradient's
projection on the direction, for every control kind (needs a GPU)."""
import numpy as np
import pytest

from paper_2609_31347_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_31347_amd import slbm
    return slbm


def plate_problem(S, pd, kind, **kw):
    d = dict(nx=pd["nx"], ny=pd["ny"], dx=pd["dx"], E=pd.get("E", 1.0), nu=pd.get("nu", 0.3), domain=S.MASKED,
             node_mask=pd["active"].astype(np.uint8), link_bc=pd["bc"], link_wall=pd["wall"],
             link_normal=pd["normal"], target=pd["target"], control_kind=kind)
    d.update(kw)
    return d


def test_tangent_E_scalar_matches_oracle_forward_mode(S, orc):
    # periodic: the paper's manufactured problem
    n = 20
    sol = I.paper_periodic(n)
    p = dict(nx=n, ny=n, dx=1 / n, E=0.11, nu=0.8, domain=0, target=sol["d"], control_kind=S.CTRL_E_SCALAR_SQ,
             fixed_force=sol["F"], tol=1e-12)
    ctx = S.solid_lbm_init(p)
    alpha = np.sqrt(0.15)
    rc, J, dJ, info = S.tangent_solve(ctx, np.array([alpha]), np.array([1.0]))
    assert info.converged
    q = orc.Problem(n, n, 1 / n, 0.11, 0.8, np.zeros((2, n, n)))
    ref = orc.fad_grad_E_sq(q, sol["d"], alpha, sol["F"], tol=1e-12)
    G = orc.objective_and_grad(q, sol["d"], "E_sq", [alpha], fixed_force=sol["F"], tol=1e-12)
    assert abs(dJ - ref) <= 1e-9 * abs(ref)
    assert abs(J - G.J) <= 1e-10 * G.J
    # plate: closures and gamma depend on E
    pd = I.paper_plate(16)
    p = plate_problem(S, pd, S.CTRL_E_SCALAR_SQ, fixed_force=pd["F"], tol=1e-12)
    ctx = S.solid_lbm_init(p)
    rc, J, dJ, info = S.tangent_solve(ctx, np.array([alpha]), np.array([1.0]))
    q = orc.Problem(pd["nx"], pd["ny"], pd["dx"], 0.1, 0.7, np.zeros((2, pd["ny"], pd["nx"])), active=pd["active"],
                    bc=pd["bc"], wall=pd["wall"], normal=pd["normal"])
    # the oracle's complex-step solve stops on the residual of the real part;
    # its imaginary part (the derivative) carries a t lambda^t term and lags, so
    # on the plate's slow modes it is run deeper than the GPU tangent, which
    # tests both parts
    ref = orc.fad_grad_E_sq(q, pd["target"], alpha, pd["F"], tol=1e-14)
    assert abs(dJ - ref) <= 1e-9 * abs(ref)
    rc, Ja, ga, _, _ = S.objective_and_grad(ctx, np.array([alpha]))
    assert abs(dJ - float(np.asarray(ga)[0])) <= 1e-9 * abs(ref)


def test_tangent_modes_match_oracle_and_adjoint(S, orc):
    n = 32
    modes = I.two_mode_basis(n)
    tgt = I.two_mode_target(n)
    p = dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=0, target=tgt, control_kind=S.CTRL_FORCE_MODES,
             n_modes=2, force_modes=modes, tol=1e-12)
    ctx = S.solid_lbm_init(p)
    a = np.array([0.1, 0.1])
    q = orc.Problem(n, n, 1 / n, 1.0, 0.3, np.zeros((2, n, n)))
    ref = orc.fad_grad_modes(q, tgt, a, modes, tol=1e-12)
    rc, J, g, _, _ = S.objective_and_grad(ctx, a)
    for i in range(2):
        e = np.zeros(2)
        e[i] = 1.0
        rc, Jt, dJ, info = S.tangent_solve(ctx, a, e)
        assert abs(dJ - ref[i]) <= 1e-9 * np.abs(ref).max()
        assert abs(dJ - g[i]) <= 1e-9 * np.abs(ref).max()
        assert abs(Jt - J) <= 1e-10 * J
    # linearity in the direction
    d = np.array([0.3, -1.7])
    rc, _, dJ, _ = S.tangent_solve(ctx, a, d)
    assert abs(dJ - d @ np.asarray(g)) <= 1e-9 * np.abs(ref).max()


def test_tangent_nodal_force_and_E_field_match_adjoint(S):
    rng = np.random.default_rng(3)
    # periodic nodal force: the direction is projected to zero mean like the control
    nx, ny, dx = 48, 40, 1 / 48
    p = dict(nx=nx, ny=ny, dx=dx, E=0.8, nu=0.25, domain=0, target=I.grf(nx, ny, dx, 1e-6, 0.15, 4, comps=2),
             control_kind=S.CTRL_FORCE_NODAL, tol=1e-12)
    ctx = S.solid_lbm_init(p)
    F = I.grf(nx, ny, dx, 0.05, 0.1, 5, comps=2)
    rc, J, g, _, _ = S.objective_and_grad(ctx, F)
    d = rng.standard_normal((2, ny, nx)) + 0.3            # non-zero mean on purpose
    rc, Jt, dJ, info = S.tangent_solve(ctx, F, d)
    ref = float(np.asarray(g).ravel() @ d.ravel())
    assert abs(dJ - ref) <= 1e-8 * abs(ref)
    # E field on a plate
    cp = I.clamped_plate(40, 25)
    tgt = 1e-4 * np.stack([cp["X"], cp["Y"]]) * cp["active"]
    pd = dict(cp, target=tgt)
    p = plate_problem(S, pd, S.CTRL_E_NODAL, tol=1e-12)
    ctx = S.solid_lbm_init(p)
    E = 1.0 + 0.3 * np.tanh(I.grf(40, 25, cp["dx"], 1.0, 0.3, 12)[0])
    rc, J, g, _, _ = S.objective_and_grad(ctx, E)
    d = rng.standard_normal((25, 40)) * cp["active"]
    rc, Jt, dJ, info = S.tangent_solve(ctx, E, d)
    ref = float(np.asarray(g).ravel() @ d.ravel())
    assert abs(dJ - ref) <= 1e-8 * abs(ref)
    # the tangent stops at a later check (value and derivative converged) than
    # the primal; on the plate's slow modes the primal's remaining error is up to
    # ~400 x its residual, doubled in J (target << d here)
    assert abs(Jt - J) <= 1e-8 * J
    # zero direction: zero derivative
    rc, Jt, dJ, info = S.tangent_solve(ctx, E, np.zeros((25, 40)))
    assert dJ == 0.0 and info.converged
