"""The paper's convergence test on the GPU (SLBM_CONV_CV): c(t) = mean over
the domain nodes of |d(t)|^2 at every check, converged when its coefficient of
variation over a window of checks is below tol (eq. convergence, eq.
convergence_crit).  The step at which the solves stop, J and the gradient
equal the oracle's own implementation of the test (needs a GPU)."""
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


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.mark.parametrize("n,window", [(32, 10), (48, 4)])
def test_cv_gradient_matches_oracle_periodic(S, orc, n, window):
    modes = I.two_mode_basis(n)
    tgt = I.two_mode_target(n)
    p = dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=S.PERIODIC, target=tgt, control_kind=S.CTRL_FORCE_MODES,
             n_modes=2, force_modes=modes, tol=1e-7, convergence=S.CONV_CV, cv_window=window)
    ctx = S.solid_lbm_init(p)
    a = np.array([0.1, 0.1])
    rc, J, grad, pi, ai = S.objective_and_grad(ctx, a)
    G = orc.objective_and_grad(orc.Problem(n, n, 1 / n, 1.0, 0.3, np.zeros((2, n, n))), tgt, "modes", a,
                               modes=modes, tol=1e-7, cv_window=window)
    assert rc == 0 and pi.converged and ai.converged
    assert (pi.steps, ai.steps) == (G.prim.steps, G.adj.steps)
    assert abs(pi.residual - G.prim.residual) <= 1e-6 * G.prim.residual
    assert abs(J - G.J) <= 1e-12 * G.J
    assert rel(grad, G.grad) < 1e-10


def test_cv_gradient_matches_oracle_plate(S, orc):
    pd = I.paper_plate(16)
    p = dict(nx=pd["nx"], ny=pd["ny"], dx=pd["dx"], E=pd["E"], nu=pd["nu"], domain=S.MASKED,
             node_mask=pd["active"].astype(np.uint8), link_bc=pd["bc"], link_wall=pd["wall"],
             link_normal=pd["normal"], target=pd["target"], control_kind=S.CTRL_FORCE_NODAL, tol=1e-7,
             convergence=S.CONV_CV)
    ctx = S.solid_lbm_init(p)
    rc, J, grad, pi, ai = S.objective_and_grad(ctx, pd["F"])
    q = orc.Problem(pd["nx"], pd["ny"], pd["dx"], pd["E"], pd["nu"], np.zeros((2, pd["ny"], pd["nx"])),
                    active=pd["active"], bc=pd["bc"], wall=pd["wall"], normal=pd["normal"])
    G = orc.objective_and_grad(q, pd["target"], "nodal", pd["F"], tol=1e-7, cv_window=10)
    assert rc == 0
    assert (pi.steps, ai.steps) == (G.prim.steps, G.adj.steps)
    assert abs(J - G.J) <= 1e-11 * G.J
    assert rel(np.asarray(grad).reshape(G.grad.shape), G.grad) < 1e-9


def test_cv_zero_state_stops_at_the_first_full_window(S):
    n = 32
    p = dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=S.PERIODIC, target=I.two_mode_target(n),
             control_kind=S.CTRL_FORCE_NODAL, tol=1e-7, convergence=S.CONV_CV, cv_window=3)
    ctx = S.solid_lbm_init(p)
    rc, info = S.primal_solve(ctx, np.zeros((2, n, n)))
    K = 2 * int(np.ceil(0.005 * n * n - 1e-9))
    assert rc == 0 and info.converged and info.steps == 3 * K and info.residual == 0.0


def test_cv_mode_limits(S):
    n = 16
    base = dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=S.PERIODIC, target=I.two_mode_target(n),
                control_kind=S.CTRL_FORCE_MODES, n_modes=2, force_modes=I.two_mode_basis(n), tol=1e-7)
    for bad in (dict(convergence=2), dict(convergence=S.CONV_CV, cv_window=1),
                dict(convergence=S.CONV_CV, cv_window=33)):
        with pytest.raises(S.SlbmError):
            S.solid_lbm_init(dict(base, **bad))
    cv = dict(base, convergence=S.CONV_CV)
    with pytest.raises(S.SlbmError):
        S.solid_lbm_batch_init([cv, base])
    ctx = S.solid_lbm_init(cv)
    with pytest.raises(S.SlbmError):
        S.tangent_solve(ctx, np.array([0.1, 0.1]), np.array([1.0, 0.0]))
