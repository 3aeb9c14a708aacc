"""Edge cases of the method and of the C ABI on the GPU, against the oracle.

* The undamped period-2 (Nyquist) mode of the periodic scheme (reading C7):
  white-noise nodal forcing excites it; the solve must still stop on the K-lag
  residual and return the two-step-averaged fixed point, primal and adjoint,
  in the wave-strip and the LDS-tiled launches.
* A target with a non-zero mean on the torus (reading C21).
* Call order: a VJP between a primal and an adjoint solve must not change
  what the adjoint differentiates.
* Error paths: max_steps reached before tol (SLBM_NOT_CONVERGED) and
  non-finite controls (SLBM_ENONFINITE, context unchanged).
"""
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


def periodic(nx, ny, target, **kw):
    d = dict(nx=nx, ny=ny, dx=1.0 / nx, E=1.0, nu=0.3, domain=0, target=target,
             control_kind=1, tol=1e-10)
    d.update(kw)
    return d


@pytest.mark.parametrize("nx,ny,shape", [(24, 20, "tiles"), (24, 20, "strips"), (130, 34, "strips")])
def test_nyquist_forcing_converges_to_the_oracle_fixed_point(S, orc, nx, ny, shape):
    """White-noise forcing has Nyquist content (the (pi, 0) and (0, pi)
    rows carry an eigenvalue -1 of the step, reading C7): the raw iterate
    never settles, but the even K-lag test passes and the two-step average is
    the fixed point.  GPU and oracle stop at the same check, primal and
    adjoint; J to 1e-12, d to 1e-12, gradient to 1e-10."""
    rng = np.random.default_rng(7)
    F = rng.standard_normal((2, ny, nx))
    F -= F.mean((1, 2), keepdims=True)
    # the forcing really has Nyquist content in both components
    for c in range(2):
        spec = np.abs(np.fft.fft2(F[c]))
        assert spec[0, nx // 2] > 1e-3 * spec.max() and spec[ny // 2, 0] > 1e-3 * spec.max()
    tgt = 1e-3 * rng.standard_normal((2, ny, nx))
    tgt -= tgt.mean((1, 2), keepdims=True)
    p = periodic(nx, ny, tgt)
    ctx = S.solid_lbm_init(p)
    S.solid_lbm_set_tuning(ctx, 8, 0)
    if shape == "tiles":
        S.solid_lbm_set_tiles(ctx, 8, 8)
    rc, J, g, pi, ai = S.objective_and_grad(ctx, F)
    assert rc == 0 and pi.converged and ai.converged
    q = orc.Problem(nx, ny, 1.0 / nx, 1.0, 0.3, np.zeros((2, ny, nx)))
    G = orc.objective_and_grad(q, tgt, "nodal", F, tol=1e-10)
    assert G.prim.rc == 0 and G.adj.rc == 0
    assert pi.steps == G.prim.steps and ai.steps == G.adj.steps
    assert abs(J - G.J) <= 1e-12 * G.J
    assert rel(S.solid_lbm_get_field(ctx, S.FIELD_DISP), G.prim.dbar) < 1e-12
    assert rel(g.reshape(2, ny, nx), G.grad) < 1e-10
    # the current (raw) state is off the fixed point by the undamped mode
    raw = S.solid_lbm_get_field(ctx, S.FIELD_CUR_DISP)
    assert rel(raw, G.prim.dbar) > 1e-8


def test_nonzero_mean_target_gradient(S, orc):
    """A shifted target on the torus: J keeps the full misfit, the adjoint
    takes its zero-mean part (reading C21); gradient equal to the oracle's, and
    the residual field is still d - d* after the adjoint."""
    n = 40
    rng = np.random.default_rng(3)
    tgt = I.grf(n, n, 1 / n, 1e-6, 0.15, 5, comps=2) + np.array([2e-3, -1e-3])[:, None, None]
    F = I.grf(n, n, 1 / n, 0.05, 0.1, 6, comps=2) + 0.01 * rng.standard_normal((2, n, n))
    p = periodic(n, n, tgt)
    ctx = S.solid_lbm_init(p)
    rc, J, g, pi, ai = S.objective_and_grad(ctx, F)
    assert rc == 0
    q = orc.Problem(n, n, 1.0 / n, 1.0, 0.3, np.zeros((2, n, n)))
    G = orc.objective_and_grad(q, tgt, "nodal", F, tol=1e-10)
    assert pi.steps == G.prim.steps and ai.steps == G.adj.steps
    assert abs(J - G.J) <= 1e-12 * G.J
    assert rel(g.reshape(2, n, n), G.grad) < 1e-10
    r = S.solid_lbm_get_field(ctx, S.FIELD_RESIDUAL)
    assert rel(r, G.prim.dbar - tgt) < 1e-12
    assert np.abs(r.mean((1, 2)) - (-np.array([2e-3, -1e-3]))).max() < 1e-6


def test_vjp_between_primal_and_adjoint_keeps_the_objective(S):
    """primal_solve, adjoint_solve_vjp with some cotangent, then adjoint_solve:
    the adjoint still differentiates J (same gradient as objective_and_grad),
    and J and the residual field are unchanged by the VJP."""
    n = 48
    modes = I.two_mode_basis(n)
    p = dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=0, target=I.two_mode_target(n), control_kind=0,
             n_modes=2, force_modes=modes, tol=1e-10)
    ctx = S.solid_lbm_init(p)
    a = np.array([0.1, 0.1])
    rc, J0, g0, _, _ = S.objective_and_grad(ctx, a)
    S.primal_solve(ctx, a)
    r0 = S.solid_lbm_get_field(ctx, S.FIELD_RESIDUAL)
    cot = np.random.default_rng(1).standard_normal((2, n, n))
    S.adjoint_solve_vjp(ctx, cot)
    assert S.solid_lbm_objective(ctx) == J0
    assert np.array_equal(S.solid_lbm_get_field(ctx, S.FIELD_RESIDUAL), r0)
    S.adjoint_solve(ctx)
    # the gradient of the objective from the adjoint just run: objective_and_grad
    # again must reproduce it bit for bit (same arithmetic, same source)
    rc, J1, g1, _, _ = S.objective_and_grad(ctx, a)
    assert J1 == J0 and np.array_equal(g1, g0)
    adj_after = S.solid_lbm_get_field(ctx, S.FIELD_ADJ_DISP)
    S.primal_solve(ctx, a)
    S.adjoint_solve_vjp(ctx, cot)
    S.adjoint_solve(ctx)
    assert np.array_equal(S.solid_lbm_get_field(ctx, S.FIELD_ADJ_DISP), adj_after)


def test_step_limit_returns_not_converged(S):
    """max_steps reached before tol: rc = SLBM_NOT_CONVERGED (> 0), outputs
    written, info says not converged at max_steps; the strict wrappers raise."""
    import torch
    from paper_2609_31347_amd import autograd as AG
    n = 64
    modes = I.two_mode_basis(n)
    p = dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=0, target=I.two_mode_target(n), control_kind=0,
             n_modes=2, force_modes=modes, tol=1e-10, max_steps=100)
    ctx = S.solid_lbm_init(p)
    rc, J, g, pi, ai = S.objective_and_grad(ctx, np.array([0.1, 0.1]))
    assert rc == S.NOT_CONVERGED
    assert not pi.converged and not ai.converged
    assert pi.steps == 100 and ai.steps == 100 and pi.sweeps == 101
    assert np.isfinite(J) and np.all(np.isfinite(g)) and pi.residual > 1e-10
    solver = AG.Solver(p, tune=False)
    x = torch.tensor([0.1, 0.1], dtype=torch.float64, device="cuda", requires_grad=True)
    with pytest.raises(S.NotConverged):
        AG.displacement(x, solver)
    lax = AG.Solver(p, tune=False, strict=False)
    d = AG.displacement(x, lax)
    assert d.shape == (2, n, n) and not lax.last_info.converged


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_non_finite_control_is_rejected_and_the_context_survives(S, bad):
    """A non-finite control entry returns SLBM_ENONFINITE before any sweep, from
    host and from device memory, and leaves the context as it was."""
    import torch
    n = 32
    p = periodic(n, n, I.two_mode_target(n))
    ctx = S.solid_lbm_init(p)
    F = I.grf(n, n, 1 / n, 0.05, 0.1, 2, comps=2)
    rc, J0, g0, _, _ = S.objective_and_grad(ctx, F)
    assert rc == 0
    badF = F.copy()
    badF[1, 3, 5] = bad
    dev_grad = torch.zeros(2 * n * n, dtype=torch.float64, device="cuda")
    for arg, gout in ((badF, None), (torch.tensor(badF, device="cuda"), dev_grad)):
        with pytest.raises(S.SlbmError) as e:
            S.objective_and_grad(ctx, arg, grad=gout)
        assert e.value.code == S.ENONFINITE
        assert S.solid_lbm_objective(ctx) == J0
    rc, J1, g1, _, _ = S.objective_and_grad(ctx, F)
    assert rc == 0 and J1 == J0 and np.array_equal(g1, g0)
    # scalar modulus control
    pe = dict(periodic(n, n, I.two_mode_target(n)), control_kind=S.CTRL_E_SCALAR_SQ, fixed_force=F)
    ce = S.solid_lbm_init(pe)
    with pytest.raises(S.SlbmError) as e:
        S.objective_and_grad(ce, np.array([bad]))
    assert e.value.code == S.ENONFINITE


def test_autograd_gradient_lands_on_the_control_device(S, orc):
    """A CPU control tensor gets a CPU gradient from the GPU adjoint."""
    import torch
    from paper_2609_31347_amd import autograd as AG
    n = 32
    modes = I.two_mode_basis(n)
    tgt = I.two_mode_target(n)
    p = dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=0, target=tgt, control_kind=0, n_modes=2,
             force_modes=modes, tol=1e-10)
    solver = AG.Solver(p, tune=False)
    a = torch.tensor([0.1, 0.1], dtype=torch.float64, requires_grad=True)       # CPU
    L = AG.misfit(AG.displacement(a, solver), tgt, 1 / n)
    L.backward()
    assert a.grad.device.type == "cpu" and a.grad.dtype == torch.float64
    q = orc.Problem(n, n, 1 / n, 1.0, 0.3, np.zeros((2, n, n)))
    G = orc.objective_and_grad(q, tgt, "modes", [0.1, 0.1], modes=modes, tol=1e-10)
    assert rel(a.grad.numpy(), G.grad) < 1e-10


def test_fused_launch_timing_of_the_solve_loops(S):
    """With launch timing on, the solve loops report their fused launches, the
    sweeps those made (T per strip launch) and a device time within the loop's
    own; off (the default) the fields stay 0.  Results do not change."""
    n = 256
    modes = I.two_mode_basis(n)
    p = dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=0, target=I.two_mode_target(n), control_kind=0,
             n_modes=2, force_modes=modes, tol=1e-10)
    ctx = S.solid_lbm_init(p)
    S.solid_lbm_set_tuning(ctx, 8, 0)
    rc, J0, g0, pi, ai = S.objective_and_grad(ctx, np.array([0.1, 0.1]))
    assert pi.fused_launches == 0 and pi.fused_sweeps == 0 and pi.fused_ms == 0.0
    S.solid_lbm_set_launch_timing(ctx, True)
    rc, J1, g1, pi, ai = S.objective_and_grad(ctx, np.array([0.1, 0.1]))
    assert J1 == J0 and np.array_equal(g1, g0)
    for info in (pi, ai):
        assert info.fused_launches > 0 and info.fused_sweeps == 8 * info.fused_launches
        assert info.fused_sweeps <= info.sweeps
        assert 0.0 < info.fused_ms <= info.device_ms
