"""The no-allocation batch entry point (batch_objective_and_grad_noalloc)
against batch_objective_and_grad, through the C ABI (needs a GPU).

Two calls in a row on different batches, the second smaller (fewer and
smaller instances, so fewer work-list entries in the static table that the
first call filled): objectives, gradients and step counts must equal those of
the allocating entry point bit for bit (same kernels, same work items).  A
launch shape whose work-lists exceed the static table is refused before any
work, and the batch stays usable.
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


def first_batch(S):
    """Periodic mode and nodal controls (wave strips), a clamped plate and an
    E-field plate (LDS tiles): both tables in use."""
    probs, ctrls = [], []
    n = 96
    probs.append(dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=0, target=I.two_mode_target(n),
                      control_kind=S.CTRL_FORCE_MODES, n_modes=2, force_modes=I.two_mode_basis(n)))
    ctrls.append(np.array([0.3, -0.2]))
    nx, ny = 150, 70
    probs.append(dict(nx=nx, ny=ny, dx=1 / nx, E=0.8, nu=0.25, domain=0,
                      target=I.grf(nx, ny, 1 / nx, 1e-6, 0.15, 4, comps=2), control_kind=S.CTRL_FORCE_NODAL))
    ctrls.append(I.grf(nx, ny, 1 / nx, 0.05, 0.1, 5, comps=2))
    cp = I.clamped_plate(64, 39)
    tgt = I.grf(64, 39, cp["dx"], 1e-8, 0.3, 8, comps=2) * cp["active"]
    probs.append(dict(nx=64, ny=39, dx=cp["dx"], E=1.0, nu=0.3, domain=S.MASKED,
                      node_mask=cp["active"].astype(np.uint8), link_bc=cp["bc"], link_wall=cp["wall"],
                      link_normal=cp["normal"], target=tgt, control_kind=S.CTRL_FORCE_NODAL))
    ctrls.append(I.grf(64, 39, cp["dx"], 0.05, 0.2, 9, comps=2) * cp["active"])
    cp = I.clamped_plate(40, 25)
    tgt = 1e-4 * np.stack([cp["X"], cp["Y"]]) * cp["active"]
    probs.append(dict(nx=40, ny=25, dx=cp["dx"], E=1.0, nu=0.3, domain=S.MASKED,
                      node_mask=cp["active"].astype(np.uint8), link_bc=cp["bc"], link_wall=cp["wall"],
                      link_normal=cp["normal"], target=tgt, control_kind=S.CTRL_E_NODAL))
    ctrls.append(1.0 + 0.3 * np.tanh(I.grf(40, 25, cp["dx"], 1.0, 0.3, 12)[0]))
    for p in probs:
        p.update(tol=1e-10, max_steps=2_000_000)
    return probs, ctrls


def second_batch(S):
    """Smaller: one small periodic instance and one small plate."""
    n = 40
    probs = [dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=0, target=I.two_mode_target(n),
                  control_kind=S.CTRL_FORCE_MODES, n_modes=2, force_modes=I.two_mode_basis(n))]
    ctrls = [np.array([0.1, 0.1])]
    cp = I.clamped_plate(32, 20)
    tgt = I.grf(32, 20, cp["dx"], 1e-8, 0.3, 3, comps=2) * cp["active"]
    probs.append(dict(nx=32, ny=20, dx=cp["dx"], E=1.0, nu=0.3, domain=S.MASKED,
                      node_mask=cp["active"].astype(np.uint8), link_bc=cp["bc"], link_wall=cp["wall"],
                      link_normal=cp["normal"], target=tgt, control_kind=S.CTRL_FORCE_NODAL))
    ctrls.append(I.grf(32, 20, cp["dx"], 0.05, 0.2, 6, comps=2) * cp["active"])
    for p in probs:
        p.update(tol=1e-10, max_steps=2_000_000)
    return probs, ctrls


def same(r0, r1):
    rc0, J0, g0, p0, a0 = r0
    rc1, J1, g1, p1, a1 = r1
    assert rc0 == rc1 == 0
    assert np.array_equal(J0, J1)
    for x, y in zip(g0, g1):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    assert [p.steps for p in p0] == [p.steps for p in p1]
    assert [a.steps for a in a0] == [a.steps for a in a1]


def test_no_alloc_batch_matches_the_allocating_entry_point_on_two_calls(S):
    probs, ctrls = first_batch(S)
    b = S.solid_lbm_batch_init(probs)
    print("no-alloc: first batch (4 instances), static tables", flush=True)
    got = S.batch_objective_and_grad_noalloc(b, ctrls)
    ref = S.batch_objective_and_grad(b, ctrls)
    same(ref, got)
    S.solid_lbm_batch_destroy(b)
    # a second, smaller call: fewer work-list entries than the first left in the table
    probs, ctrls = second_batch(S)
    b = S.solid_lbm_batch_init(probs)
    print("no-alloc: second batch (2 instances)", flush=True)
    got = S.batch_objective_and_grad_noalloc(b, ctrls)
    ref = S.batch_objective_and_grad(b, ctrls)
    same(ref, got)
    # and again after the allocating call on the same batch
    same(ref, S.batch_objective_and_grad_noalloc(b, ctrls))
    S.solid_lbm_batch_destroy(b)


def test_no_alloc_batch_refuses_work_lists_beyond_the_static_table(S):
    """15 periodic 1024^2 instances with 2 steps and 4 rows per launch need
    15 x 18 x 256 = 69120 strip entries > 65536: refused before any work."""
    n = 1024
    probs = [dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=0, target=I.two_mode_target(n),
                  control_kind=S.CTRL_FORCE_MODES, n_modes=2, force_modes=I.two_mode_basis(n),
                  tol=0.0, max_steps=4) for _ in range(15)]
    b = S.solid_lbm_batch_init(probs)
    S.solid_lbm_batch_set_tuning(b, 2, 4)
    ctrls = [np.array([0.1, 0.1])] * 15
    print("no-alloc: oversized work-lists", flush=True)
    with pytest.raises(S.SlbmError) as e:
        S.batch_objective_and_grad_noalloc(b, ctrls, want_grad=False)
    assert e.value.code == S.EINVAL and "69120" in str(e.value) and "65536" in str(e.value)
    # default shape (8 steps per launch) fits: 15 x 22 x 43 = 14190 entries
    S.solid_lbm_batch_set_tuning(b, -1, 0)
    rc, J, _, pi, _ = S.batch_objective_and_grad_noalloc(b, ctrls, want_grad=False)
    rc2, J2, _, _, _ = S.batch_objective_and_grad(b, ctrls, want_grad=False)
    assert rc == rc2 == 0 and np.array_equal(J, J2) and all(p.steps == 4 for p in pi)
    S.solid_lbm_batch_destroy(b)
