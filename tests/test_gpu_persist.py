"""The persistent, graph-captured batch path (solid_lbm_batch_set_persistent)
against the host-driven batch launches, individual solves and the oracle
(needs a GPU).

The persistent kernel runs every instance as LDS tiles with its own step
counter and check schedule; a small round budget per launch makes each solve
half replay the captured graph many times (with the host's synchronisation
and status read between replays), so every replay's result feeds the next
and the final states are compared with the eager (host-driven) path.
"""
import numpy as np
import pytest

from test_gpu_batch import mixed_problems

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_31347_amd import slbm
    return slbm


def test_persistent_batch_equals_host_driven_individual_and_oracle(S, orc):
    probs, ctrls = mixed_problems(S)
    host = S.solid_lbm_batch_init(probs)
    rc, J, grads, pi, ai = S.batch_objective_and_grad(host, ctrls)
    assert rc == 0
    pers = S.solid_lbm_batch_init(probs)
    S.solid_lbm_batch_set_persistent(pers, True, 50)
    print("persistent batch: 8 instances, 50 rounds per graph replay", flush=True)
    rcp, Jp, gp, pip, aip = S.batch_objective_and_grad(pers, ctrls)
    launches, rounds = S.solid_lbm_batch_persistent_stats(pers)
    assert rcp == 0 and all(x.converged for x in pip) and all(x.converged for x in aip)
    assert launches > 3 and rounds > 150                 # the adjoint half replayed the graph many times
    for i in range(len(probs)):
        assert pip[i].steps == pi[i].steps and aip[i].steps == ai[i].steps, i
        assert abs(Jp[i] - J[i]) <= 1e-13 * abs(J[i]), i
        assert rel(gp[i], grads[i]) <= 1e-12, i
    # individual solves
    for i in (0, 3, 6):
        ctx = S.solid_lbm_init(probs[i])
        rci, Ji, gi, pii, aii = S.objective_and_grad(ctx, ctrls[i])
        assert pii.steps == pip[i].steps and aii.steps == aip[i].steps, i
        assert abs(Jp[i] - Ji) <= 1e-13 * abs(Ji) and rel(gp[i], gi) < 1e-12, i
    # the oracle on four instance kinds: periodic modes, periodic nodal force,
    # plate nodal force, E = alpha^2 on the torus
    n = 32
    q = orc.Problem(n, n, 1 / n, 1.0, 0.3, np.zeros((2, n, n)))
    G = orc.objective_and_grad(q, probs[0]["target"], "modes", ctrls[0], modes=probs[0]["force_modes"], tol=1e-10)
    assert G.prim.steps == pip[0].steps and abs(Jp[0] - G.J) / G.J < 1e-12 and rel(gp[0], G.grad) < 1e-10
    p = probs[1]
    q = orc.Problem(p["nx"], p["ny"], p["dx"], p["E"], p["nu"], np.zeros((2, p["ny"], p["nx"])))
    G = orc.objective_and_grad(q, p["target"], "nodal", ctrls[1], tol=1e-10)
    assert G.prim.steps == pip[1].steps and abs(Jp[1] - G.J) / G.J < 1e-12
    assert rel(np.asarray(gp[1]).reshape(G.grad.shape), G.grad) < 1e-10
    p = probs[3]
    q = orc.Problem(p["nx"], p["ny"], p["dx"], 0.1, 0.7, np.zeros((2, p["ny"], p["nx"])), active=p["node_mask"],
                    bc=p["link_bc"], wall=p["link_wall"], normal=p["link_normal"])
    G = orc.objective_and_grad(q, p["target"], "nodal", ctrls[3], tol=1e-10, project=False)
    assert G.prim.steps == pip[3].steps and abs(Jp[3] - G.J) / G.J < 1e-12
    assert rel(np.asarray(gp[3]).reshape(G.grad.shape), G.grad) < 1e-10
    p = probs[5]
    q = orc.Problem(p["nx"], p["ny"], p["dx"], 0.11, 0.8, np.zeros((2, p["ny"], p["nx"])))
    G = orc.objective_and_grad(q, p["target"], "E_sq", ctrls[5], fixed_force=p["fixed_force"], tol=1e-10)
    assert G.prim.steps == pip[5].steps and abs(Jp[5] - G.J) / G.J < 1e-12 and rel(gp[5], G.grad) < 1e-10


def test_persistent_batch_fixed_steps_and_replay_budgets(S):
    """tol <= 0: exactly max_steps steps per instance; the rounds per replay and
    the steps per tile do not change any result."""
    probs, ctrls = mixed_problems(S, tol=0.0, large=False)
    for p in probs:
        p["max_steps"] = 333
    host = S.solid_lbm_batch_init(probs)
    rc, J, grads, pi, ai = S.batch_objective_and_grad(host, ctrls)
    for budget, Tt in ((7, -1), (0, 3), (0, 8)):
        b = S.solid_lbm_batch_init(probs)
        S.solid_lbm_batch_set_persistent(b, True, budget)
        S.solid_lbm_batch_set_tile_steps(b, Tt)
        rcp, Jp, gp, pip, aip = S.batch_objective_and_grad(b, ctrls)
        assert all(x.steps == 333 for x in pip) and all(x.steps == 333 for x in aip)
        assert rel(Jp, J) <= 1e-13
        for g, g0 in zip(gp, grads):
            assert rel(g, g0) <= 1e-12
