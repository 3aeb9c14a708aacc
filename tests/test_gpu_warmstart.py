"""Warm-start network on the GPU (needs a GPU): MFMA convolution forward and
backward against the CPU reference, whole-network gradients against the CPU
reference, and a trained network that cuts primal steps without changing the
converged result."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_31347_amd import warmstart
    return warmstart


def relnorm(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("Cin,Cout,H,Wd,relu,dil", [(4, 32, 7, 45, 1, 1), (32, 32, 5, 13, 1, 2), (32, 2, 9, 33, 0, 1),
                                                   (3, 5, 1, 70, 1, 1), (32, 32, 12, 40, 1, 8)])
def test_conv_kernels_match_reference(W, Cin, Cout, H, Wd, relu, dil):
    import torch
    from oracle import convnet as C
    rng = np.random.default_rng(Cin * 100 + Cout)
    B = 2
    x = rng.standard_normal((B, Cin, H, Wd)).astype(np.float32)
    w = (rng.standard_normal((Cout, Cin, 3, 3)) * 0.3).astype(np.float32)
    b = rng.standard_normal(Cout).astype(np.float32)
    xg = W.to_bf16(torch.from_numpy(x).cuda())
    w32 = torch.from_numpy(w.reshape(Cout, Cin * 9)).cuda()
    wp = torch.zeros(32 * W._kp(Cin * 9), dtype=torch.bfloat16, device="cuda")
    wt = torch.zeros(32 * W._kp(Cout * 9), dtype=torch.bfloat16, device="cuda")
    W._chk(W._L.slbm_pack_weights(W._p(w32), W._p(wp), W._p(wt), Cin, Cout, W._stream()), "pack")
    y = torch.empty((B, Cout, H, Wd), dtype=torch.float32, device="cuda")
    W._chk(W._L.slbm_conv3x3_forward(W._p(xg), W._p(wp), W._p(torch.from_numpy(b).cuda()), W._p(y), None, B, Cin,
                                     Cout, H, Wd, relu, dil, W._stream()), "fwd")
    ref = C.conv3x3(C.bf16(x), C.bf16(w), b, dil)
    if relu:
        ref = np.maximum(ref, 0)
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max()
    # weight gradient (FP32 dz, bf16 x) and data gradient (bf16 dz, flipped weights)
    dz = rng.standard_normal((B, Cout, H, Wd)).astype(np.float32)
    gw = torch.empty((Cout, Cin * 9), dtype=torch.float32, device="cuda")
    gb = torch.empty(Cout, dtype=torch.float32, device="cuda")
    dzg = torch.from_numpy(dz).cuda()
    W._chk(W._L.slbm_conv3x3_backward_weight(W._p(dzg), W._p(xg), W._p(gw), W._p(gb), B, Cin, Cout, H, Wd, dil,
                                             W._stream()), "bww")
    rw, rb = C.conv3x3_grad_w(dz, C.bf16(x), dil)
    assert np.abs(gw.cpu().numpy().reshape(rw.shape) - rw).max() <= 1e-5 * np.abs(rw).max()
    assert np.abs(gb.cpu().numpy() - rb).max() <= 1e-5 * np.abs(rb).max()
    dx = torch.empty((B, Cin, H, Wd), dtype=torch.float32, device="cuda")
    W._chk(W._L.slbm_conv3x3_forward(W._p(W.to_bf16(dzg)), W._p(wt), None, W._p(dx), None, B, Cout, Cin, H, Wd, 0,
                                     dil, W._stream()), "bwd data")
    rx = C.conv3x3_grad_x(C.bf16(dz), C.bf16(w), dil)
    assert np.abs(dx.cpu().numpy() - rx).max() <= 1e-5 * np.abs(rx).max()


def test_network_gradients_match_reference(W):
    import torch
    from oracle import convnet as C
    net = W.ConvNet(seed=3)
    rng = np.random.default_rng(7)
    B, H, Wd = 3, 11, 37
    x = rng.standard_normal((B, net.layers[0][0], H, Wd)).astype(np.float32)
    t = rng.standard_normal((B, 2, H, Wd)).astype(np.float32) * 0.1
    mask = (rng.random((B, H, Wd)) > 0.3).astype(np.float32)
    # make the last layer non-trivial
    net.w[-1].mul_(10.0)
    net.pack()
    y = net.forward(W.to_bf16(torch.from_numpy(x).cuda()))
    loss, dy = W.mse(y, torch.from_numpy(t).cuda(), torch.from_numpy(mask).cuda())
    net.backward(dy)
    layers = [(w.cpu().numpy().reshape(co, ci, 3, 3), b.cpu().numpy(), relu, dil)
              for (ci, co, relu, dil), w, b in zip(net.layers, net.w, net.b)]
    rl, rg, ry = C.net_forward_backward(x, layers, t, mask)
    # Both sides round every activation to bf16.  The GPU's FP32 sums of 288
    # products and the reference's FP64 sums differ by ~1e-6 relative, so a
    # few activations in 1e4 land on opposite sides of a bf16 rounding boundary
    # (spacing ~4e-3) and differ by one bf16 ulp; those flips reach the output
    # through the later layers at ~1e-4 relative (the per-layer tests above
    # check each kernel to 1e-5 on identical bf16 inputs).
    assert relnorm(y.cpu().numpy(), ry) < 2e-3
    assert abs(loss.item() - rl) <= 2e-3 * rl
    for i, ((gw, gb), w) in enumerate(zip(rg, net.gw)):
        assert relnorm(w.cpu().numpy().reshape(gw.shape), gw) < 2e-3, i
        assert relnorm(net.gb[i].cpu().numpy(), gb) < 2e-3, i


def test_trained_warm_start_cuts_steps_same_fixed_point(W):
    from paper_2609_31347_amd import slbm as S
    ws = W.WarmStart(nx_coarse=32, seed=0)
    ws.reference(tol=1e-10)
    X, Y, info = ws.make_data(256, seed0=0, tol=1e-9)
    hist = ws.train(X, Y, iters=600, batch=32, lr=1e-3)
    assert hist[-1]["loss"] < 0.5 * hist[0]["loss"], hist
    cold_steps, warm_steps = [], []
    for seed in (5001, 5002, 5003):
        E = W.e_field(ws.cp, seed)
        ctx = S.solid_lbm_init(W.plate_problem(ws.cp, 1e-10))
        rc, info = S.primal_solve(ctx, E)
        d_cold = S.solid_lbm_get_field(ctx, S.FIELD_DISP)
        d0 = ws.predict(ws.cp, E)
        rc, info2 = S.primal_solve(ctx, E, d0)
        d_warm = S.solid_lbm_get_field(ctx, S.FIELD_DISP)
        assert info.converged and info2.converged
        # both stop at a K-lag residual < 1e-10; for this plate the slowest mode
        # decays over ~4 pseudo-time units against the 0.01 window of the test,
        # so each is within ~4e-8 of the fixed point (the same for both starts)
        assert relnorm(d_warm, d_cold) < 1e-6
        cold_steps.append(info.steps)
        warm_steps.append(info2.steps)
    print("cold", cold_steps, "warm", warm_steps, "loss", hist[0]["loss"], hist[-1]["loss"], flush=True)
    assert np.mean(warm_steps) < 0.9 * np.mean(cold_steps), (cold_steps, warm_steps)


def test_warm_started_batched_gradients_take_less_wall_time(W):
    """Batched E-field identification gradients (primal and adjoint to 1e-10)
    on the 64 x 39 plate: the trained network's initial displacements give the
    same J and gradients as cold starts, in fewer primal steps and in less
    wall time including the prediction (the cold start fixes the reference result)."""
    import time
    import torch
    from paper_2609_31347_amd import slbm as S
    ws = W.WarmStart(nx_coarse=64, seed=0)
    ws.reference(tol=1e-10)
    X, Y, _ = ws.make_data(384, seed0=0, tol=1e-9)
    ws.train(X, Y, iters=800, batch=32, lr=1e-3)
    cp = ws.cp
    ctx = S.solid_lbm_init(W.plate_problem(cp, 1e-10))
    S.primal_solve(ctx, W.e_field(cp, 99999))
    target = S.solid_lbm_get_field(ctx, S.FIELD_DISP)
    fields = [W.e_field(cp, 7000 + k) for k in range(12)]
    cold, warm = [], []
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Jc, gc, pc, ac = W.batch_gradients(cp, fields, target, 1e-10)
        cold.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        d0s = ws.predict_batch(cp, fields)
        Jw, gw, pw, aw = W.batch_gradients(cp, fields, target, 1e-10, init_disps=d0s)
        warm.append(time.perf_counter() - t0)
    print("cold s", cold, "warm s", warm, "cold steps", [p.steps for p in pc], "warm steps",
          [p.steps for p in pw], flush=True)
    assert all(p.converged and a.converged for p, a in zip(pc + pw, ac + aw))
    for k in range(len(fields)):
        assert abs(Jw[k] - Jc[k]) <= 1e-5 * abs(Jc[k]), k
        assert relnorm(gw[k], gc[k]) < 1e-4, k
    assert np.mean([p.steps for p in pw]) < 0.9 * np.mean([p.steps for p in pc])
    assert max(p.steps for p in pw) < max(p.steps for p in pc)
    assert min(warm) < min(cold), (cold, warm)
