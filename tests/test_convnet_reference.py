"""Pins of the CPU reference of the warm-start network: the convolution is a
library correlation, the gradients are finite differences of the forward."""
import numpy as np
import pytest
from scipy import signal

from oracle import convnet as C


def test_dilated_conv_is_a_correlation_with_a_spread_kernel():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((1, 2, 9, 11))
    w = rng.standard_normal((3, 2, 3, 3))
    y = C.conv3x3(x, w, dil=2)
    for co in range(3):
        ref = 0
        for ci in range(2):
            k = np.zeros((5, 5))
            k[::2, ::2] = w[co, ci]
            ref = ref + signal.correlate2d(x[0, ci], k, mode="same", boundary="fill")
        assert np.abs(y[0, co] - ref).max() < 1e-12


def test_conv3x3_is_a_zero_padded_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 7, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = C.conv3x3(x, w, b)
    for bb in range(2):
        for co in range(4):
            ref = b[co] + sum(signal.correlate2d(x[bb, ci], w[co, ci], mode="same", boundary="fill")
                              for ci in range(3))
            assert np.abs(y[bb, co] - ref).max() < 1e-12


@pytest.mark.parametrize("dil", [1, 2])
def test_conv_gradients_match_finite_differences(dil):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 5, 6))
    w = rng.standard_normal((2, 3, 3, 3))
    dz = rng.standard_normal((2, 2, 5, 6))
    f = lambda x_, w_: float((C.conv3x3(x_, w_, dil=dil) * dz).sum())
    dw, db = C.conv3x3_grad_w(dz, x, dil)
    dx = C.conv3x3_grad_x(dz, w, dil)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 2, 2, 1), (0, 1, 1, 2)]:
        e = np.zeros_like(w)
        e[idx] = h
        assert abs((f(x, w + e) - f(x, w - e)) / (2 * h) - dw[idx]) < 1e-7
    for idx in [(0, 0, 0, 0), (1, 2, 4, 5), (0, 1, 2, 3)]:
        e = np.zeros_like(x)
        e[idx] = h
        assert abs((f(x + e, w) - f(x - e, w)) / (2 * h) - dx[idx]) < 1e-7
    assert np.allclose(db, dz.sum((0, 2, 3)))


def test_bf16_rounding_is_nearest_even():
    """bfloat16 keeps 8 significant bits: spacing 2^-7 just above 1."""
    u = 2.0 ** -7
    x = np.array([1.0, 1.0 + u / 2, 1.0 + 3 * u / 2, 1.0 + 0.75 * u, 1.0 + 0.25 * u, -2.5], dtype=np.float32)
    r = C.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                  # tie between 1 and 1 + u: even mantissa (1.0)
    assert r[2] == np.float32(1.0 + 2 * u)   # tie between 1 + u and 1 + 2u: even (1 + 2u)
    assert r[3] == np.float32(1.0 + u)
    assert r[4] == 1.0
    assert r[5] == -2.5


def test_network_forward_backward_equals_autograd_when_every_rounding_is_exact():
    """With inputs, weights, activations and the back-propagated data gradient
    all exactly representable in bfloat16 (small integers and a power-of-two
    normalisation), the reference's bf16 rounding points change nothing, so its
    loss and weight gradients must equal torch autograd of the same network in
    float64 (zero-padded dilated correlation, ReLU, masked mean squared error)."""
    import torch
    import torch.nn.functional as F
    rng = np.random.default_rng(5)
    B, H, W = 2, 6, 7
    x = rng.integers(0, 2, (B, 2, H, W)).astype(np.float64)
    w1 = rng.integers(-1, 2, (3, 2, 3, 3)).astype(np.float64)
    b1 = np.array([1.0, 0.0, 2.0])
    w2 = rng.integers(-1, 2, (2, 3, 3, 3)).astype(np.float64)
    b2 = np.array([0.0, 1.0])
    mask = np.zeros(B * H * W)
    mask[rng.choice(B * H * W, 16, replace=False)] = 1.0      # 2 channels x 16 nodes: norm 32
    mask = mask.reshape(B, H, W)
    # target = output + small integer offsets, so every y - t is a small integer
    y_ref = C.conv3x3(np.maximum(C.conv3x3(x, w1, b1, 1), 0.0), w2, b2, 2)
    t = y_ref + rng.integers(-2, 3, y_ref.shape)
    loss, grads, y = C.net_forward_backward(x.astype(np.float32), [(w1, b1, True, 1), (w2, b2, False, 2)], t, mask)

    tt = lambda a, g=False: torch.tensor(a, dtype=torch.float64, requires_grad=g)
    W1, B1, W2, B2 = tt(w1, True), tt(b1, True), tt(w2, True), tt(b2, True)
    y2 = F.conv2d(F.relu(F.conv2d(tt(x), W1, B1, padding=1)), W2, B2, padding=2, dilation=2)
    m = tt(mask)[:, None]
    L = (m * (y2 - tt(t)) ** 2).sum() / (2 * m.sum())
    L.backward()
    assert np.abs(y - y2.detach().numpy()).max() == 0.0
    assert abs(loss - L.item()) <= 1e-15 * abs(L.item())
    for (dw, db), Wt, Bt in zip(grads, (W1, W2), (B1, B2)):
        assert np.abs(dw - Wt.grad.numpy()).max() < 1e-12
        assert np.abs(db - Bt.grad.numpy()).max() < 1e-12
    assert np.abs(grads[0][0]).max() > 0.0                    # the first layer's gradient went through both layers
