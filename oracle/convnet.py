"""CPU reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

3x3 convolutions with zero padding, their weight and input gradients, ReLU and
a masked mean-squared error, written from their definitions in float64
(explicit loops over the nine taps with numpy slicing).  `bf16` rounds to
bfloat16 (round to nearest even) so the reference can use exactly the operands
the GPU kernels multiply.
"""
import numpy as np


def bf16(x):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _shift(x, dy, dx):
    """x[..., y + dy, x + dx] with zeros outside the image."""
    H, W = x.shape[-2:]
    out = np.zeros_like(x)
    ys, yd = (slice(dy, H), slice(0, H - dy)) if dy >= 0 else (slice(0, H + dy), slice(-dy, H))
    xs, xd = (slice(dx, W), slice(0, W - dx)) if dx >= 0 else (slice(0, W + dx), slice(-dx, W))
    out[..., yd, xd] = x[..., ys, xs]
    return out


def conv3x3(x, w, b=None, dil=1):
    """y[b, co] = b[co] + sum_{ci, ky, kx} w[co, ci, ky, kx] x[b, ci, y + dil (ky - 1), x + dil (kx - 1)]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    y = np.zeros((x.shape[0], w.shape[0]) + x.shape[2:])
    for ky in range(3):
        for kx in range(3):
            xs = _shift(x, dil * (ky - 1), dil * (kx - 1))
            y += np.einsum("oc,bchw->bohw", w[:, :, ky, kx], xs)
    if b is not None:
        y += np.asarray(b, np.float64)[None, :, None, None]
    return y


def conv3x3_grad_w(dz, x, dil=1):
    """dw[co, ci, ky, kx] = sum_{b, y, x} dz[b, co, y, x] x[b, ci, y + dil (ky - 1), x + dil (kx - 1)]."""
    dz = np.asarray(dz, np.float64)
    x = np.asarray(x, np.float64)
    dw = np.zeros((dz.shape[1], x.shape[1], 3, 3))
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.einsum("bohw,bchw->oc", dz, _shift(x, dil * (ky - 1), dil * (kx - 1)))
    return dw, dz.sum((0, 2, 3))


def conv3x3_grad_x(dz, w, dil=1):
    """dx[b, ci, y, x] = sum_{co, ky, kx} w[co, ci, ky, kx] dz[b, co, y - dil (ky - 1), x - dil (kx - 1)]."""
    dz = np.asarray(dz, np.float64)
    w = np.asarray(w, np.float64)
    dx = np.zeros((dz.shape[0], w.shape[1]) + dz.shape[2:])
    for ky in range(3):
        for kx in range(3):
            dx += np.einsum("oc,bohw->bchw", w[:, :, ky, kx], _shift(dz, dil * (1 - ky), dil * (1 - kx)))
    return dx


def mse(y, t, mask):
    """sum mask (y - t)^2 / (channels * sum mask) and its gradient."""
    nc = y.shape[1]
    norm = nc * mask.sum()
    d = (y - t) * mask[:, None]
    return float((d * (y - t)).sum() / norm), 2.0 * d / norm


def net_forward_backward(x, layers, t, mask):
    """Forward + backward of a stack of (w, b, relu, dilation) layers with the GPU's
    rounding points: inputs and activations fed to a convolution are rounded
    to bf16, weights are bf16, sums are exact (float64); the data gradient
    entering each convolution is rounded to bf16.  Returns (loss, grads, y)."""
    acts = [bf16(x)]
    outs = []
    for w, b, relu, dil in layers:
        y = conv3x3(acts[-1], bf16(w), b, dil)
        if relu:
            y = np.maximum(y, 0.0)
        outs.append(y)
        acts.append(bf16(y.astype(np.float32)))
    loss, dy = mse(outs[-1], t, mask)
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        w, b, relu, dil = layers[i]
        dz = dy * (outs[i] > 0) if relu else dy
        grads[i] = conv3x3_grad_w(dz, acts[i], dil)
        if i > 0:
            dy = conv3x3_grad_x(bf16(dz.astype(np.float32)), bf16(w), dil)
    return loss, grads, outs[-1]
