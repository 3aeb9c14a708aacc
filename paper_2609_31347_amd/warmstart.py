"""Learned warm start for the primal solve of the E-field identification on the
clamped elliptic plate.

The paper starts every primal solve from d_0 = 0.  Steps to a residual tol
grow like ln(e_0 / tol) / (1 - |lambda_slow|), so a better initial
displacement d_0 saves steps in proportion to ln(1 / e_0).  Here a small
convolutional network predicts d_0 from the modulus field E(x):

  input  (7 channels): u = 1/E - 1 on the plate, the plate mask, the
         displacement of the same plate with E = 1 (d_ref, 2 channels, scaled),
         and u averaged over 4 and 16 nodes and over the whole plate,
  output (2 channels): (d - d_ref) / s, s = max |d_ref|,
  6 layers of 3x3 convolutions (dilations 1, 2, 4, 8, 4, 1), 32 channels, ReLU
  between them, bf16 weights and activations with FP32 accumulation on
  gfx950's 32x32x16 bf16 MFMA (forward and data gradient) and the FP32 MFMA
  (weight gradient) in csrc/slbm_net.hip, trained with Adam by the same
  kernels.

It is trained on solver outputs at a coarse resolution (batched FP64 solves);
for a finer grid, E is sampled onto the coarse grid, the prediction is
interpolated back (bilinear, in physical coordinates) and passed as init_disp
to the FP64 solver, whose arithmetic and convergence test are unchanged: the
result is the same fixed point, only reached in fewer steps, and the cold
start remains the fallback.
"""
import ctypes
import time

import numpy as np
import torch

from . import inputs as I
from . import slbm as S

# (inputs, outputs, ReLU, dilation): six 3x3 layers, 32 channels; the dilations
# widen the receptive field to 41 nodes, since the displacement depends on E
# over the whole plate
LAYERS = ((7, 32, True, 1), (32, 32, True, 2), (32, 32, True, 4), (32, 32, True, 8), (32, 32, True, 4),
          (32, 2, False, 1))
NU = 0.3


def _kp(k):
    """K of the packed bf16 weights: rounded up to a 16-wide MFMA k-slice."""
    return (k + 15) // 16 * 16


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _chk(rc, what):
    if rc != 0:
        raise S.SlbmError(rc, what)


def _need(t, dtype, shape, what):
    """The kernels read whole [B][C][H][W] planes through the pointer: a tensor
    of another dtype, shape or layout, or on the host, would be misread."""
    if not torch.is_tensor(t) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{what}: needs a contiguous {dtype} CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: shape {tuple(t.shape)}, expected {tuple(shape)}")


_L = S.LIB
_P = ctypes.c_void_p
_i32, _i64, _f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
_L.slbm_conv3x3_forward.argtypes = [_P, _P, _P, _P, _P, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _P]
_L.slbm_conv3x3_backward_weight.argtypes = [_P, _P, _P, _P, _i32, _i32, _i32, _i32, _i32, _i32, _P]
_L.slbm_act_backward.argtypes = [_P, _P, _P, _P, _i64, _i32, _P]
_L.slbm_pack_weights.argtypes = [_P, _P, _P, _i32, _i32, _P]
_L.slbm_to_bf16.argtypes = [_P, _P, _i64, _P]
_L.slbm_mse.argtypes = [_P, _P, _P, _P, _P, _i32, _i32, _i64, _P]
_L.slbm_adam.argtypes = [_P, _P, _P, _P, _i64, _f32, _f32, _f32, _f32, _i32, _P]


def to_bf16(x):
    """FP32 tensor -> bf16 tensor by the library's rounding kernel (CUDA tensors)."""
    if not torch.is_tensor(x) or not x.is_cuda:
        raise TypeError("to_bf16: needs a CUDA tensor")
    x = x.contiguous().float()
    y = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    _chk(_L.slbm_to_bf16(_p(x), _p(y), x.numel(), _stream()), "to_bf16")
    return y


class ConvNet:
    """Weights in FP32 (Adam master copy) packed to bf16 for the MFMA kernels."""

    def __init__(self, seed=0, layers=LAYERS):
        g = torch.Generator().manual_seed(seed)
        self.layers = layers
        self.w, self.b, self.wp, self.wt, self.m, self.v = [], [], [], [], [], []
        for i, (ci, co, relu, dil) in enumerate(layers):
            std = (2.0 / (ci * 9)) ** 0.5 * (0.1 if i == len(layers) - 1 else 1.0)
            w = (torch.randn(co, ci * 9, generator=g) * std).float().cuda()
            b = torch.zeros(co, dtype=torch.float32, device="cuda")
            self.w.append(w)
            self.b.append(b)
            self.wp.append(torch.zeros(32 * _kp(ci * 9), dtype=torch.bfloat16, device="cuda"))
            self.wt.append(torch.zeros(32 * _kp(co * 9), dtype=torch.bfloat16, device="cuda"))
            self.m.append([torch.zeros_like(w), torch.zeros_like(b)])
            self.v.append([torch.zeros_like(w), torch.zeros_like(b)])
        self.t = 0
        self.pack()

    def pack(self):
        for (ci, co, _, _), w, wp, wt in zip(self.layers, self.w, self.wp, self.wt):
            _chk(_L.slbm_pack_weights(_p(w), _p(wp), _p(wt), ci, co, _stream()), "pack")

    def forward(self, xb):
        """xb: bf16 [B, 7, H, W] (the input channels of the first layer).
        Returns the FP32 output [B, 2, H, W]; keeps the activations."""
        B, _, H, W = xb.shape
        _need(xb, torch.bfloat16, (B, self.layers[0][0], H, W), "forward input")
        self.acts, self.outs = [xb], []
        for (ci, co, relu, dil), wp, b in zip(self.layers, self.wp, self.b):
            y = torch.empty((B, co, H, W), dtype=torch.float32, device="cuda")
            yb = torch.empty((B, co, H, W), dtype=torch.bfloat16, device="cuda")
            _chk(_L.slbm_conv3x3_forward(_p(self.acts[-1]), _p(wp), _p(b), _p(y), _p(yb), B, ci, co, H, W,
                                         int(relu), dil, _stream()), "conv forward")
            self.outs.append(y)
            self.acts.append(yb)
        return self.outs[-1]

    def backward(self, dy):
        """Gradients of the loss whose output gradient is dy (FP32 [B, 2, H, W]),
        after a forward of the same batch."""
        if not getattr(self, "acts", None):
            raise RuntimeError("backward needs a forward first")
        B, _, H, W = self.acts[0].shape
        _need(dy, torch.float32, (B, self.layers[-1][1], H, W), "output gradient")
        self.gw, self.gb = [None] * len(self.layers), [None] * len(self.layers)
        for i in range(len(self.layers) - 1, -1, -1):
            ci, co, relu, dil = self.layers[i]
            dz = torch.empty_like(dy)
            dzb = torch.empty(dy.shape, dtype=torch.bfloat16, device="cuda")
            _chk(_L.slbm_act_backward(_p(dy), _p(self.outs[i]), _p(dz), _p(dzb), dy.numel(), int(relu),
                                      _stream()), "act backward")
            gw = torch.empty((co, ci * 9), dtype=torch.float32, device="cuda")
            gb = torch.empty(co, dtype=torch.float32, device="cuda")
            _chk(_L.slbm_conv3x3_backward_weight(_p(dz), _p(self.acts[i]), _p(gw), _p(gb), B, ci, co, H, W, dil,
                                                 _stream()), "weight gradient")
            self.gw[i], self.gb[i] = gw, gb
            if i > 0:
                dx = torch.empty((B, ci, H, W), dtype=torch.float32, device="cuda")
                _chk(_L.slbm_conv3x3_forward(_p(dzb), _p(self.wt[i]), None, _p(dx), None, B, co, ci, H, W, 0, dil,
                                             _stream()), "data gradient")
                dy = dx
        return self.gw, self.gb

    def step(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        for i in range(len(self.layers)):
            for k, (p, g) in enumerate(((self.w[i], self.gw[i]), (self.b[i], self.gb[i]))):
                _chk(_L.slbm_adam(_p(p), _p(g), _p(self.m[i][k]), _p(self.v[i][k]), p.numel(), lr, b1, b2, eps,
                                  self.t, _stream()), "adam")
        self.pack()


def mse(y, t, mask):
    """Masked mean squared error of y against t (FP32 [B, nc, H, W]) over the
    nodes where mask (FP32 [B, H, W]) is non-zero; returns (loss, dloss/dy)."""
    B, nc, H, W = y.shape
    t, mask = t.contiguous(), mask.contiguous()
    _need(y, torch.float32, (B, nc, H, W), "mse prediction")
    _need(t, torch.float32, (B, nc, H, W), "mse target")
    _need(mask, torch.float32, (B, H, W), "mse mask")
    dy = torch.empty_like(y)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    _chk(_L.slbm_mse(_p(y), _p(t), _p(mask), _p(dy), _p(loss), B, nc, H * W, _stream()), "mse")
    return loss, dy


# ------------------------------------------------------------------ problem data

def plate(nx):
    """Clamped elliptic plate with ny = ceil(0.6 nx) nodes (semi-axes 1 x 0.6)."""
    return I.clamped_plate(nx, int(np.ceil(0.6 * nx)))


def e_field(cp, seed, var=1.0, ell=0.15):
    """E(x) = 1 + 0.5 tanh(GRF), squared-exponential GRF of length ell (physical)."""
    ny, nx = cp["active"].shape
    return 1.0 + 0.5 * np.tanh(I.grf(nx, ny, cp["dx"], var, ell, seed)[0])


def plate_problem(cp, tol, max_steps=50_000_000, target=None):
    ny, nx = cp["active"].shape
    t = np.zeros((2, ny, nx)) if target is None else target
    return dict(nx=nx, ny=ny, dx=cp["dx"], E=1.0, nu=NU, domain=S.MASKED, node_mask=cp["active"].astype(np.uint8),
                link_bc=cp["bc"], link_wall=cp["wall"], link_normal=cp["normal"], target=t,
                normalize_objective=0 if target is None else 1, control_kind=S.CTRL_E_NODAL, tol=tol,
                max_steps=max_steps)


def solve_batch(cp, fields, tol, chunk=96, progress=None):
    """Converged displacements of the plate for a list of E fields (batched FP64
    solves); progress(phase, step, residual) is reported every 30 s if given."""
    out, steps = [], []
    for k in range(0, len(fields), chunk):
        part = fields[k:k + chunk]
        batch = S.solid_lbm_batch_init([plate_problem(cp, tol) for _ in part])
        if progress:
            S.solid_lbm_batch_set_progress(batch, progress, 30.0)
        rc, J, _, pi, _ = S.batch_objective_and_grad(batch, list(part), want_grad=False)
        # training targets must be steady states
        S.require_converged(rc, "batched plate solves", next((x for x in pi if not x.converged), None))
        for c in batch.contexts:
            out.append(S.solid_lbm_get_field(c, S.FIELD_DISP))
        steps += [x.steps for x in pi]
        S.solid_lbm_batch_destroy(batch)
    return np.stack(out), np.array(steps)


BLURS = (4.0, 16.0)        # Gaussian widths (nodes) of the non-local input channels


def features(E, mask, dref, s):
    """Input channels: the compliance perturbation u = 1/E - 1 on the plate, the
    plate mask, d_ref / s (2), u averaged over the plate with Gaussian weights
    of width 4 and 16 nodes (normalised convolution inside the plate), and the
    plate mean of u.  The displacement change is a global response to the
    local source u; the averages hand the 41-node receptive field information
    from farther away."""
    from scipy import ndimage
    m = mask.astype(np.float64)
    u = (1.0 / E - 1.0) * m
    ch = [u, m, dref[0] / s, dref[1] / s]
    for sig in BLURS:
        num = ndimage.gaussian_filter(u, sig, mode="constant")
        den = ndimage.gaussian_filter(m, sig, mode="constant")
        ch.append(num / np.maximum(den, 1e-12) * m)
    ch.append(np.full_like(u, u[m > 0].mean() if m.any() else 0.0) * m)
    return np.stack(ch).astype(np.float32)


# ------------------------------------------------------------------ training

class WarmStart:
    """A trained network for one coarse plate resolution."""

    def __init__(self, nx_coarse=64, seed=0):
        self.cp = plate(nx_coarse)
        self.net = ConvNet(seed)
        self.history = []

    def reference(self, tol=1e-10):
        d, st = solve_batch(self.cp, [np.ones_like(self.cp["active"], dtype=np.float64)], tol)
        self.dref = d[0]
        self.s = float(np.abs(self.dref).max())
        return st[0]

    def make_data(self, n, seed0=0, tol=1e-8):
        fields = [e_field(self.cp, seed0 + i) for i in range(n)]
        t0 = time.perf_counter()
        d, steps = solve_batch(self.cp, fields, tol)
        m = self.cp["active"]
        X = np.stack([features(E, m, self.dref, self.s) for E in fields])
        Y = ((d - self.dref[None]) / self.s * m).astype(np.float32)
        return X, Y, dict(solves=n, wall_s=time.perf_counter() - t0, mean_steps=float(steps.mean()))

    def train(self, X, Y, iters=2000, batch=32, lr=5e-4, seed=0, log_every=200, log=None, Xv=None, Yv=None):
        rng = np.random.Generator(np.random.PCG64(seed))
        Xg = torch.from_numpy(X).cuda()
        Yg = torch.from_numpy(Y).cuda()
        mask = torch.from_numpy(self.cp["active"].astype(np.float32)).cuda()
        t0 = time.perf_counter()
        for it in range(iters):
            idx = torch.from_numpy(rng.integers(0, len(X), batch)).cuda()
            xb = to_bf16(Xg[idx])
            y = self.net.forward(xb)
            loss, dy = mse(y, Yg[idx], mask[None].expand(batch, -1, -1).contiguous())
            self.net.backward(dy)
            lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * it / iters))
            self.net.step(lr_t)
            if it % log_every == 0 or it == iters - 1:
                rec = dict(it=it, loss=float(loss.item()), wall_s=round(time.perf_counter() - t0, 2))
                if Xv is not None:
                    rec["val_loss"] = self.evaluate(Xv, Yv)
                self.history.append(rec)
                if log:
                    log(rec)
        return self.history

    def evaluate(self, X, Y, batch=64):
        """Mean masked MSE of the network on (X, Y)."""
        mask = torch.from_numpy(self.cp["active"].astype(np.float32)).cuda()
        tot, n = 0.0, 0
        for k in range(0, len(X), batch):
            xb = to_bf16(torch.from_numpy(X[k:k + batch]).cuda())
            y = self.net.forward(xb)
            loss, _ = mse(y, torch.from_numpy(Y[k:k + batch]).cuda(), mask[None].expand(len(xb), -1, -1).contiguous())
            tot += float(loss.item()) * len(xb)
            n += len(xb)
        return tot / n

    def predict_coarse(self, E_coarse, use_net=True):
        if not use_net:                       # ablation: the E = 1 displacement alone
            return self.dref * self.cp["active"]
        x = torch.from_numpy(features(E_coarse, self.cp["active"], self.dref, self.s)[None]).cuda()
        y = self.net.forward(to_bf16(x))
        return self.dref + self.s * y[0].double().cpu().numpy() * self.cp["active"]

    def predict(self, cp_fine, E_fine, use_net=True):
        """Initial displacement for a plate of any resolution (same geometry)."""
        if cp_fine["active"].shape == self.cp["active"].shape:
            return self.predict_coarse(E_fine, use_net) * cp_fine["active"]
        Ec = _resample(E_fine, cp_fine, self.cp, fill_outside=False)
        dc = self.predict_coarse(Ec, use_net)
        return self.to_fine(dc, cp_fine)

    def to_fine(self, dc, cp_fine):
        """A displacement on the coarse plate, interpolated onto cp_fine."""
        if cp_fine["active"].shape == self.cp["active"].shape:
            return dc * cp_fine["active"]
        return np.stack([_resample(dc[c], self.cp, cp_fine, fill_outside=True) for c in range(2)]) * cp_fine["active"]

    def predict_batch(self, cp_fine, fields):
        """predict() for many E fields with one network forward pass."""
        m = self.cp["active"]
        same = cp_fine["active"].shape == m.shape
        Ec = [E if same else _resample(E, cp_fine, self.cp, fill_outside=False) for E in fields]
        x = torch.from_numpy(np.stack([features(E, m, self.dref, self.s) for E in Ec])).cuda()
        y = self.net.forward(to_bf16(x)).double().cpu().numpy()
        return [self.to_fine(self.dref + self.s * y[k] * m, cp_fine) for k in range(len(fields))]


def batch_gradients(cp, fields, target, tol, init_disps=None, max_steps=50_000_000, progress=None):
    """E-field identification gradients of many fields on one plate in one
    batch: J and dJ/dE per field, primal started cold or from init_disps;
    progress(phase, step, residual) is reported every 30 s if given.
    Returns (J, grads, primal infos, adjoint infos)."""
    probs = [plate_problem(cp, tol, max_steps=max_steps, target=target) for _ in fields]
    batch = S.solid_lbm_batch_init(probs)
    if progress:
        S.solid_lbm_batch_set_progress(batch, progress, 30.0)
    rc, J, grads, pi, ai = S.batch_objective_and_grad(batch, list(fields), init_disps=init_disps)
    S.require_converged(rc, "batched E-field gradients")
    S.solid_lbm_batch_destroy(batch)
    return J, grads, pi, ai


def _resample(f, src, dst, fill_outside):
    """Bilinear resampling of a nodal field between two plate grids of the
    same geometry (both centred on the ellipse), in physical coordinates.
    fill_outside: first extend the field from the plate to its surroundings
    by nearest plate values so the interpolation near the rim sees no zeros."""
    from scipy import ndimage
    g = np.asarray(f, dtype=np.float64)
    if fill_outside:
        _, ind = ndimage.distance_transform_edt(~src["active"], return_indices=True)
        g = g[ind[0], ind[1]]
    ny_s, nx_s = src["active"].shape
    ny_d, nx_d = dst["active"].shape
    xs = (np.arange(nx_d) - 0.5 * (nx_d - 1)) * dst["dx"] / src["dx"] + 0.5 * (nx_s - 1)
    ys = (np.arange(ny_d) - 0.5 * (ny_d - 1)) * dst["dx"] / src["dx"] + 0.5 * (ny_s - 1)
    Yd, Xd = np.meshgrid(ys, xs, indexing="ij")
    return ndimage.map_coordinates(g, [Yd, Xd], order=1, mode="nearest")
