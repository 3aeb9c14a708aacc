"""Differentiation of the steady solid-LBM solution map with torch.autograd.

`displacement(control, solver)` returns the converged, two-step-averaged
displacement d(control) (2, ny, nx) as a CUDA float64 tensor; its backward is
the discrete adjoint (Algorithm "ALBM", eq. optimality) run by the HIP library
with the incoming gradient as the adjoint source (`adjoint_solve_vjp`).  Any
loss written in torch on d therefore gets its control gradient from one
adjoint solve, whatever the dimension of the control.

The adjoint needs the converged primal state.  The solver context holds one
state; if another forward ran on the same solver before this backward, the
state is brought back either from a checkpoint of the averaged populations
saved in forward (mode "checkpoint": 8 planes kept on the GPU) or by solving
the primal again warm-started from the saved displacement (mode "recompute":
2 planes kept, one extra primal solve).
"""
import numpy as np
import torch

from . import slbm as S

MODES = ("checkpoint", "recompute")


class Solver:
    """One problem on the current GPU (owns the library context).

    strict (default True): a primal or adjoint solve that stops at max_steps
    before reaching tol raises slbm.NotConverged instead of handing a
    non-steady displacement or gradient to autograd."""

    def __init__(self, problem, tune=True, tune_control=None, strict=True):
        self.strict = bool(strict)
        self.problem = dict(problem)
        self.problem.setdefault("stream", torch.cuda.current_stream().cuda_stream)
        self.ctx = S.solid_lbm_init(self.problem)
        self.nx, self.ny = int(problem["nx"]), int(problem["ny"])
        self.kind = int(problem.get("control_kind", S.CTRL_FORCE_MODES))
        self.solve_id = 0
        self.last_info = None
        self.last_adjoint_info = None
        if tune and tune_control is not None:
            from .autotune import autotune
            autotune(self.ctx, self.problem, tune_control)

    def _dev(self, a):
        t = torch.as_tensor(a, dtype=torch.float64)
        return t.to("cuda").contiguous()

    def solve(self, control, init_disp=None):
        c = self._dev(control)
        d0 = None if init_disp is None else self._dev(init_disp)
        rc, info = S.primal_solve(self.ctx, c, d0)
        self.solve_id += 1
        self.last_info = info
        if self.strict:
            S.require_converged(rc, "primal solve", info)
        d = torch.empty((2, self.ny, self.nx), dtype=torch.float64, device="cuda")
        S.solid_lbm_get_field(self.ctx, S.FIELD_DISP, d)
        return d

    def checkpoint(self):
        pops = torch.empty((8, self.ny, self.nx), dtype=torch.float64, device="cuda")
        S.solid_lbm_get_field(self.ctx, S.FIELD_AVG_POPS, pops)
        return pops

    def restore(self, control, pops):
        S.solid_lbm_restore_solve(self.ctx, self._dev(control), pops.contiguous())
        self.solve_id += 1

    def vjp(self, d_cot, grad_shape):
        g = torch.empty(self.ctx.grad_len(), dtype=torch.float64, device="cuda")
        rc, g, info = S.adjoint_solve_vjp(self.ctx, d_cot.detach().to(torch.float64).contiguous(), g)
        self.last_adjoint_info = info
        if self.strict:
            S.require_converged(rc, "adjoint solve", info)
        return g.reshape(grad_shape)

    def objective(self):
        """J of eq. discrete_J for the last solve (the problem's target and normalisation)."""
        return S.solid_lbm_objective(self.ctx)


class _Displacement(torch.autograd.Function):
    @staticmethod
    def forward(fctx, control, solver, mode):
        if mode not in MODES:
            raise ValueError(f"mode must be one of {MODES}")
        c = control.detach().to(torch.float64).contiguous()
        d = solver.solve(c)
        fctx.solver, fctx.mode, fctx.sid, fctx.shape = solver, mode, solver.solve_id, tuple(control.shape)
        fctx.cdev, fctx.cdtype = control.device, control.dtype
        saved = solver.checkpoint() if mode == "checkpoint" else d.detach().clone()
        fctx.save_for_backward(c, saved)
        return d

    @staticmethod
    def backward(fctx, grad_d):
        solver = fctx.solver
        c, saved = fctx.saved_tensors
        if solver.solve_id != fctx.sid:
            if fctx.mode == "checkpoint":
                solver.restore(c, saved)
            else:
                solver.solve(c, init_disp=saved)
            fctx.sid = solver.solve_id
        g = solver.vjp(grad_d.to("cuda"), fctx.shape)
        # autograd wants the gradient where the control lives (it may be a CPU tensor)
        return g.to(fctx.cdev, fctx.cdtype), None, None


def displacement(control, solver, mode="checkpoint"):
    """Converged displacement d(control), differentiable w.r.t. control."""
    return _Displacement.apply(control, solver, mode)


def misfit(d, target, dx, mask=None, normalize=True):
    """eq. discrete_J written in torch: 1/2 sum_obs |d - d*|^2 dx^2 / Cbar."""
    t = torch.as_tensor(target, dtype=torch.float64, device=d.device)
    m = torch.ones(d.shape[1:], dtype=torch.float64, device=d.device) if mask is None else \
        torch.as_tensor(np.asarray(mask, dtype=np.float64), device=d.device)
    cb = ((t * t).sum(0) * m).sum() * dx * dx if normalize else torch.tensor(1.0, dtype=torch.float64)
    return 0.5 * (((d - t) ** 2).sum(0) * m).sum() * dx * dx / cb
