"""Python binding of the HIP solid-LBM library (argument marshalling only).

Every function has the name of the C entry point it calls (include/solid_lbm.h);
all work runs in libslbm.so.  Arrays may be numpy arrays (host) or torch CUDA
tensors (device pointers are passed through, no copies).  If the library has
not been built the import of this module raises: there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslbm.so")

OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, ESTATE, ENONFINITE = 0, 1, -1, -2, -3, -4, -5
PERIODIC, MASKED = 0, 1
CTRL_FORCE_MODES, CTRL_FORCE_NODAL, CTRL_E_NODAL, CTRL_E_SCALAR_SQ = 0, 1, 2, 3
PTR_HOST, PTR_DEVICE = 0, 1
CONV_KLAG, CONV_CV = 0, 1
(FIELD_DISP, FIELD_STRESS, FIELD_ADJ_DISP, FIELD_POPS, FIELD_ADJ_POPS, FIELD_RESIDUAL, FIELD_CUR_DISP,
 FIELD_AVG_POPS) = range(8)
FIELD_COMPS = {FIELD_DISP: 2, FIELD_STRESS: 3, FIELD_ADJ_DISP: 2, FIELD_POPS: 8, FIELD_ADJ_POPS: 8,
               FIELD_RESIDUAL: 2, FIELD_CUR_DISP: 2, FIELD_AVG_POPS: 8}
EXPORTS = ("solid_lbm_init", "primal_solve", "adjoint_solve", "objective_and_grad", "objective_and_grad_from",
           "adjoint_solve_vjp", "tangent_solve",
           "solid_lbm_restore_solve", "solid_lbm_objective", "solid_lbm_set_control",
           "solid_lbm_run_steps", "solid_lbm_run_adjoint_steps", "solid_lbm_get_field",
           "solid_lbm_time_sweeps", "solid_lbm_set_tuning", "solid_lbm_set_tiles", "solid_lbm_set_progress",
           "solid_lbm_set_launch_timing",
           "solid_lbm_last_error",
           "solid_lbm_destroy",
           "solid_lbm_batch_init", "batch_objective_and_grad", "batch_objective_and_grad_noalloc",
           "batch_objective_and_grad_from",
           "batch_gradient", "solid_lbm_batch_set_tuning", "solid_lbm_batch_set_tile_steps", "solid_lbm_batch_set_persistent",
           "solid_lbm_batch_persistent_stats", "solid_lbm_batch_set_progress",
           "solid_lbm_batch_time_sweeps", "solid_lbm_batch_instance", "solid_lbm_batch_last_error",
           "solid_lbm_batch_destroy")


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double)


class SlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"solid_lbm error {code}: {msg}")
        self.code = code


class NotConverged(SlbmError):
    """A solve stopped at max_steps before its residual reached tol
    (SLBM_NOT_CONVERGED): its outputs exist but are not a steady state."""

    def __init__(self, what, info=None):
        extra = "" if info is None else f" (steps {info.steps}, residual {info.residual:.3e})"
        super().__init__(NOT_CONVERGED, f"{what}: max_steps reached before tol{extra}")
        self.info = info


def require_converged(rc, what, info=None):
    """Raises NotConverged for rc == SLBM_NOT_CONVERGED (the wrappers whose
    results feed gradients, optimisers or training data call this)."""
    if rc == NOT_CONVERGED:
        raise NotConverged(what, info)
    return rc


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double),
        ("E", ctypes.c_double), ("nu", ctypes.c_double), ("domain", ctypes.c_int32),
        ("node_mask", ctypes.c_void_p), ("link_bc", ctypes.c_void_p), ("link_wall", ctypes.c_void_p),
        ("link_normal", ctypes.c_void_p), ("fixed_force", ctypes.c_void_p), ("target", ctypes.c_void_p),
        ("obs_mask", ctypes.c_void_p), ("control_kind", ctypes.c_int32), ("n_modes", ctypes.c_int32),
        ("force_modes", ctypes.c_void_p), ("zero_mean_projection", ctypes.c_int32),
        ("normalize_objective", ctypes.c_int32), ("tol", ctypes.c_double), ("max_steps", ctypes.c_int64),
        ("check_interval", ctypes.c_int32), ("stream", ctypes.c_void_p),
        ("convergence", ctypes.c_int32), ("cv_window", ctypes.c_int32),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("sweeps", ctypes.c_int64), ("residual", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("device_ms", ctypes.c_double), ("converged", ctypes.c_int32),
                ("fused_launches", ctypes.c_int64), ("fused_sweeps", ctypes.c_int64), ("fused_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python paper_2609_31347_amd/build.py`")
    # torch first: the library then binds to the HIP runtime torch has already
    # loaded (same soname), so one runtime serves torch's tensors and the
    # library.  Loaded first, the library would pull in the system ROCm's
    # runtime and torch would add its own: two runtimes on one device refuse
    # each other's allocations and pointers.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, pp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)
    info = ctypes.POINTER(SolveInfo)
    lib.solid_lbm_init.argtypes = [ctypes.POINTER(_Problem), pp]
    lib.primal_solve.argtypes = [P, P, P, ctypes.c_int32, info]
    lib.adjoint_solve.argtypes = [P, info]
    lib.objective_and_grad.argtypes = [P, P, ctypes.POINTER(ctypes.c_double), P, ctypes.c_int32, info, info]
    lib.solid_lbm_set_control.argtypes = [P, P, P, ctypes.c_int32]
    lib.solid_lbm_run_steps.argtypes = [P, ctypes.c_int64]
    lib.solid_lbm_run_adjoint_steps.argtypes = [P, ctypes.c_int64]
    lib.solid_lbm_get_field.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32]
    lib.solid_lbm_time_sweeps.argtypes = [P, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    lib.solid_lbm_set_tuning.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    lib.tangent_solve.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.c_int32, info]
    lib.solid_lbm_set_tiles.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    lib.solid_lbm_set_progress.argtypes = [P, PROGRESS_FN, P, ctypes.c_double]
    lib.solid_lbm_set_launch_timing.argtypes = [P, ctypes.c_int32]
    lib.adjoint_solve_vjp.argtypes = [P, P, P, ctypes.c_int32, info]
    lib.objective_and_grad_from.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_double), P, ctypes.c_int32, info, info]
    lib.solid_lbm_restore_solve.argtypes = [P, P, P, ctypes.c_int32]
    lib.solid_lbm_objective.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    lib.solid_lbm_last_error.argtypes = [P]
    lib.solid_lbm_last_error.restype = ctypes.c_char_p
    lib.solid_lbm_destroy.argtypes = [P]
    lib.solid_lbm_destroy.restype = None
    lib.solid_lbm_batch_init.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int32, pp]
    lib.batch_objective_and_grad.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, info, info]
    lib.batch_gradient.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, info]
    lib.batch_objective_and_grad_noalloc.argtypes = lib.batch_objective_and_grad.argtypes
    lib.batch_objective_and_grad_from.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_void_p),
                                                  ctypes.c_int32, info, info]
    lib.solid_lbm_batch_set_persistent.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    lib.solid_lbm_batch_persistent_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.solid_lbm_batch_set_tuning.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    lib.solid_lbm_batch_set_tile_steps.argtypes = [P, ctypes.c_int32]
    lib.solid_lbm_batch_set_progress.argtypes = [P, PROGRESS_FN, P, ctypes.c_double]
    lib.solid_lbm_batch_time_sweeps.argtypes = [P, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    lib.solid_lbm_batch_instance.argtypes = [P, ctypes.c_int32]
    lib.solid_lbm_batch_instance.restype = ctypes.c_void_p
    lib.solid_lbm_batch_last_error.argtypes = [P]
    lib.solid_lbm_batch_last_error.restype = ctypes.c_char_p
    lib.solid_lbm_batch_destroy.argtypes = [P]
    lib.solid_lbm_batch_destroy.restype = None
    for f in EXPORTS:
        if f not in ("solid_lbm_last_error", "solid_lbm_destroy", "solid_lbm_batch_instance",
                     "solid_lbm_batch_last_error", "solid_lbm_batch_destroy"):
            getattr(lib, f).restype = ctypes.c_int
    return lib


LIB = _load()


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _tensor_ok(a, size, what):
    # the library reads and writes FP64 arrays of a known length through the
    # pointer: anything else would be misread or overrun
    if str(a.dtype) != "torch.float64":
        raise TypeError(f"{what}: tensors must be float64, got {a.dtype}")
    if not a.is_contiguous():
        raise ValueError(f"{what}: tensors must be contiguous")
    if size is not None and a.numel() != size:
        raise ValueError(f"{what}: {a.numel()} elements, expected {size}")


def _arg(a, keep, dtype=np.float64, size=None, what="array"):
    """(pointer, ptr_kind) of an input array; host arrays are converted to
    contiguous `dtype` and kept alive; device tensors must be float64 and
    contiguous; `size` (if given) is the required element count."""
    if a is None:
        return None, PTR_HOST
    if _is_torch(a):
        if a.is_cuda:
            _tensor_ok(a, size, what)
            return a.data_ptr(), PTR_DEVICE
        a = a.detach().numpy()
    arr = np.ascontiguousarray(a, dtype=dtype)
    if size is not None and arr.size != size:
        raise ValueError(f"{what}: {arr.size} elements, expected {size}")
    keep.append(arr)
    return arr.ctypes.data, PTR_HOST


def _out(a, size, what):
    """(pointer, ptr_kind) of a caller's output buffer, written in place: a
    float64, contiguous, writeable array or tensor of exactly `size` elements."""
    if _is_torch(a):
        _tensor_ok(a, size, what)
        return a.data_ptr(), PTR_DEVICE if a.is_cuda else PTR_HOST
    if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags.c_contiguous \
            or not a.flags.writeable:
        raise TypeError(f"{what}: output arrays must be writeable, contiguous float64 numpy arrays")
    if a.size != size:
        raise ValueError(f"{what}: {a.size} elements, expected {size}")
    return a.ctypes.data, PTR_HOST


class Context:
    """Owns one slbm_ctx (freed by solid_lbm_destroy or on garbage collection),
    or borrows one of a batch (owned=False)."""

    def __init__(self, handle, problem, owned=True):
        self.handle = handle
        self.owned = owned
        self.nx, self.ny = problem["nx"], problem["ny"]
        self.N = self.nx * self.ny
        self.control_kind = problem.get("control_kind", CTRL_FORCE_MODES)
        self.n_modes = problem.get("n_modes", 0)

    def grad_len(self):
        return {CTRL_FORCE_MODES: self.n_modes, CTRL_FORCE_NODAL: 2 * self.N, CTRL_E_NODAL: self.N,
                CTRL_E_SCALAR_SQ: 1}[self.control_kind]

    def __del__(self, _destroy=LIB.solid_lbm_destroy):
        # the destroy function is bound at definition time: at interpreter
        # shutdown the module globals may already be gone
        if getattr(self, "handle", None) and getattr(self, "owned", True):
            _destroy(self.handle)
            self.handle = None


def _check(ctx, rc):
    if rc < 0:
        msg = LIB.solid_lbm_last_error(ctx.handle if ctx is not None else None)
        raise SlbmError(rc, msg.decode() if msg else "")
    return rc


def _problem_struct(problem, keep):
    p = _Problem()
    p.nx, p.ny = int(problem["nx"]), int(problem["ny"])
    p.dx = float(problem["dx"])
    p.E, p.nu = float(problem.get("E", 1.0)), float(problem["nu"])
    p.domain = int(problem.get("domain", PERIODIC))
    p.control_kind = int(problem.get("control_kind", CTRL_FORCE_MODES))
    p.n_modes = int(problem.get("n_modes", 0))
    # element counts the library reads (layouts of include/solid_lbm.h); the mode
    # fields are read only for FORCE_MODES, and the library checks the sizes themselves
    N = p.nx * p.ny if p.nx > 0 and p.ny > 0 else 0
    modes = p.n_modes * 2 * N if p.control_kind == CTRL_FORCE_MODES and p.n_modes > 0 else None
    for name, dt, size in (("node_mask", np.uint8, N), ("link_bc", np.uint8, 8 * N),
                           ("link_wall", np.float64, 16 * N), ("link_normal", np.float64, 16 * N),
                           ("fixed_force", np.float64, 2 * N), ("target", np.float64, 2 * N),
                           ("obs_mask", np.uint8, N), ("force_modes", np.float64, modes)):
        v = problem.get(name)
        if v is not None:
            ptr, kind = _arg(v, keep, dt, size, name)
            if kind != PTR_HOST:
                raise ValueError(f"{name} must be host memory")
            setattr(p, name, ptr)
    p.zero_mean_projection = int(problem.get("zero_mean_projection", 1))
    p.normalize_objective = int(problem.get("normalize_objective", 1))
    p.tol = float(problem.get("tol", 1e-10))
    p.max_steps = int(problem.get("max_steps", 10_000_000))
    p.check_interval = int(problem.get("check_interval", 0))
    p.stream = problem.get("stream")
    p.convergence = int(problem.get("convergence", CONV_KLAG))
    p.cv_window = int(problem.get("cv_window", 0))
    return p


def solid_lbm_init(problem):
    """problem: dict with the fields of slbm_problem (arrays as numpy)."""
    keep = []
    p = _problem_struct(problem, keep)
    h = ctypes.c_void_p()
    rc = LIB.solid_lbm_init(ctypes.byref(p), ctypes.byref(h))
    if rc < 0:
        raise SlbmError(rc, LIB.solid_lbm_last_error(None).decode())
    return Context(h, dict(problem))


def primal_solve(ctx, control, init_disp=None):
    """(rc, info): solve the primal to steady state for `control` (cold start, or
    warm-started from the displacement init_disp); rc 1 = step limit reached."""
    keep = []
    cp, kind = _arg(control, keep, size=ctx.grad_len(), what="control")
    ip, kind2 = _arg(init_disp, keep, size=2 * ctx.N, what="init_disp")
    if init_disp is not None and kind2 != kind:
        raise ValueError("control and init_disp must live in the same memory kind")
    info = SolveInfo()
    rc = _check(ctx, LIB.primal_solve(ctx.handle, cp, ip, kind, ctypes.byref(info)))
    return rc, info


def adjoint_solve(ctx):
    """(rc, info): solve the adjoint of the last completed primal solve."""
    info = SolveInfo()
    rc = _check(ctx, LIB.adjoint_solve(ctx.handle, ctypes.byref(info)))
    return rc, info


def objective_and_grad(ctx, control, grad=None, want_grad=True, init_disp=None):
    """Returns (rc, J, grad, primal_info, adjoint_info).  grad: optional output
    array/tensor (device tensors are written in place); allocated on the host
    when not given.  init_disp: warm start of the primal (objective_and_grad_from)."""
    keep = []
    cp, kind = _arg(control, keep, size=ctx.grad_len(), what="control")
    ip, kind2 = _arg(init_disp, keep, size=2 * ctx.N, what="init_disp")
    if init_disp is not None and kind2 != kind:
        raise ValueError("control and init_disp must live in the same memory kind")
    out = None
    gp = None
    if want_grad:
        out = np.zeros(ctx.grad_len()) if grad is None else grad
        gp, gkind = _out(out, ctx.grad_len(), "grad")
        if gkind != kind:
            raise ValueError("control and grad must live in the same memory kind")
    J = ctypes.c_double()
    pi, ai = SolveInfo(), SolveInfo()
    if init_disp is None:
        rc = _check(ctx, LIB.objective_and_grad(ctx.handle, cp, ctypes.byref(J), gp, kind, ctypes.byref(pi),
                                                ctypes.byref(ai)))
    else:
        rc = _check(ctx, LIB.objective_and_grad_from(ctx.handle, cp, ip, ctypes.byref(J), gp, kind,
                                                     ctypes.byref(pi), ctypes.byref(ai)))
    return rc, J.value, out, pi, ai


def solid_lbm_set_control(ctx, control, init_disp=None):
    """Set the control and reset the primal state (to rest, or to the
    equilibrium of init_disp) without solving."""
    keep = []
    cp, kind = _arg(control, keep, size=ctx.grad_len(), what="control")
    ip, kind2 = _arg(init_disp, keep, size=2 * ctx.N, what="init_disp")
    if init_disp is not None and kind2 != kind:
        raise ValueError("control and init_disp must live in the same memory kind")
    return _check(ctx, LIB.solid_lbm_set_control(ctx.handle, cp, ip, kind))


def solid_lbm_run_steps(ctx, n):
    """Advance the current primal state by n fixed steps (no convergence test)."""
    return _check(ctx, LIB.solid_lbm_run_steps(ctx.handle, int(n)))


def solid_lbm_run_adjoint_steps(ctx, n):
    """Restart the adjoint from rest and advance it by n fixed steps, with the
    residual of the last primal solve as its source."""
    return _check(ctx, LIB.solid_lbm_run_adjoint_steps(ctx.handle, int(n)))


def solid_lbm_get_field(ctx, which, out=None):
    """Copy field `which` (FIELD_*) into out (host array or CUDA tensor of
    FIELD_COMPS[which] x ny x nx doubles; allocated on the host when None)."""
    comps = FIELD_COMPS[which]
    if out is None:
        out = np.zeros((comps, ctx.ny, ctx.nx))
    op, okind = _out(out, comps * ctx.N, "out")
    _check(ctx, LIB.solid_lbm_get_field(ctx.handle, which, op, okind))
    return out


def solid_lbm_time_sweeps(ctx, adjoint, n):
    """Milliseconds of n primal (adjoint = 0) or adjoint sweeps in the current
    launch shape, measured with HIP events; advances the state."""
    ms = ctypes.c_double()
    _check(ctx, LIB.solid_lbm_time_sweeps(ctx.handle, int(adjoint), int(n), ctypes.byref(ms)))
    return ms.value


def adjoint_solve_vjp(ctx, d_cot, grad=None):
    """(rc, grad, info): grad = (d dbar / d control)^T d_cot at the last primal solve."""
    keep = []
    dp, kind = _arg(d_cot, keep, size=2 * ctx.N, what="d_cot")
    if grad is None:
        if kind == PTR_DEVICE:
            raise ValueError("pass a device grad tensor with a device cotangent")
        grad = np.zeros(ctx.grad_len())
    gp, gkind = _out(grad, ctx.grad_len(), "grad")
    if gkind != kind:
        raise ValueError("d_cot and grad must live in the same memory kind")
    info = SolveInfo()
    rc = _check(ctx, LIB.adjoint_solve_vjp(ctx.handle, dp, gp, kind, ctypes.byref(info)))
    return rc, grad, info


def tangent_solve(ctx, control, direction):
    """Forward mode: (rc, J, dJ, info) with dJ = grad J . direction."""
    keep = []
    cp, kind = _arg(control, keep, size=ctx.grad_len(), what="control")
    dp, kind2 = _arg(direction, keep, size=ctx.grad_len(), what="direction")
    if kind2 != kind:
        raise ValueError("control and direction must live in the same memory kind")
    J, dJ = ctypes.c_double(), ctypes.c_double()
    info = SolveInfo()
    rc = _check(ctx, LIB.tangent_solve(ctx.handle, cp, dp, ctypes.byref(J), ctypes.byref(dJ), kind,
                                       ctypes.byref(info)))
    return rc, J.value, dJ.value, info


def solid_lbm_restore_solve(ctx, control, avg_pops):
    """Reinstate a converged primal solve from its two-step-averaged
    populations (FIELD_AVG_POPS) without iterating."""
    keep = []
    cp, kind = _arg(control, keep, size=ctx.grad_len(), what="control")
    ap, kind2 = _arg(avg_pops, keep, size=8 * ctx.N, what="avg_pops")
    if kind != kind2:
        raise ValueError("control and avg_pops must live in the same memory kind")
    return _check(ctx, LIB.solid_lbm_restore_solve(ctx.handle, cp, ap, kind))


def solid_lbm_objective(ctx):
    """J of the last completed primal solve."""
    J = ctypes.c_double()
    _check(ctx, LIB.solid_lbm_objective(ctx.handle, ctypes.byref(J)))
    return J.value


def solid_lbm_set_tuning(ctx, steps_per_launch=-1, rows_per_wave=0):
    """Launch shape: time steps fused per launch (-1 automatic) and rows per
    wave of the wave-strip kernel (0 automatic); results do not change."""
    return _check(ctx, LIB.solid_lbm_set_tuning(ctx.handle, int(steps_per_launch), int(rows_per_wave)))


def solid_lbm_set_progress(ctx, fn=None, every_s=30.0):
    """fn(phase, step, residual) is called from inside long solves at least
    every_s seconds apart (phase 0 primal, 1 adjoint); None turns it off."""
    if fn is None:
        ctx._progress = None
        return _check(ctx, LIB.solid_lbm_set_progress(ctx.handle, PROGRESS_FN(), None, 0.0))
    cb = PROGRESS_FN(lambda user, phase, step, res: fn(int(phase), int(step), float(res)))
    ctx._progress = cb                        # keeps the C callback alive with the context
    return _check(ctx, LIB.solid_lbm_set_progress(ctx.handle, cb, None, float(every_s)))


def solid_lbm_set_launch_timing(ctx, on=True):
    """Fused-launch timing of the solve loops (SolveInfo.fused_launches / fused_sweeps / fused_ms)."""
    return _check(ctx, LIB.solid_lbm_set_launch_timing(ctx.handle, 1 if on else 0))


def solid_lbm_set_tiles(ctx, tile_w=0, tile_h=0):
    """Tile of the LDS-tiled kernel (0, 0 automatic); results do not change."""
    return _check(ctx, LIB.solid_lbm_set_tiles(ctx.handle, int(tile_w), int(tile_h)))


def solid_lbm_destroy(ctx):
    """Free the context's device memory now (otherwise on garbage collection)."""
    if ctx.handle:
        LIB.solid_lbm_destroy(ctx.handle)
        ctx.handle = None


# ------------------------------------------------------------------ batches

class Batch:
    """Owns one slbm_batch; `contexts[i]` are its instances (borrowed)."""

    def __init__(self, handle, problems):
        self.handle = handle
        self.problems = [dict(p) for p in problems]
        self.contexts = [Context(LIB.solid_lbm_batch_instance(handle, i), p, owned=False)
                         for i, p in enumerate(problems)]

    def __len__(self):
        return len(self.contexts)

    def __del__(self, _destroy=LIB.solid_lbm_batch_destroy):
        if getattr(self, "handle", None):
            for c in self.contexts:
                c.handle = None
            _destroy(self.handle)
            self.handle = None


def _bcheck(batch, rc):
    if rc < 0:
        msg = LIB.solid_lbm_batch_last_error(batch.handle if batch is not None else None)
        raise SlbmError(rc, msg.decode() if msg else "")
    return rc


def solid_lbm_batch_init(problems):
    """Batch of independent problems (any sizes and kinds) solved in shared launches."""
    keep = []
    arr = (_Problem * len(problems))()
    for i, pr in enumerate(problems):
        arr[i] = _problem_struct(pr, keep)
    h = ctypes.c_void_p()
    rc = LIB.solid_lbm_batch_init(arr, len(problems), ctypes.byref(h))
    if rc < 0:
        raise SlbmError(rc, LIB.solid_lbm_batch_last_error(None).decode())
    return Batch(h, problems)


def batch_objective_and_grad(batch, controls, grads=None, want_grad=True, noalloc=False, init_disps=None):
    """Returns (rc, J (array), grads (list), primal infos, adjoint infos).
    noalloc: call batch_objective_and_grad_noalloc (launch tables in the
    library's static device array; nothing is allocated during the call).
    init_disps: per-instance initial displacements (2N each, None entries =
    cold start) for batch_objective_and_grad_from."""
    B = len(batch)
    keep = []
    cptr = (ctypes.c_void_p * B)()
    kinds = set()
    if len(controls) != B:
        raise ValueError(f"{len(controls)} controls for {B} instances")
    for i, c in enumerate(controls):
        ptr, kind = _arg(c, keep, size=batch.contexts[i].grad_len(), what=f"controls[{i}]")
        cptr[i] = ptr
        kinds.add(kind)
    if len(kinds) != 1:
        raise ValueError("controls must all be host or all device")
    kind = kinds.pop()
    gptr = None
    if want_grad:
        if grads is None:
            if kind == PTR_DEVICE:
                raise ValueError("pass device grads with device controls")
            grads = [np.zeros(ctx.grad_len()) for ctx in batch.contexts]
        if len(grads) != B:
            raise ValueError(f"{len(grads)} grads for {B} instances")
        gptr = (ctypes.c_void_p * B)()
        for i, g in enumerate(grads):
            gptr[i], gkind = _out(g, batch.contexts[i].grad_len(), f"grads[{i}]")
            if gkind != kind:
                raise ValueError("controls and grads must live in the same memory kind")
    J = (ctypes.c_double * B)()
    pi, ai = (SolveInfo * B)(), (SolveInfo * B)()
    if init_disps is not None:
        if noalloc:
            raise ValueError("the no-allocation variant has no warm start")
        if len(init_disps) != B:
            raise ValueError(f"{len(init_disps)} init_disps for {B} instances")
        dptr = (ctypes.c_void_p * B)()
        for i, d0 in enumerate(init_disps):
            if d0 is None:
                dptr[i] = None
                continue
            dptr[i], dkind = _arg(d0, keep, size=2 * batch.contexts[i].N, what=f"init_disps[{i}]")
            if dkind != kind:
                raise ValueError("controls and init_disps must live in the same memory kind")
        rc = _bcheck(batch, LIB.batch_objective_and_grad_from(batch.handle, cptr, dptr, J, gptr, kind, pi, ai))
        return rc, np.array(J[:]), grads, list(pi), list(ai)
    fn = LIB.batch_objective_and_grad_noalloc if noalloc else LIB.batch_objective_and_grad
    rc = _bcheck(batch, fn(batch.handle, cptr, J, gptr, kind, pi, ai))
    return rc, np.array(J[:]), grads, list(pi), list(ai)


def batch_objective_and_grad_noalloc(batch, controls, grads=None, want_grad=True):
    """batch_objective_and_grad without device allocation during the call."""
    return batch_objective_and_grad(batch, controls, grads, want_grad, noalloc=True)


def batch_gradient(batch, grads=None):
    """After batch_objective_and_grad(..., want_grad=False) with host controls:
    (rc, grads, adjoint infos)."""
    B = len(batch)
    if grads is None:
        grads = [np.zeros(ctx.grad_len()) for ctx in batch.contexts]
    if len(grads) != B:
        raise ValueError(f"{len(grads)} grads for {B} instances")
    gptr = (ctypes.c_void_p * B)()
    kinds = set()
    for i, g in enumerate(grads):
        gptr[i], gkind = _out(g, batch.contexts[i].grad_len(), f"grads[{i}]")
        kinds.add(gkind)
    if len(kinds) != 1:
        raise ValueError("grads must all be host or all device")
    ai = (SolveInfo * B)()
    rc = _bcheck(batch, LIB.batch_gradient(batch.handle, gptr, kinds.pop(), ai))
    return rc, grads, list(ai)


def solid_lbm_batch_set_tuning(batch, steps_per_launch=-1, rows_per_wave=0):
    """Launch shape of the batch's shared launches (-1 / 0 automatic); results do not change."""
    return _bcheck(batch, LIB.solid_lbm_batch_set_tuning(batch.handle, int(steps_per_launch), int(rows_per_wave)))


def solid_lbm_batch_set_tile_steps(batch, steps_per_launch=-1):
    """Steps per launch of the batch's tiled instances (-1 automatic, 1 .. 8); results do not change."""
    return _bcheck(batch, LIB.solid_lbm_batch_set_tile_steps(batch.handle, int(steps_per_launch)))


def solid_lbm_batch_set_persistent(batch, on=True, rounds_per_launch=0):
    """Persistent, graph-captured launches for the batch's solves (see the header)."""
    return _bcheck(batch, LIB.solid_lbm_batch_set_persistent(batch.handle, 1 if on else 0, int(rounds_per_launch)))


def solid_lbm_batch_persistent_stats(batch):
    """(graph replays, rounds) of the last persistent solve half."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _bcheck(batch, LIB.solid_lbm_batch_persistent_stats(batch.handle, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def solid_lbm_batch_set_progress(batch, fn=None, every_s=30.0):
    """fn(phase, step, residual) is called from inside long batch solves at
    least every_s seconds apart (phase 0 primal, 1 adjoint; step and residual
    as the header states); None turns it off."""
    if fn is None:
        batch._progress = None
        return _bcheck(batch, LIB.solid_lbm_batch_set_progress(batch.handle, PROGRESS_FN(), None, 0.0))
    cb = PROGRESS_FN(lambda user, phase, step, res: fn(int(phase), int(step), float(res)))
    batch._progress = cb                      # keeps the C callback alive with the batch
    return _bcheck(batch, LIB.solid_lbm_batch_set_progress(batch.handle, cb, None, float(every_s)))


def solid_lbm_batch_time_sweeps(batch, adjoint, n):
    """Milliseconds of n batched primal (adjoint = 0) or adjoint sweeps of every
    instance; invalidates the instances' states."""
    ms = ctypes.c_double()
    _bcheck(batch, LIB.solid_lbm_batch_time_sweeps(batch.handle, int(adjoint), int(n), ctypes.byref(ms)))
    return ms.value


def solid_lbm_batch_destroy(batch):
    """Free the batch and its instances now (otherwise on garbage collection)."""
    if batch.handle:
        for c in batch.contexts:
            c.handle = None
        LIB.solid_lbm_batch_destroy(batch.handle)
        batch.handle = None
