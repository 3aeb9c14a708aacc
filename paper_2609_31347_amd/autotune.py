"""Launch-shape autotuner for the fused (multi-step) sweeps.

For one problem context it times a small set of candidate shapes -- time steps
fused per launch T and rows per wave H -- with the library's own HIP-event
timer (`solid_lbm_time_sweeps`, primal and adjoint sweeps), keeps the fastest
and caches the choice per (GPU, grid, domain, control kind) in a JSON file, so
later contexts of the same shape skip the timing.  The timed sweeps advance the
context's current state; call it before a solve (primal_solve resets the state).
"""
import json
import os

from . import slbm as S

# in order of preference on near-ties (larger T moves fewer HBM bytes per step)
CANDIDATES = ((8, 24), (8, 48), (8, 64), (8, 96), (6, 24), (6, 48), (4, 24), (1, 0))
TIE = 0.02
CACHE = os.environ.get("SLBM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "slbm_autotune.json"))


def _key(ctx, problem, device):
    return f"{device}|{problem['nx']}x{problem['ny']}|dom{problem.get('domain', 0)}|ctrl{problem.get('control_kind', 0)}"


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def autotune(ctx, problem, control, sweeps=96, device="gpu0", use_cache=True, candidates=CANDIDATES):
    """Chooses and sets (T, H) for ctx.  `control` is any valid control for the
    problem (it sets the forcing the sweeps run with).  Returns
    {"T": T, "H": H, "us": {"T,H": (primal_us, adjoint_us)}, "cached": bool}."""
    key = _key(ctx, problem, device)
    cache = _load() if use_cache else {}
    if key in cache:
        T, H = cache[key]["T"], cache[key]["H"]
        S.solid_lbm_set_tuning(ctx, T, H)
        return dict(cache[key], cached=True)
    S.solid_lbm_set_control(ctx, control)
    times = {}
    for T, H in candidates:
        S.solid_lbm_set_tuning(ctx, T, H)
        n = max(sweeps // max(T, 1), 1) * max(T, 1)
        S.solid_lbm_time_sweeps(ctx, 0, max(T, 1) * 2)               # warm-up of this shape
        tp = S.solid_lbm_time_sweeps(ctx, 0, n) / n * 1e3
        times[(T, H)] = tp
    fastest = min(times.values())
    best = next(c for c in candidates if times[c] <= fastest * (1.0 + TIE))
    S.solid_lbm_set_tuning(ctx, best[0], best[1])
    out = {"T": best[0], "H": best[1], "us": {f"{k[0]},{k[1]}": round(v, 3) for k, v in times.items()}}
    if use_cache:
        cache = _load()
        cache[key] = out
        _save(cache)
    return dict(out, cached=False)


def autotune_batch(batch, controls=None, sweeps=48,
                   candidates=((8, 24), (8, 48), (8, 96), (6, 24), (6, 48), (4, 24), (1, 0))):
    """Chooses the fused shape (T, H) of a batch's periodic instances by timing
    batched primal sweeps of all instances (plates run their single steps in
    the same timing); near-ties go to the earlier candidate.  Returns
    {"T", "H", "us"} with the time per batched step."""
    from . import slbm as S
    times = {}
    for T, H in candidates:
        S.solid_lbm_batch_set_tuning(batch, T, H)
        t = max(T, 1)
        S.solid_lbm_batch_time_sweeps(batch, 0, 2 * t)
        n = max(sweeps // t, 1) * t
        times[(T, H)] = S.solid_lbm_batch_time_sweeps(batch, 0, n) / n * 1e3
    fastest = min(times.values())
    best = next(c for c in candidates if times[c] <= fastest * (1.0 + TIE))
    S.solid_lbm_batch_set_tuning(batch, best[0], best[1])
    return {"T": best[0], "H": best[1], "us": {f"{k[0]},{k[1]}": round(v, 3) for k, v in times.items()}}
