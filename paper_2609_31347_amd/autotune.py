"""Launch-shape autotuner for the fused (multi-step) sweeps.

For one problem context it times a small set of candidate launch shapes with
the library's own HIP-event timer (`solid_lbm_time_sweeps`, primal sweeps),
keeps the fastest and caches the choice per (GPU, grid, domain, control kind)
in a JSON file, so later contexts of the same shape skip the timing.  A
candidate is (T, H, tw, th): T time steps per launch; H rows per wave of the
wave-strip kernel (periodic, uniform material) or, with tw, th > 0, a tw x th
tile of the LDS-tiled kernel (any problem); T = 1 is one step per launch.
Plates and E-field controls only take tiled or single-step shapes.  The timed
sweeps advance the context's current state; call it before a solve
(primal_solve resets the state).
"""
import json
import os

from . import slbm as S

# in order of preference on near-ties (larger T moves fewer HBM bytes per step)
# short strips (H = 8, 12 with T <= 6) give grids that do not fill the chip more waves
STRIP = ((8, 24, 0, 0), (8, 32, 0, 0), (8, 48, 0, 0), (8, 64, 0, 0), (8, 96, 0, 0), (8, 12, 0, 0), (6, 24, 0, 0),
         (6, 48, 0, 0), (6, 12, 0, 0), (4, 24, 0, 0), (8, 8, 0, 0), (6, 8, 0, 0), (4, 12, 0, 0), (4, 8, 0, 0),
         (2, 8, 0, 0))
# 3 steps with 26 x 26 tiles: one workgroup per compute unit at 512 x 308 (240 tiles), where 20 x 20
# tiles (416) take two rounds (measured 4.47 against 5.0 us per step)
TILES = ((8, 0, 16, 16), (6, 0, 20, 20), (4, 0, 24, 24), (6, 0, 52, 4), (8, 0, 8, 8), (8, 0, 12, 12),
         (3, 0, 26, 26), (5, 0, 22, 22))
SINGLE = ((1, 0, 0, 0),)
CANDIDATES = STRIP + TILES + SINGLE
TIE = 0.02
CACHE = os.environ.get("SLBM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "slbm_autotune.json"))


def _tiled_only(problem):
    return int(problem.get("domain", 0)) == S.MASKED or int(problem.get("control_kind", 0)) == S.CTRL_E_NODAL


def _apply(ctx, c):
    T, H, tw, th = c
    S.solid_lbm_set_tiles(ctx, 0, 0)
    if tw > 0:
        # tiles first at one step per launch (odd step counts need tiles on
        # periodic problems; the tile must fit with the final halo)
        S.solid_lbm_set_tuning(ctx, 1, 0)
        S.solid_lbm_set_tiles(ctx, tw, th)
    S.solid_lbm_set_tuning(ctx, T, H)


def _name(c):
    return f"{c[0]},{c[1]}" if c[2] == 0 else f"{c[0]},tile{c[2]}x{c[3]}"


def _key(ctx, problem, device):
    # the candidate set is part of the key: a cached choice from another set is not reused
    cands = len(STRIP), len(TILES), len(SINGLE)
    return (f"{device}|{problem['nx']}x{problem['ny']}|dom{problem.get('domain', 0)}"
            f"|ctrl{problem.get('control_kind', 0)}|cand{cands[0]}.{cands[1]}.{cands[2]}")


def device_key():
    """The current GPU's architecture and name: a cached shape is reused only on
    the same kind of GPU."""
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(props, 'gcnArchName', '')}:{props.name}"


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = f"{CACHE}.{os.getpid()}.tmp"       # per process: concurrent tuners do not share it
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def autotune(ctx, problem, control, sweeps=96, device=None, use_cache=True, candidates=None):
    """Chooses and sets the launch shape of ctx.  `control` is any valid
    control for the problem (it sets the forcing the sweeps run with).  Returns
    {"T", "H", "tiles": [tw, th], "us": {shape: primal us per step}, "cached"}.
    `device` names the GPU in the cache key (default: device_key())."""
    key = _key(ctx, problem, device_key() if device is None else device)
    if candidates is None:
        candidates = (TILES + SINGLE) if _tiled_only(problem) else CANDIDATES
    cache = _load() if use_cache else {}
    if key in cache and "tiles" in cache[key]:
        e = cache[key]
        _apply(ctx, (e["T"], e["H"], e["tiles"][0], e["tiles"][1]))
        return dict(e, cached=True)
    S.solid_lbm_set_control(ctx, control)
    times = {}
    for c in candidates:
        _apply(ctx, c)
        T = max(c[0], 1)
        n = max(sweeps // T, 1) * T
        S.solid_lbm_time_sweeps(ctx, 0, T * 2)               # warm-up of this shape
        times[c] = S.solid_lbm_time_sweeps(ctx, 0, n) / n * 1e3
    fastest = min(times.values())
    best = next(c for c in candidates if times[c] <= fastest * (1.0 + TIE))
    _apply(ctx, best)
    out = {"T": best[0], "H": best[1], "tiles": [best[2], best[3]],
           "us": {_name(k): round(v, 3) for k, v in times.items()}}
    if use_cache:
        cache = _load()
        cache[key] = out
        _save(cache)
    return dict(out, cached=False)


def autotune_batch(batch, controls=None, sweeps=48,
                   candidates=((8, 24), (8, 48), (8, 96), (6, 24), (6, 48), (4, 24), (1, 0)),
                   tile_candidates=(6, 4, 3, 8)):
    """Chooses the fused shape (T, H) of a batch's periodic instances, then the
    steps per launch of its tiled instances (plates, E fields), by timing
    batched primal sweeps of all instances; near-ties go to the earlier
    candidate.  Returns {"T", "H", "Tt", "us", "us_tiles"} with the time per
    batched step."""
    from . import slbm as S
    times = {}
    S.solid_lbm_batch_set_tile_steps(batch, tile_candidates[0])
    for T, H in candidates:
        S.solid_lbm_batch_set_tuning(batch, T, H)
        t = max(T, 1)
        S.solid_lbm_batch_time_sweeps(batch, 0, 2 * t)
        n = max(sweeps // t, 1) * t
        times[(T, H)] = S.solid_lbm_batch_time_sweeps(batch, 0, n) / n * 1e3
    fastest = min(times.values())
    best = next(c for c in candidates if times[c] <= fastest * (1.0 + TIE))
    S.solid_lbm_batch_set_tuning(batch, best[0], best[1])
    tile_times = {}
    n = 24 * max(sweeps // 24, 1)                 # a multiple of every candidate's steps
    for Tt in tile_candidates:
        S.solid_lbm_batch_set_tile_steps(batch, Tt)
        S.solid_lbm_batch_time_sweeps(batch, 0, 2 * Tt)
        tile_times[Tt] = S.solid_lbm_batch_time_sweeps(batch, 0, n) / n * 1e3
    fastest = min(tile_times.values())
    best_t = next(c for c in tile_candidates if tile_times[c] <= fastest * (1.0 + TIE))
    S.solid_lbm_batch_set_tile_steps(batch, best_t)
    return {"T": best[0], "H": best[1], "Tt": best_t, "us": {f"{k[0]},{k[1]}": round(v, 3) for k, v in times.items()},
            "us_tiles": {str(k): round(v, 3) for k, v in tile_times.items()}}
