"""Host logic of the launch-shape autotuner: the cache key separates GPUs,
grids, domains and control kinds, and the JSON cache round-trips (no GPU)."""
import json

from paper_2609_31347_amd import autotune as T


def test_cache_key_separates_device_grid_domain_and_control():
    p = dict(nx=64, ny=48, domain=0, control_kind=0)
    base = T._key(None, p, "gfx950:A")
    assert T._key(None, p, "gfx950:A") == base
    assert T._key(None, p, "gfx942:B") != base
    assert T._key(None, dict(p, nx=48, ny=64), "gfx950:A") != base
    assert T._key(None, dict(p, domain=1), "gfx950:A") != base
    assert T._key(None, dict(p, control_kind=2), "gfx950:A") != base
    assert f"cand{len(T.STRIP)}.{len(T.TILES)}.{len(T.SINGLE)}" in base


def test_cache_round_trip_and_unreadable_file(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "tune.json"
    monkeypatch.setattr(T, "CACHE", str(path))
    assert T._load() == {}                       # missing file: empty cache
    entry = {"T": 8, "H": 24, "tiles": [0, 0], "us": {"8,24": 5.3}}
    T._save({"k": entry})
    assert T._load() == {"k": entry}
    assert not list(path.parent.glob("*.tmp"))   # the temporary file was renamed into place
    path.write_text("{not json")
    assert T._load() == {}                       # unreadable cache: treated as empty
    T._save({"k2": entry})
    assert json.loads(path.read_text()) == {"k2": entry}


def test_plates_and_e_fields_take_only_tiled_or_single_step_shapes():
    assert T._tiled_only(dict(domain=T.S.MASKED, control_kind=T.S.CTRL_FORCE_NODAL))
    assert T._tiled_only(dict(domain=T.S.PERIODIC, control_kind=T.S.CTRL_E_NODAL))
    assert not T._tiled_only(dict(domain=T.S.PERIODIC, control_kind=T.S.CTRL_FORCE_MODES))
    assert all(c[2] > 0 for c in T.TILES) and all(c[2] == 0 for c in T.STRIP)


class _ShapeRules:
    """The library's shape checks on a periodic uniform problem: odd steps per
    launch only with tiles; a tile plus its halo (the current steps) within
    1024 nodes."""

    def __init__(self):
        self.T, self.tw, self.th, self.calls = 1, 0, 0, []

    def solid_lbm_set_tiles(self, ctx, tw, th):
        h = max(self.T, 1)
        if tw > 0 and (tw + 2 * h) * (th + 2 * h) > 1024:
            raise ValueError("tile plus halo exceeds 1024 nodes")
        self.tw, self.th = tw, th
        self.calls.append(("tiles", tw, th))

    def solid_lbm_set_tuning(self, ctx, T, H):
        if self.tw == 0 and T > 1 and T % 2:
            raise ValueError("periodic bulk problems fuse 2, 4, 6 or 8 steps per launch")
        if self.tw > 0 and T > 1 and (self.tw + 2 * T) * (self.th + 2 * T) > 1024:
            raise ValueError("tile plus halo exceeds 1024 nodes")
        self.T = T
        self.calls.append(("tuning", T, H))


def test_every_candidate_applies_after_any_other(monkeypatch):
    """_apply sets each candidate shape (odd-step tiles included) whatever
    shape was set before, and ends in exactly that shape."""
    rules = _ShapeRules()
    monkeypatch.setattr(T, "S", rules)
    for prev in T.CANDIDATES:
        for c in T.CANDIDATES:
            T._apply(None, prev)
            T._apply(None, c)
            assert (rules.T, rules.tw, rules.th) == (c[0], c[2], c[3])
