"""The C-ABI library loads and exports every entry point its header declares,
and rejects bad problems on the host (no GPU needed: validation runs before
any device call)."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def S():
    from paper_2609_31347_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_2609_31347_amd import slbm
    return slbm


def declared(header="solid_lbm.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*|slbm_ctx\s*\*)\s*\**\s*(\w+)\s*\(", src,
                                 flags=re.M)))


def test_every_declared_symbol_is_exported(S):
    headers = sorted(h for h in os.listdir(os.path.join(ROOT, "include")) if h.endswith(".h"))
    assert "solid_lbm.h" in headers and "solid_lbm_net.h" in headers
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    for h in headers:
        names = declared(h)
        assert len(names) >= 7, h
        for n in names:
            assert n in exported, (h, n)
            assert hasattr(S.LIB, n)
    # the binding lists exactly the solver header's entry points
    assert set(S.EXPORTS) == set(declared("solid_lbm.h"))


def base_problem(**kw):
    n = 8
    p = dict(nx=n, ny=n, dx=1 / n, E=1.0, nu=0.3, domain=0, control_kind=1, tol=1e-10, max_steps=100)
    p.update(kw)
    p.setdefault("target", np.ones((2, p["ny"], p["nx"])))
    return p


@pytest.mark.parametrize("bad,code", [
    (dict(nx=2), -1), (dict(dx=0.0), -1), (dict(nu=1.0), -1), (dict(nu=-1.5), -1), (dict(E=-1.0), -1),
    (dict(control_kind=7), -1), (dict(max_steps=0), -1), (dict(check_interval=-3), -1),
    (dict(domain=5), -1), (dict(control_kind=0, n_modes=0), -1), (dict(target=None), -1),
    (dict(domain=1), -1), (dict(tol=float("nan")), -1), (dict(dx=1e-12), -1), (dict(dx=1e-200), -1),
    (dict(convergence=2), -1), (dict(convergence=1, cv_window=1), -1), (dict(convergence=1, cv_window=33), -1),
])
def test_init_rejects_bad_problems(S, bad, code):
    p = base_problem(**bad)
    with pytest.raises(S.SlbmError) as e:
        S.solid_lbm_init(p)
    assert e.value.code == code
    assert str(e.value)


def test_init_rejects_non_finite_target(S):
    t = np.ones((2, 8, 8))
    t[1, 3, 3] = np.nan
    with pytest.raises(S.SlbmError) as e:
        S.solid_lbm_init(base_problem(target=t))
    assert e.value.code == S.ENONFINITE


def test_init_rejects_inconsistent_plate(S):
    from paper_2609_31347_amd import inputs as I
    pd = I.paper_plate(16)
    p = dict(nx=pd["nx"], ny=pd["ny"], dx=pd["dx"], E=0.1, nu=0.7, domain=1,
             node_mask=pd["active"].astype(np.uint8), link_bc=pd["bc"].copy(), link_wall=pd["wall"],
             link_normal=pd["normal"], target=pd["target"], control_kind=1)
    p["link_bc"][0][pd["active"] & (pd["bc"][0] == 0)] = 1          # a link into an inside node
    with pytest.raises(S.SlbmError) as e:
        S.solid_lbm_init(p)
    assert e.value.code == S.EINVAL and "cut links" in str(e.value)
    edge = pd["active"].astype(np.uint8).copy()
    edge[0, 5] = 1
    with pytest.raises(S.SlbmError) as e:
        S.solid_lbm_init(dict(p, node_mask=edge, link_bc=pd["bc"]))
    assert "box edge" in str(e.value)


def test_binding_refuses_to_run_without_library(tmp_path):
    """The product path has no CPU fallback: a missing library is an ImportError."""
    code = ("import sys, importlib.util; spec = importlib.util.spec_from_file_location('s', sys.argv[1]);"
            "m = importlib.util.module_from_spec(spec); m.__file__ = sys.argv[2]\n"
            "import os\nsrc = open(sys.argv[1]).read().replace('HERE = os.path.dirname(os.path.abspath(__file__))',"
            " 'HERE = sys.argv[2]')\n"
            "try:\n    exec(compile(src, 'slbm', 'exec'), {'__name__': 's', 'sys': sys})\nexcept ImportError as e:\n"
            "    print('IMPORTERROR', e)\n")
    out = subprocess.run(["python", "-c", code, os.path.join(ROOT, "paper_2609_31347_amd", "slbm.py"),
                          str(tmp_path)], capture_output=True, text=True)
    assert "IMPORTERROR" in out.stdout


def test_binding_checks_dtype_length_and_layout(S):
    """Arrays cross the C ABI as bare FP64 pointers of a known length, so the
    binding refuses anything the library would misread or overrun (no GPU
    needed: host arrays and CPU tensors)."""
    import torch
    keep = []
    ptr, kind = S._arg([1, 2, 3], keep, size=3)                       # lists and ints convert
    assert kind == S.PTR_HOST and keep[-1].dtype == np.float64
    with pytest.raises(ValueError):
        S._arg(np.zeros(4), keep, size=3, what="control")
    S._out(np.zeros(6), 6, "grad")
    S._out(torch.zeros(2, 3, dtype=torch.float64), 6, "grad")
    for bad in (np.zeros(6, np.float32), np.zeros((6, 2))[:, 0], np.zeros(6).astype(np.float64)[::1].view(),
                torch.zeros(6, dtype=torch.float32), torch.zeros(12, dtype=torch.float64)[::2], [0.0] * 6):
        if isinstance(bad, np.ndarray) and bad.dtype == np.float64 and bad.flags.c_contiguous:
            bad.flags.writeable = False                                 # read-only output buffer
        with pytest.raises((TypeError, ValueError)):
            S._out(bad, 6, "grad")
    with pytest.raises(ValueError):
        S._out(np.zeros(5), 6, "grad")


def test_one_hip_runtime_when_the_binding_is_imported_before_torch():
    """Imported first, the binding must not bring in a second HIP runtime next to
    the one torch ships (two runtimes in one process refuse device allocations)."""
    code = ("from paper_2609_31347_amd import slbm\n"
            "import torch\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_binding_checks_problem_array_lengths(S):
    """Every problem array must have the length the library reads (N, 8N, 16N,
    2N or n_modes * 2N entries); a short one is refused before the call."""
    from paper_2609_31347_amd import inputs as I
    n = 8
    with pytest.raises(ValueError, match="target"):
        S.solid_lbm_init(base_problem(target=np.ones((2, n, n - 1))))
    with pytest.raises(ValueError, match="force_modes"):
        S.solid_lbm_init(base_problem(control_kind=0, n_modes=2, force_modes=np.ones((1, 2, n, n))))
    with pytest.raises(ValueError, match="obs_mask"):
        S.solid_lbm_init(base_problem(obs_mask=np.ones(n * n - 1, np.uint8)))
    pd = I.paper_plate(8)
    plate = base_problem(nx=pd["nx"], ny=pd["ny"], dx=pd["dx"], domain=1, node_mask=pd["active"].astype(np.uint8),
                         link_bc=pd["bc"], link_wall=pd["wall"], link_normal=pd["normal"], target=pd["target"])
    for name in ("node_mask", "link_bc", "link_wall", "link_normal"):
        short = np.asarray(plate[name]).ravel()[:-1]
        with pytest.raises(ValueError, match=name):
            S.solid_lbm_init(dict(plate, **{name: short}))


def test_init_rejects_a_grid_beyond_the_node_limit(S):
    """More than 2^31 nodes is refused before any array is read, so a tiny
    target buffer stands in for the 2N doubles such a grid would need."""
    import ctypes
    p = S._Problem()
    p.nx = p.ny = 46341                        # 46341^2 > 2^31
    p.dx, p.E, p.nu, p.domain, p.control_kind = 1 / 46341, 1.0, 0.3, 0, 1
    tiny = np.zeros(2)
    p.target = tiny.ctypes.data
    p.max_steps, p.tol = 100, 1e-10
    h = ctypes.c_void_p()
    assert S.LIB.solid_lbm_init(ctypes.byref(p), ctypes.byref(h)) == S.EINVAL
    assert "too large" in S.LIB.solid_lbm_last_error(None).decode()
    assert not h.value
