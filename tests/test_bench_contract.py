"""Host-side parts of the benchmark's contract (no GPU): one GPU only, and the
stored per-launch traffic figures are plausible for fused launches and tied to
the kernel sources they were measured with."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300, cwd=ROOT)
    assert out.returncode != 0
    assert "one GPU" in out.stdout + out.stderr


def test_traffic_per_launch_lies_between_the_state_and_the_single_step_bytes():
    sys.path.insert(0, ROOT)
    import bench
    for (n, T, H), e in bench.TRAFFIC.items():
        per_node = e["bytes"] / (n * n)
        # at least the 128 B of state read and written once per launch, at most
        # the 144 B per step of T single-step sweeps
        assert 128.0 <= per_node < bench.BYTES_PER_NODE * T, (n, T, H, per_node)
        assert len(e["sources"]) == 16


def test_kernel_source_hash_names_the_sweep_sources():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()


def test_kernel_source_hash_ignores_comments_and_layout():
    """Comment and whitespace edits keep the hash (the counters still describe
    the kernel); code edits and string contents do not."""
    sys.path.insert(0, ROOT)
    import bench
    a = 'int f(int x) { return x + 1; } // one\nconst char* s = "a // b";'
    b = '/* note */ int  f(int x)\n{\n    return x + 1;   // other words\n}\nconst char* s = "a // b";'
    assert bench.code_text(a) == bench.code_text(b)
    assert bench.code_text(a) != bench.code_text(a.replace("x + 1", "x + 2"))
    assert bench.code_text(a) != bench.code_text(a.replace('"a // b"', '"a  // b"'))


def test_primal_only_warm_start_parts_are_checked_before_any_device_call():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--mode", "warmstart", "--ws-primal",
                          "cold,bogus"], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert out.returncode != 0
    assert "--ws-primal takes cold, warm or cold,warm" in out.stdout + out.stderr
