"""Host-side parts of the benchmark's contract (no GPU): one GPU only, and the
stored per-launch traffic figures are plausible for fused launches."""
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
    for (n, T, H), bytes_per_launch in bench.TRAFFIC_BYTES.items():
        per_node_step = bytes_per_launch / (n * n * T)
        # at least the 128 B of state read and written once per launch, at most
        # the 144 B per step of single-step sweeps
        assert 128.0 / T <= per_node_step < bench.BYTES_PER_NODE, (n, T, H, per_node_step)
