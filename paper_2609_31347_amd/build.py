"""Builds the HIP library libslbm.so for gfx950 with hipcc (in-tree)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libslbm.so")
SRC = [os.path.join(HERE, "csrc", "slbm.hip"), os.path.join(HERE, "csrc", "slbm_net.hip")]
ARCH = os.environ.get("SLBM_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(force=True, verbose=False):
    """Compile every HIP source into libslbm.so (always recompiles when force)."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    # -ffp-contract=on: a multiply-add is fused only within one source
    # expression, so the node arithmetic shared by the single-step and the
    # fused kernels rounds the same in every kernel (hipcc's default "fast"
    # lets the backend decide per kernel)
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", tmp] + SRC
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
