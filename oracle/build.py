"""Builds the CPU oracle (test infrastructure) into oracle/liboracle.so with gcc.

Plain FP64: -O2 -ffp-contract=off -fno-fast-math, no vectorised math library,
single-threaded.  Called by the package build step and, if the library is
missing, by the test suite.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "slbm_oracle.c")


def build(force=True):
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall",
           "-Wno-unused-function", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
