"""Builds the CPU oracle (test infrastructure) into oracle/liboracle.so with gcc.

Plain FP64: -O2 -ffp-contract=off -fno-fast-math, no vectorised math library,
single-threaded.  Called by the package build step and, if the library is
missing, by the test suite.  build(sanitize=True) makes liboracle_san.so, the
same source under AddressSanitizer and UndefinedBehaviorSanitizer, which a CPU
test loads in a child process (SLBM_ORACLE_LIB) to run oracle pins under them.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "slbm_oracle.c")


SAN_LIB = os.path.join(HERE, "liboracle_san.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source (host
# code only; the oracle has no GPU code): every error aborts the process.
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]


def build(force=True, sanitize=False):
    lib = SAN_LIB if sanitize else LIB
    if not force and os.path.exists(lib):
        return lib
    tmp = lib + ".tmp"
    opt = SAN_FLAGS if sanitize else ["-O2"]
    cmd = ["gcc", "-std=c11"] + opt + ["-ffp-contract=off", "-fno-fast-math", "-Wall",
                                       "-Wno-unused-function", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build())
