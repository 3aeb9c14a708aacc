"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds oracle/liboracle_san.so (same C source, -fsanitize=address,undefined,
no recovery) and runs a selection of oracle pins in a child process that
loads it (SLBM_ORACLE_LIB) with the ASan runtime preloaded into Python.  The
selection reaches every entry point of the C oracle: steps, runs and K-lag
solves (periodic, plate closures, E fields), the complex-step solve, the
adjoint step, solve and source, and the local gradient.  Any out-of-bounds
access, use after free or undefined operation aborts the child, which fails
this test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PINS = ("test_marched_solve_matches_fourier_closed_form or test_adjoint_step_is_the_transpose or "
        "test_plate_adjoint_is_transpose or test_plate_marched_solve_matches_sparse or "
        "test_E_scalar_gradient_matches_fad or test_cv_adjoint or test_cbar_and_two_mode or "
        "test_exact_fit")


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_address_and_undefined_behaviour_sanitizers():
    from oracle import build
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = build.build(force=True, sanitize=True)
    env = dict(os.environ, SLBM_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", PINS]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr, tail
    assert "runtime error" not in r.stderr, tail
