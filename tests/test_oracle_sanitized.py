"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle is built a second time with -fsanitize=address,undefined (host code;
no GPU code is involved) and all of its pinned tests run again in a child
process with the ASan runtime preloaded: every routine (kernel matrix,
products and row sums, Cholesky, CG, FGMRES, flexible CG, gradient, prediction,
Matern) executes there, and any out-of-bounds access, use of freed memory or
undefined behaviour aborts the run.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    try:
        out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_sanitizers():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime for gcc here")
    oracle.build(force=True, sanitize=True)
    env = dict(os.environ, LD_PRELOAD=rt, KRR_ORACLE_SANITIZE="1", OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle.py"), "-q", "-x",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    log = r.stdout + r.stderr
    assert r.returncode == 0, log[-4000:]
    assert "AddressSanitizer" not in log and "runtime error" not in log, log[-4000:]
    assert " passed" in log
