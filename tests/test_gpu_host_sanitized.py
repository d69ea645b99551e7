"""The library's host code under AddressSanitizer + UndefinedBehaviorSanitizer, on the GPU: argument checks,
key setup, the plain path, streams, batches, the serving loop (three submitting threads, one cancelling, one
polling; host and device buffers), the diagnostics and the unit checks, every result checked against the plain
path or a direct definition (tests/native/host_sanitize.cpp).  The program is built beforehand by
tests/native/build_sanitized.py (host code instrumented, kernels unchanged); the test is skipped when it is not
there."""
import os
import subprocess

import pytest

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "_build", "sanitize", "host_asan_ubsan")
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "SUMMARY: UndefinedBehaviorSanitizer")


def test_host_code_under_asan_ubsan():
    need_gpu()
    if not os.path.exists(EXE):
        pytest.skip("host_asan_ubsan not built (python tests/native/build_sanitized.py asan_ubsan)")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:exitcode=66", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([EXE], capture_output=True, text=True, env=env, timeout=240)
    out = run.stdout + run.stderr
    for rep in REPORTS:
        assert rep not in out, out[-6000:]
    assert run.returncode == 0 and "host sanitize: OK" in run.stdout, out[-6000:]
