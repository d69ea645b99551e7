"""The library's host code under AddressSanitizer + UndefinedBehaviorSanitizer, on the GPU: argument checks,
key setup, the plain path, streams, batches, the serving loop (three submitting threads, one cancelling, one
polling; host and device buffers), the diagnostics and the unit checks, every result checked against the plain
path or a direct definition (tests/native/host_sanitize.cpp).  The test builds the program from the current
sources first (tests/native/build_sanitized.py: host code instrumented, kernels unchanged), so it never runs a
stale or missing binary."""
import importlib.util
import os
import subprocess

import pytest

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "SUMMARY: UndefinedBehaviorSanitizer")


def _builder():
    spec = importlib.util.spec_from_file_location("_lz_build_sanitized", os.path.join(HERE, "native",
                                                                                        "build_sanitized.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_host_code_under_asan_ubsan(tmp_path):
    need_gpu()
    say("building host_asan_ubsan")
    exe = _builder().build("asan_ubsan", str(tmp_path))
    say("running", exe)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:exitcode=66", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=240)
    out = run.stdout + run.stderr
    for rep in REPORTS:
        assert rep not in out, out[-6000:]
    assert run.returncode == 0 and "host sanitize: OK" in run.stdout, out[-6000:]
