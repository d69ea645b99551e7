"""Builds the host-sanitizer test programs (run them on a machine with the GPU).

    python tests/native/build_sanitized.py

tests/test_gpu_host_sanitized.py calls build() itself, into a fresh directory, before each run.

The program is tests/native/host_sanitize.cpp linked with every library source compiled as in the package
build, plus AddressSanitizer and UndefinedBehaviorSanitizer: each sanitizer option is passed through -Xarch_host, so
the gfx950 kernels are the ordinary ones and only host code is instrumented.  Output:
_build/sanitize/host_asan_ubsan at the repository root, with a lsan.supp beside it for the allocations the
uninstrumented ROCm runtime keeps until exit.  (A ThreadSanitizer build of the same program runs its host-only
part, but under ThreadSanitizer the ROCm runtime finds no GPU, so the threads of the serving loop are covered by
the AddressSanitizer run and by the GPU tests, not by a race detector.)
"""
from __future__ import annotations

import importlib.util
import os
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(ROOT, "_build", "sanitize")

_spec = importlib.util.spec_from_file_location("_lz_build", os.path.join(ROOT, "paper_1201_3114_amd", "build.py"))
LB = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(LB)

HOST_DEBUG = ["-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer"]
KINDS = {
    "asan_ubsan": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-sanitize-recover=undefined"],
}
# leaks the ROCm runtime keeps until exit (it is not built with the sanitizer)
LSAN_SUPP = "leak:libamdhip64\nleak:libhsa-runtime64\nleak:libdrm\nleak:libamd_comgr\n"


def build(kind: str, out_dir: str = OUT) -> str:
    """Builds host_<kind> (and lsan.supp) in out_dir; returns the program's path."""
    flags = KINDS[kind]
    os.makedirs(out_dir, exist_ok=True)
    with tempfile.TemporaryDirectory(prefix="lzsan") as objdir:
        return _build_in(kind, flags, objdir, out_dir)


def _build_in(kind: str, flags: list[str], objdir: str, out_dir: str) -> str:
    cmds, objs = [], []
    srcs = [(os.path.join(LB.CSRC, s), s) for s in LB.SOURCES] + [(os.path.join(HERE, "host_sanitize.cpp"),
                                                                    "host_sanitize.cpp")]
    for path, name in srcs:
        obj = os.path.join(objdir, name + ".o")
        if name.endswith(".hip"):
            lang = ["-x", "hip"] + LB.DEVICE
        else:
            lang = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
        cmds.append([LB.HIPCC, *LB.COMMON, *HOST_DEBUG, *flags, *lang, "-c", path, "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as pool:
        list(pool.map(LB._run, cmds))
    exe = os.path.join(out_dir, "host_" + kind)
    LB._run([LB.HIPCC, f"--offload-arch={LB.ARCH}", *flags, *objs, "-o", exe, "-lpthread"])
    with open(os.path.join(out_dir, "lsan.supp"), "w") as f:
        f.write(LSAN_SUPP)
    return exe


if __name__ == "__main__":
    for k in sys.argv[1:] or sorted(KINDS):
        print(build(k))
