"""Builds liblorenz_cipher.so (gfx950) in-tree with hipcc.

Every translation unit is compiled with -ffp-contract=off (the cipher's
binary64 arithmetic must be the exact IEEE operation sequence, no fused
multiply-add) and with packed fp32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblorenz_cipher.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("LZ_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-result"]
# loop headers on 64-byte boundaries: with one wave per SIMD nothing hides a fetch stall, and the
# unaligned Euler loop of the served kernel ran 25% slower than the same loop aligned
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-falign-loops=64"]
SOURCES = ["kernels.hip", "diag_hist.hip", "diag_lags.hip", "diag_fft.hip", "copy.hip", "noalloc.hip", "runtime.cpp",
           "server.cpp", "stream.cpp", "keysetup.cpp", "units.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[-1]}")
    return r


def build(verbose: bool = False) -> str:
    """Compiles every source and links the shared library; returns its path."""
    from concurrent.futures import ThreadPoolExecutor

    with tempfile.TemporaryDirectory(prefix="lzbuild") as tmp:
        cmds, objs = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            lang = ["-x", "hip"] + DEVICE if src.endswith(".hip") else ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
            cmds.append([HIPCC, *COMMON, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
            objs.append(obj)
            if verbose:
                print(" ".join(cmds[-1]))
        workers = max(1, min(len(cmds), os.cpu_count() or 1, 6))
        with ThreadPoolExecutor(max_workers=workers) as pool:
            list(pool.map(_run, cmds))  # re-raises the first failure
        tmp_lib = LIB + ".tmp"
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp_lib, "-lpthread"])
        os.replace(tmp_lib, LIB)
    return LIB


def assembly(out_dir: str) -> list[str]:
    """Writes the gfx950 assembly of the kernels (for instruction-mix checks)."""
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "kernels-gfx950.s")
    _run([HIPCC, *COMMON, "-x", "hip", *DEVICE, "--cuda-device-only", "-S", os.path.join(CSRC, "kernels.hip"),
          "-o", out])
    return [out]


if __name__ == "__main__":
    print(build(verbose=True))
