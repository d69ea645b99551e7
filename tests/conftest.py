import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def pytest_sessionstart(session):
    """A fresh checkout has no built library: build it once (hipcc for gfx950) before any test imports it."""
    lib = os.path.join(ROOT, "paper_1201_3114_amd", "liblorenz_cipher.so")
    if os.path.exists(lib):
        return
    import importlib.util

    spec = importlib.util.spec_from_file_location("_lz_build", os.path.join(ROOT, "paper_1201_3114_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.build()
