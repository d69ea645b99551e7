"""Helpers shared by the GPU tests (no cipher arithmetic here)."""
import os
import sys

import numpy as np
import pytest

ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU on this machine")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(arr):
    import torch

    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.uint8)).cuda()


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()
