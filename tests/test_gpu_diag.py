"""Section 4 diagnostics on the GPU (byte histogram, lag sums / autocorrelation) vs numpy, exactly."""
import numpy as np
import pytest

import oracle
from gpu_util import host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lz():
    need_gpu()
    import paper_1201_3114_amd as lz

    return lz


@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 1000, 65537, 3_000_001])
def test_histogram_exact(lz, n):
    import torch

    rng = np.random.default_rng(80 + n)
    x = rng.integers(0, 256, n, dtype=np.uint8)
    ctx = lz.Context(0)
    d = to_dev(x) if n else torch.zeros(0, dtype=torch.uint8, device="cuda")
    h = host(lz.histogram(ctx, d)).astype(np.int64)
    assert np.array_equal(h, np.bincount(x, minlength=256))
    if n > 1:  # misaligned start
        h2 = host(lz.histogram(ctx, d[1:])).astype(np.int64)
        assert np.array_equal(h2, np.bincount(x[1:], minlength=256))


@pytest.mark.parametrize("n,L", [(0, 5), (1, 0), (10, 20), (5000, 300), (200_003, 256), (1_000_000, 1000)])
def test_lag_sums_exact(lz, n, L):
    import torch

    rng = np.random.default_rng(90 + n)
    x = rng.integers(0, 256, n, dtype=np.uint8)
    ctx = lz.Context(0)
    d = to_dev(x) if n else torch.zeros(0, dtype=torch.uint8, device="cuda")
    got = host(lz.lag_sums(ctx, d, L)).astype(np.int64)
    xi = x.astype(np.int64)
    want = np.array([int(np.dot(xi[:n - k], xi[k:])) if k < n else 0 for k in range(L + 1)], dtype=np.int64)
    assert np.array_equal(got, want)


def test_autocorrelation_and_entropy_of_ciphertext(lz):
    """Sanity only: a low-entropy plaintext's ciphertext is near-uniform and uncorrelated (Section 4)."""
    rng = np.random.default_rng(95)
    P = rng.integers(64, 96, 1 << 16, dtype=np.uint8)
    ctx = lz.Context(0)
    C = ctx.encrypt(to_dev(P), b"123456")[:-24].contiguous()
    assert np.array_equal(host(C), oracle.encrypt(b"123456", P, nthreads=8)[:-24])
    S = lz.entropy(lz.histogram(ctx, C))
    assert S > 7.99
    r = lz.autocorrelation(ctx, C, 64)
    xc = host(C).astype(np.float64) - host(C).mean()
    want = np.array([np.dot(xc[:len(xc) - k], xc[k:]) for k in range(65)]) / np.dot(xc, xc)
    assert np.allclose(r, want, rtol=0, atol=1e-9)
    assert abs(r[0] - 1.0) < 1e-12
    assert np.max(np.abs(r[1:])) < 0.03
