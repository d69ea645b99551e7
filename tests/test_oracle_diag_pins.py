"""Pins of the Section 4 diagnostics oracle (oracle/diagnostics.py) against closed forms,
brute force and an independent route (Wiener-Khinchin through the FFT)."""
import math

import numpy as np
import pytest

from oracle import diagnostics as dg


def test_histogram_and_entropy_closed_forms():
    assert dg.histogram(np.arange(256, dtype=np.uint8)).tolist() == [1] * 256
    assert dg.entropy(dg.histogram(np.arange(256, dtype=np.uint8))) == 8.0  # S_max = 8
    assert dg.entropy(dg.histogram(np.full(1000, 7, np.uint8))) == 0.0
    assert dg.entropy(dg.histogram(np.array([3, 9] * 50, np.uint8))) == 1.0
    assert dg.entropy(np.zeros(256, np.int64)) == 0.0
    # p = (1/2, 1/4, 1/4) -> 1.5 bits
    assert dg.entropy(dg.histogram(np.array([1, 1, 2, 3], np.uint8))) == 1.5
    h = dg.histogram(np.array([0, 255, 255, 17], np.uint8))
    assert h[0] == 1 and h[255] == 2 and h[17] == 1 and h.sum() == 4


def test_lag_sums_brute_force():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, 57, dtype=np.uint8)
    got = dg.lag_sums(x, 70)
    xs = [int(v) for v in x]
    for k in range(71):
        assert got[k] == sum(xs[i] * xs[i + k] for i in range(len(xs) - k))
    assert dg.lag_sums(np.ones(10, np.uint8), 12).tolist() == [10 - k if k < 10 else 0 for k in range(13)]


def _acf1_brute(x, L):
    """r_k of the mean-removed sequence from its definition, in exact rationals."""
    from fractions import Fraction
    xs = [int(v) for v in x]
    n = len(xs)
    m = Fraction(sum(xs), n)
    den = sum((v - m) ** 2 for v in xs)
    return [float(sum((xs[i] - m) * (xs[i + k] - m) for i in range(n - k)) / den) for k in range(L + 1)]


def test_autocorrelation_1d():
    # alternating sequence: r_k = (-1)^k (n-k)/n, from the definition and from the oracle
    x = np.array([10, 30] * 20, np.uint8)
    want = [(-1) ** k * (40 - k) / 40 for k in range(7)]
    assert _acf1_brute(x, 6) == want
    assert dg.autocorrelation(x, 6).tolist() == want
    rng = np.random.default_rng(4)
    y = rng.integers(0, 256, 45, dtype=np.uint8)
    got = dg.autocorrelation(y, 50)
    assert got[:45].tolist() == _acf1_brute(y, 44)
    assert (got[45:] == 0).all() and got[0] == 1.0
    assert np.isnan(dg.autocorrelation(np.full(9, 4, np.uint8), 3)).all()
    assert np.isnan(dg.autocorrelation(np.zeros(0, np.uint8), 3)).all()


def test_autocorrelation_2d_closed_forms():
    H, W = 6, 8
    xx, yy = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    checker = (100 + 50 * ((xx + yy) % 2)).astype(np.uint8)
    A = dg.autocorrelation_2d(checker)
    assert np.array_equal(A, ((-1.0) ** (xx + yy)))
    stripes = (7 + 200 * (xx % 2)).astype(np.uint8)
    assert np.array_equal(dg.autocorrelation_2d(stripes), (-1.0) ** xx)
    assert np.isnan(dg.autocorrelation_2d(np.full((3, 4), 9, np.uint8))).all()


def test_autocorrelation_2d_invariants_and_fft_route():
    rng = np.random.default_rng(5)
    X = rng.integers(0, 256, (9, 14), dtype=np.uint8)
    A = dg.autocorrelation_2d(X)
    assert A[0, 0] == 1.0
    assert np.abs(A).max() <= 1.0
    # A[d] = A[-d] (circular symmetry)
    assert np.array_equal(A, np.roll(A[::-1, ::-1], shift=(1, 1), axis=(0, 1)))
    # Wiener-Khinchin through numpy's FFT, an independent route
    Xc = X.astype(np.float64) - X.mean()
    G = np.fft.ifft2(np.abs(np.fft.fft2(Xc)) ** 2).real
    assert np.allclose(A, G / G[0, 0], rtol=0, atol=1e-13)
    # one entry from the mean-removed definition in exact rationals
    from fractions import Fraction
    xs = [[int(v) for v in row] for row in X]
    m = Fraction(sum(map(sum, xs)), X.size)
    num = sum((xs[x][y] - m) * (xs[(x + 2) % 9][(y + 5) % 14] - m) for x in range(9) for y in range(14))
    den = sum((v - m) ** 2 for row in xs for v in row)
    assert dg.autocorrelation_2d_at(X, 2, 5) == float(num / den)


def test_power_spectrum_closed_forms():
    H, W = 8, 6
    P = dg.power_spectrum_2d(np.full((H, W), 3, np.uint8))
    want = np.zeros((H, W))
    want[0, 0] = (3 * H * W) ** 2
    assert np.allclose(P, want, rtol=0, atol=1e-9)
    imp = np.zeros((H, W), np.uint8)
    imp[2, 5] = 7
    assert np.allclose(dg.power_spectrum_2d(imp), 49.0, rtol=0, atol=1e-11)
    row = np.zeros((H, W), np.uint8)
    row[0, :] = 1
    want = np.zeros((H, W))
    want[:, 0] = W ** 2
    assert np.allclose(dg.power_spectrum_2d(row), want, rtol=0, atol=1e-11)
    xx, yy = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    chk = ((xx + yy) % 2).astype(np.uint8)
    want = np.zeros((H, W))
    want[0, 0] = want[H // 2, W // 2] = (H * W / 2) ** 2
    assert np.allclose(dg.power_spectrum_2d(chk), want, rtol=0, atol=1e-9)


def test_power_spectrum_direct_sum_parseval_symmetry():
    rng = np.random.default_rng(6)
    X = rng.integers(0, 256, (5, 7), dtype=np.uint8)
    P = dg.power_spectrum_2d(X)
    Z = dg.dft2_direct(X)
    assert np.allclose(P, np.abs(Z) ** 2, rtol=1e-12, atol=1e-6)
    x = X.astype(np.float64)
    assert math.isclose(P.sum(), X.size * (x * x).sum(), rel_tol=1e-13)
    assert np.allclose(P, np.roll(P[::-1, ::-1], shift=(1, 1), axis=(0, 1)), rtol=1e-12, atol=1e-6)


@pytest.mark.parametrize("mistake", ["sign", "transpose", "no_mean"])
def test_planted_mistakes_fail_a_pin(mistake):
    """Each plausible slip in the 2-D routines trips one of the pins above."""
    H, W = 6, 8
    xx, yy = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    if mistake == "sign":  # inverse instead of forward transform: same power, so check a phase pin instead
        imp = np.zeros((H, W), np.uint8)
        imp[1, 0] = 1
        Z = np.fft.ifft2(imp) * H * W
        assert not np.allclose(Z, dg.dft2_direct(imp))
    elif mistake == "transpose":
        row = np.zeros((H, W), np.uint8)
        row[0, :] = 1
        # H and W swapped in the exponent
        u, v, x, y = np.meshgrid(np.arange(H), np.arange(W), np.arange(H), np.arange(W), indexing="ij")
        Z = (row[x, y] * np.exp(-2j * np.pi * (u * x / W + v * y / H))).sum(axis=(2, 3))
        wrong = np.abs(Z) ** 2
        want = np.zeros((H, W))
        want[:, 0] = W ** 2
        assert not np.allclose(wrong, want)
    else:
        stripes = (7 + 200 * (xx % 2)).astype(np.uint8)
        X = stripes.astype(np.int64)
        raw = np.array([[(X * np.roll(X, (-a, -b), (0, 1))).sum() for b in range(W)] for a in range(H)], float)
        assert not np.array_equal(raw / raw[0, 0], (-1.0) ** xx)
