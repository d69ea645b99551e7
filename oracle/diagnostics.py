"""CPU oracle of the statistical analyses of Section 4 -- TEST INFRASTRUCTURE.

Only the test suite and the benchmark may import this module.  Each function
is the plain definition of the quantity, in exact integers where the quantity
is an integer sum, in binary64 otherwise.

* Frequency analysis: the histogram of the 256 byte values.
* Shannon entropy of that histogram (the formula S given in Section 4).
* Autocorrelation: lag sums of a byte sequence, and the circular
  autocorrelation matrix of a byte matrix (the text or image laid out row by
  row), normalised by the zero-lag value of the mean-removed data.
* The 2-D Fourier power spectrum of a byte matrix, |DFT2|^2 without shift or
  window.  The paper shows these only as figures; the exact normalisation,
  the circular (periodic) lags and the mean removal are this oracle's reading.
"""
from __future__ import annotations

import numpy as np


def histogram(x) -> np.ndarray:
    """Section 4, frequency analysis: count of each byte value 0..255."""
    x = np.asarray(x, dtype=np.uint8).ravel()
    return np.bincount(x, minlength=256).astype(np.int64)


def entropy(hist) -> float:
    """Section 4: S = -sum p_i log2 p_i over the byte values that occur (0 log 0 = 0)."""
    h = np.asarray(hist, dtype=np.float64)
    n = h.sum()
    if n == 0:
        return 0.0
    p = h[h > 0] / n
    return float(-(p * np.log2(p)).sum())


def lag_sums(x, max_lag: int) -> np.ndarray:
    """S_k = sum_{i < n-k} x_i x_{i+k} for k = 0..max_lag, exact (Section 4, autocorrelation)."""
    x = np.asarray(x, dtype=np.uint8).ravel().astype(np.int64)
    n = len(x)
    return np.array([int(np.dot(x[:n - k], x[k:])) if k < n else 0 for k in range(max_lag + 1)], dtype=np.int64)


def autocorrelation(x, max_lag: int) -> np.ndarray:
    """r_k = sum_{i<n-k} (x_i - m)(x_{i+k} - m) / sum_i (x_i - m)^2 for k = 0..max_lag.

    Multiplied through by n^2 every term is an integer: with T = sum x,
    A_k = sum_{i<n-k} x_i and B_k = sum_{i>=k} x_i the numerator is
    n^2 S_k - n T (A_k + B_k) + (n-k) T^2 and the denominator n^2 S_0 - n T^2,
    so each r_k is one correctly rounded ratio.  r_k = 0 for k >= n; NaN for a
    constant (or empty) sequence.
    """
    xs = np.asarray(x, dtype=np.uint8).ravel().astype(np.int64)
    n = len(xs)
    S = [int(v) for v in lag_sums(xs.astype(np.uint8), max_lag)]
    T = int(xs.sum())
    den = n * n * S[0] - n * T * T if n else 0
    if den == 0:
        return np.full(max_lag + 1, np.nan)
    out = np.empty(max_lag + 1)
    for k in range(max_lag + 1):
        if k >= n:
            out[k] = 0.0
            continue
        A = int(xs[:n - k].sum())
        B = int(xs[k:].sum())
        out[k] = (n * n * S[k] - n * T * (A + B) + (n - k) * T * T) / den
    return out


def circular_lag_sum(img, dx: int, dy: int) -> int:
    """sum_{x,y} X[x][y] * X[(x+dx) mod H][(y+dy) mod W], exact."""
    X = np.asarray(img, dtype=np.uint8).astype(np.int64)
    return int((X * np.roll(X, shift=(-dx, -dy), axis=(0, 1))).sum())


def autocorrelation_2d_at(img, dx: int, dy: int) -> float:
    """One entry of the circular autocorrelation matrix of the mean-removed image.

    With n = H*W, S1 = sum X, S2 = sum X^2 and S(d) the circular lag sum, the
    mean-removed lag sum is S(d) - S1^2/n, so the coefficient is
    (n S(d) - S1^2) / (n S2 - S1^2): a ratio of exact integers, rounded once.
    A constant image has no coefficient (NaN).
    """
    X = np.asarray(img, dtype=np.uint8).astype(np.int64)
    n = X.size
    s1 = int(X.sum())
    s2 = int((X * X).sum())
    den = n * s2 - s1 * s1
    if den == 0:
        return float("nan")
    num = n * circular_lag_sum(img, dx, dy) - s1 * s1
    return num / den  # Python int / int is correctly rounded


def autocorrelation_2d(img) -> np.ndarray:
    """The full circular autocorrelation matrix, entry (dx, dy) for every lag (brute force, small images)."""
    X = np.asarray(img, dtype=np.uint8)
    H, W = X.shape
    out = np.empty((H, W), dtype=np.float64)
    for dx in range(H):
        for dy in range(W):
            out[dx, dy] = autocorrelation_2d_at(X, dx, dy)
    return out


def power_spectrum_2d(img) -> np.ndarray:
    """Section 4, 2-D Fourier power spectrum: P[u][v] = |sum_{x,y} X[x][y] e^{-2 pi i (ux/H + vy/W)}|^2."""
    X = np.asarray(img, dtype=np.uint8).astype(np.float64)
    Z = np.fft.fft2(X)
    return Z.real * Z.real + Z.imag * Z.imag


def dft2_direct(img) -> np.ndarray:
    """The same DFT written as the double sum, for pinning the FFT on tiny images."""
    X = np.asarray(img, dtype=np.float64)
    H, W = X.shape
    Z = np.zeros((H, W), dtype=np.complex128)
    for u in range(H):
        for v in range(W):
            acc = 0j
            for x in range(H):
                for y in range(W):
                    acc += X[x, y] * np.exp(-2j * np.pi * ((u * x) / H + (v * y) / W))
            Z[u, v] = acc
    return Z
