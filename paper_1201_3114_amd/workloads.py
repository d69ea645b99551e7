"""Seeded synthetic inputs of the benchmark configurations.

Holds none of the cipher's arithmetic: only random bytes, printable-ASCII
passwords, message sizes, tamper offsets and arrival times, drawn from numpy's
PCG64 with fixed seeds, so the GPU path and the CPU oracle receive the same
inputs.  The paper measured on a book and an image that are not available;
uniform random bytes stand in for them, as the benchmark specification asks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

KiB, MiB = 1024, 1024 * 1024

# seeds of the five configurations
SEED = {"plain_64k": 100, "plain_64m": 101, "batch": 102, "batch_integrity": 103, "serve": 104, "sequential": 105,
        "serve_data": 106, "serve_sample": 107, "diagnostics": 108}


def password(rng: np.random.Generator, n: int) -> bytes:
    """n random printable-ASCII bytes (codes 32..126)."""
    return bytes(rng.integers(32, 127, n, dtype=np.uint8))


def random_bytes(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.integers(0, 256, n, dtype=np.uint8)


def plain(name: str = "plain_64k"):
    """One message and one password: 64 KiB with 16-byte password, or 64 MiB with 32-byte password."""
    n, npw = {"plain_64k": (64 * KiB, 16), "plain_64m": (64 * MiB, 32)}[name]
    rng = np.random.default_rng(SEED[name])
    P = random_bytes(rng, n)
    pw = password(rng, npw)
    return P, pw


def batch_sizes(rng: np.random.Generator, count: int, lo: int = KiB, hi: int = MiB) -> np.ndarray:
    """Sizes log-uniform in [lo, hi]."""
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(np.int64)


@dataclass
class BatchWorkload:
    sizes: np.ndarray        # plaintext lengths
    passwords: list          # bytes, 8..64 each
    data: np.ndarray         # all plaintexts end to end
    offsets: np.ndarray      # start of message i in data


def batch(count: int = 4096, seed: int | None = None, lo: int = KiB, hi: int = MiB) -> BatchWorkload:
    """Messages with log-uniform sizes, uniform random bytes, own 8..64-byte password each."""
    rng = np.random.default_rng(SEED["batch"] if seed is None else seed)
    sizes = batch_sizes(rng, count, lo, hi)
    pws = [password(rng, int(k)) for k in rng.integers(8, 65, count)]
    data = random_bytes(rng, int(sizes.sum()))
    offs = np.zeros(count, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    return BatchWorkload(sizes, pws, data, offs)


def tamper_plan(ct_lens, frac: float = 0.1, seed: int | None = None):
    """floor(frac * count) ciphertexts chosen without replacement, each with one byte at a
    random offset (tag included) XORed with a random nonzero value: (index, offset, xor)."""
    rng = np.random.default_rng(SEED["batch_integrity"] if seed is None else seed)
    count = len(ct_lens)
    k = int(math.floor(frac * count))
    idx = np.sort(rng.choice(count, size=k, replace=False))
    offs = np.array([rng.integers(0, int(ct_lens[i])) for i in idx], dtype=np.int64)
    vals = rng.integers(1, 256, k).astype(np.uint8)
    return idx, offs, vals


# Offered loads of the serving runs, fixed: QPS = load x capacity / mean request size, with the
# capacity 0.90 GB/s per direction of the plain path at 64 MiB on one MI355X (encrypt 0.8998 GB/s)
# and the mean request size 50,115.4 bytes of the 200,000-request trace below (seed 104).
SERVE_CAPACITY_GBPS = 0.90
SERVE_MEAN_REQUEST_BYTES = 50115.4
SERVE_QPS = {load: round(load * SERVE_CAPACITY_GBPS * 1e9 / SERVE_MEAN_REQUEST_BYTES, 1)
             for load in (0.3, 0.5, 0.7, 0.9)}


@dataclass
class ServeTrace:
    arrival_s: np.ndarray    # seconds from the trace start
    decrypt: np.ndarray      # 0 = encrypt, 1 = decrypt
    sizes: np.ndarray        # plaintext lengths
    passwords: list


def serve_trace(count: int = 200_000, qps: float = 1000.0, median: int = 16 * KiB, sigma: float = 1.5,
                lo: int = 64, hi: int = 16 * MiB, seed: int | None = None) -> ServeTrace:
    """Poisson arrivals at qps, 50/50 encrypt/decrypt, lognormal sizes clamped to [lo, hi],
    16..64-byte printable passwords."""
    rng = np.random.default_rng(SEED["serve"] if seed is None else seed)
    gaps = rng.exponential(1.0 / qps, count)
    arrival = np.cumsum(gaps) - gaps[0]
    dec = rng.integers(0, 2, count).astype(np.int8)
    sizes = np.clip(np.floor(rng.lognormal(math.log(median), sigma, count)), lo, hi).astype(np.int64)
    pws = [password(rng, int(k)) for k in rng.integers(16, 65, count)]
    return ServeTrace(arrival, dec, sizes, pws)
