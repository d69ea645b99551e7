"""Section 4 diagnostics on the GPU vs the oracle (oracle/diagnostics.py).

Integer results (histogram, lag sums) are compared exactly.  Floating-point
results use error bounds derived from the arithmetic, written in each test
(eps = 2^-53 is the unit roundoff of binary64).
"""
import numpy as np
import pytest

import oracle
from oracle import diagnostics as dg
from gpu_util import host, need_gpu, say, to_dev

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def lz():
    need_gpu()
    import paper_1201_3114_amd as lz

    return lz


@pytest.fixture(scope="module")
def ctx(lz):
    return lz.Context(0)


def _dev(x):
    import torch

    return to_dev(x) if x.size else torch.zeros(0, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 1000, 65537, 3_000_001])
def test_histogram_exact(lz, ctx, n):
    rng = np.random.default_rng(80 + n)
    x = rng.integers(0, 256, n, dtype=np.uint8)
    d = _dev(x)
    h = host(lz.histogram(ctx, d)).astype(np.int64)
    assert np.array_equal(h, dg.histogram(x))
    if n > 1:  # misaligned start
        assert np.array_equal(host(lz.histogram(ctx, d[1:])).astype(np.int64), dg.histogram(x[1:]))


@pytest.mark.parametrize("kind", ["constant", "text", "two_values"])
def test_histogram_skewed_exact(lz, ctx, kind):
    """Inputs where many lanes see the same byte value (the case the interleaved LDS copies are for)."""
    rng = np.random.default_rng(82)
    n = 5_000_003
    if kind == "constant":
        x = np.full(n, 32, np.uint8)
    elif kind == "text":
        x = rng.choice(np.frombuffer(b"       eeeetttaaoinshrdlu.,\n", np.uint8), n)
    else:
        x = rng.choice(np.array([0, 255], np.uint8), n, p=[0.9, 0.1])
    d = _dev(x)
    assert np.array_equal(host(lz.histogram(ctx, d)).astype(np.int64), dg.histogram(x))
    assert np.array_equal(host(lz.histogram(ctx, d[7:])).astype(np.int64), dg.histogram(x[7:]))


def test_histogram_calls_in_a_row_on_two_streams(lz, ctx):
    """Each call leaves the context's merge copies and workgroup counter cleared for the next: calls of one
    workgroup and of hundreds, queued back to back on two streams, each equal their byte counts."""
    import torch

    rng = np.random.default_rng(83)
    sizes = [1, 100, 16384, 16385, 3_000_001, 20_000_000, 0, 5]
    xs = [rng.integers(0, 256, n, dtype=np.uint8) for n in sizes]
    ds = [_dev(x) if len(x) else torch.zeros(0, dtype=torch.uint8, device="cuda") for x in xs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for rep in range(3):
        for i, d in enumerate(ds):
            outs.append((i, lz.histogram(ctx, d, stream=streams[(i + rep) % 2])))
    torch.cuda.synchronize()
    for i, h in outs:
        assert np.array_equal(host(h).astype(np.int64), dg.histogram(xs[i])), sizes[i]


@pytest.mark.parametrize("kind", ["empty", "one", "two", "uniform", "skewed", "all"])
def test_entropy(lz, ctx, kind):
    rng = np.random.default_rng(81)
    x = {"empty": np.zeros(0, np.uint8), "one": np.full(100, 5, np.uint8),
         "two": np.array([1, 2] * 500, np.uint8), "uniform": rng.integers(0, 256, 1 << 20, dtype=np.uint8),
         "skewed": (rng.exponential(20, 200_000).clip(0, 255)).astype(np.uint8),
         "all": np.arange(256 * 7, dtype=np.int64).astype(np.uint8)}[kind]
    S = lz.entropy(ctx, lz.histogram(ctx, _dev(x)))
    want = dg.entropy(dg.histogram(x))
    # 256 terms, each within a few ulps (log2 and one division), summed in another order: |dS| <= 256 * 16 eps * 8
    assert abs(S - want) <= 256 * 16 * EPS * 8, (S, want)
    if kind in ("empty", "one"):
        assert S == 0.0
    if kind == "two":
        assert S == 1.0


@pytest.mark.parametrize("n,L", [(0, 5), (1, 0), (10, 20), (5000, 300), (200_003, 256), (1_000_000, 1000),
                                 (50_000, 4095), (50_000, 4096), (30_001, 16384), (3, 16384), (15, 1), (16, 16),
                                 (65_537, 127), (98_309, 511), (100_003, 8191), (100_003, 8192), (77_777, 12289),
                                 (20_000, 16383), (31, 255), (33, 32), (64, 33), (2_000_037, 256), (1_048_576, 224),
                                 (32_800, 225), (40_000, 257)])
def test_lag_sums_exact(lz, ctx, n, L):
    """The lags run on the matrix cores (bytes offset by -128, then corrected exactly): up to lag 256 on
    32-byte rows in one launch (1 to 9 column tiles), beyond that in windows of 4096 lags, one launch
    each, whose sums the correction kernel takes window by window. Tile and window edges, lags beyond n
    and partial rows are compared exactly."""
    rng = np.random.default_rng(90 + n)
    x = rng.integers(0, 256, n, dtype=np.uint8)
    got = host(lz.lag_sums(ctx, _dev(x), L)).astype(np.int64)
    assert np.array_equal(got, dg.lag_sums(x, L))


def test_lag_sums_and_histograms_in_a_row_on_two_streams(lz, ctx):
    """The lag sums below 4096 and the histogram share the context's merge copies, which each call clears:
    calls with lags falling and rising (300, 100, 300, 4095, 0, ...), interleaved with histograms and queued
    back to back on two streams, each equal their exact values."""
    import torch

    rng = np.random.default_rng(97)
    cases = [(200_000, 300), (5_000, 100), (1_000_000, 300), (70_000, 4095), (33, 0), (9_999, 17), (64, 4095)]
    xs = [rng.integers(0, 256, n, dtype=np.uint8) for n, _ in cases]
    ds = [_dev(x) for x in xs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for rep in range(2):
        for i, (d, (n, L)) in enumerate(zip(ds, cases)):
            st = streams[(i + rep) % 2]
            outs.append(("sums", i, lz.lag_sums(ctx, d, L, stream=st)))
            outs.append(("hist", i, lz.histogram(ctx, d, stream=streams[(i + rep + 1) % 2])))
    torch.cuda.synchronize()
    for kind, i, t in outs:
        want = dg.lag_sums(xs[i], cases[i][1]) if kind == "sums" else dg.histogram(xs[i])
        assert np.array_equal(host(t).astype(np.int64), want), (kind, cases[i])


def _ramp_histogram(n):
    """Byte counts of x_i = i mod 256, i < n (closed form)."""
    return np.array([n // 256 + (1 if v < n % 256 else 0) for v in range(256)], dtype=np.int64)


def _ramp_lag_sum(n, k):
    """S_k of x_i = i mod 256, i < n: (n - k) // 256 whole periods of the pairs (a, (a + k) mod 256), then
    the first (n - k) mod 256 pairs of one more (closed form, Python integers)."""
    if k >= n:
        return 0
    q, r = divmod(n - k, 256)
    per = [a * ((a + k) % 256) for a in range(256)]
    return q * sum(per) + sum(per[:r])


def test_histogram_and_lag_sums_past_4GiB(lz, ctx):
    """Maximum sizes: 2^32 + 4099 bytes of the ramp x_i = i mod 256, so bin counts and lag sums pass 2^32 and
    the byte index passes 32 bits, checked exactly against closed forms (themselves checked against the
    oracle on a short ramp first)."""
    import torch

    short = np.arange(70_001, dtype=np.int64).astype(np.uint8)
    assert np.array_equal(_ramp_histogram(len(short)), dg.histogram(short))
    ls = dg.lag_sums(short, 300)
    assert all(int(ls[k]) == _ramp_lag_sum(len(short), k) for k in range(301))
    n = (1 << 32) + 4099
    big = torch.arange(256, dtype=torch.uint8, device="cuda").repeat(n // 256 + 1)[:n]
    assert big.is_contiguous() and big.numel() == n
    say("histogram and lag sums of", n, "bytes")
    h = host(lz.histogram(ctx, big)).astype(np.int64)
    assert np.array_equal(h, _ramp_histogram(n))
    for L in (256, 300):  # 32-byte rows (512 tasks per workgroup, partial sums flushed on the way), 16-byte rows
        got = host(lz.lag_sums(ctx, big, L))
        for k in range(L + 1):
            assert int(got[k]) == _ramp_lag_sum(n, k), (L, k)
    got = host(lz.lag_sums(ctx, big, 4200))  # two lag windows
    for k in (0, 1, 255, 4095, 4096, 4097, 4111, 4199, 4200):
        assert int(got[k]) == _ramp_lag_sum(n, k), k
    del big
    torch.cuda.empty_cache()


@pytest.mark.parametrize("L", [0, 100, 256, 4095])
def test_lag_sums_unaligned_and_many_tasks(lz, ctx, L):
    """A data pointer off 4-byte alignment (byte loads when staging), and 40 MiB + 3 bytes: more
    tasks than workgroups on a 256-CU device, so workgroups take several tasks in turn (with the
    next task's loads in flight for lags up to 256).
    The large case is checked exactly at sampled lags (a lag sum is a plain dot product)."""
    import torch

    rng = np.random.default_rng(95 + L)
    x = rng.integers(0, 256, 300_001, dtype=np.uint8)
    d = _dev(x)
    got = host(lz.lag_sums(ctx, d[3:], L)).astype(np.int64)
    assert np.array_equal(got, dg.lag_sums(x[3:], L))
    n = 40 * (1 << 20) + 3
    big = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda",
                        generator=torch.Generator(device="cuda").manual_seed(96 + L))
    got = host(lz.lag_sums(ctx, big, L)).astype(np.int64)
    xb = host(big).astype(np.int64)
    for k in sorted({0, min(1, L), L // 2, L}):
        assert got[k] == int(np.dot(xb[: n - k], xb[k:])), k


@pytest.mark.parametrize("n,L,kind", [(0, 4, "rand"), (1, 3, "rand"), (7, 12, "rand"), (40, 6, "alt"),
                                      (5000, 300, "rand"), (100_000, 700, "text"), (1000, 5, "const"),
                                      (300_001, 2000, "rand"), (20_000, 16384, "rand"), (2_000_003, 256, "text"),
                                      (200, 256, "alt")])
def test_autocorrelation_1d(lz, ctx, n, L, kind):
    """Up to lag 256 the correction kernel also normalises; past it a separate kernel does."""
    rng = np.random.default_rng(91 + n)
    if kind == "alt":
        x = np.array([10, 30] * (n // 2), np.uint8)
    elif kind == "const":
        x = np.full(n, 77, np.uint8)
    elif kind == "text":  # letters and spaces, strongly non-uniform
        x = rng.choice(np.frombuffer(b"etaoin shrdlu       ", np.uint8), n)
    else:
        x = rng.integers(0, 256, n, dtype=np.uint8)
    got = host(lz.autocorrelation(ctx, _dev(x), L))
    want = dg.autocorrelation(x, L)
    if kind == "const" or n == 0 or (n == 1):
        assert np.isnan(got).all() and np.isnan(want).all()
        return
    xs = x.astype(np.float64)
    S0, T = float((xs * xs).sum()), float(xs.sum())
    # every term of num and den is at most S0 in size and carries a few roundings: |dr| <= 64 eps S0 / den
    tol = 64 * EPS * S0 / (S0 - T * T / n)
    assert np.max(np.abs(got - want)) <= tol, (np.max(np.abs(got - want)), tol)
    if kind == "alt":
        assert np.allclose(got, [(-1) ** k * max(n - k, 0) / n for k in range(L + 1)], rtol=0, atol=tol)


@pytest.mark.parametrize("n,kind", [(1000, "rand"), (1_000_003, "text"), (257, "rand"), (100, "rand")])
def test_autocorrelation_fused_normalisation_is_bit_identical(lz, ctx, n, kind):
    """The coefficients up to lag 256 come from the correction kernel of the one-launch lag sums (the
    fused normalisation); asking for lag 257 runs the windowed lag sums and the separate normalisation
    kernel.  Both take the same binary64 operations on the same exact sums, so r_0..r_256 agree bit for
    bit (n = 100: the lags at or past n are exactly 0 on both)."""
    rng = np.random.default_rng(130 + n)
    if kind == "text":
        x = rng.choice(np.frombuffer(b"etaoin shrdlu       ", np.uint8), n)
    else:
        x = rng.integers(0, 256, n, dtype=np.uint8)
    d = _dev(x)
    fused = host(lz.autocorrelation(ctx, d, 256))
    windowed = host(lz.autocorrelation(ctx, d, 257))
    assert fused.view(np.uint64).tolist() == windowed[:257].view(np.uint64).tolist()


def _dz_max(x):
    """Bound on the error of each DFT value Z[u][v] after the two passes.  A direct pass sums N
    complex products w x with |w| = 1 in fused multiply-adds, 2N roundings per real component, so
    each component is off by at most 2N eps sum|x| (twiddle errors add a few eps more); the complex
    magnitude adds sqrt 2 twice over.  Both passes: |dZ| <= 4 (h + w + 4) eps S1, S1 = sum x.
    A radix-2 FFT pass (power-of-two lengths) is within the same bound: each of its log2 N stages
    adds at most about 6 eps times the magnitude of partial sums whose moduli add up to at most
    sum|x|, so |dZ| <= 6 (log2 h + log2 w) eps S1 < 4 (h + w + 4) eps S1."""
    h, w = x.shape
    return 4 * (h + w + 4) * EPS * float(x.astype(np.float64).sum())


def _power_tol(x):
    """|dP| <= 2 |Z| |dZ| + |dZ|^2 + 2 eps |Z|^2 with |Z| <= S1."""
    S1 = float(x.astype(np.float64).sum())
    dz = _dz_max(x)
    return 2 * S1 * dz + dz * dz + 2 * EPS * S1 * S1


@pytest.mark.parametrize("h,w", [(1, 1), (1, 37), (29, 1), (2, 2), (8, 8), (64, 64), (67, 131), (128, 200),
                                 (512, 512), (3, 4096), (4096, 3), (2048, 2048), (2, 8192), (1000, 24),
                                 (768, 960), (45, 81), (7, 250), (4050, 2), (1024, 1024), (1024, 7), (6, 1024),
                                 (1024, 1), (1024, 4093), (1009, 1009)])
def test_power_spectrum_2d(lz, ctx, h, w):
    """All routes of a pass: the 1024-point pass of one wave per column (1024; with 1, 6, 7, 1024 and
    4093 columns, so some workgroups have idle waves), the power-of-two FFT up to 4096 (2, 8, 64, 128,
    512, 2048, 4096, and the 1 x 1 identity), the mixed-radix FFT for lengths with no prime factor above
    5 (3, 24, 45, 81, 200, 250, 768, 960, 1000, 4050: radix 5, 3, 4, 2 stages, 4050 needing 130 KB of
    LDS), and the direct DFT on the matrix cores for the others (7, 29, 37, 67, 131, 1009, 4093) and for
    8192, above the FFTs' limit; several cases mix them.  The first pass keeps indices up to h/2 of its
    column transforms and the second writes the other rows as mirror images, so odd and even h, and
    h = 1 and 2 (no mirror rows), are all here."""
    rng = np.random.default_rng(100 + h * 7 + w)
    x = rng.integers(0, 256, (h, w), dtype=np.uint8)
    say("power spectrum", h, w)
    got = host(lz.power_spectrum_2d(ctx, to_dev(x.ravel()).view(h, w)))
    want = dg.power_spectrum_2d(x)
    err = np.max(np.abs(got - want))
    assert err <= _power_tol(x), (err, _power_tol(x))
    # the zero frequency is exactly (sum x)^2 up to the same bound
    assert abs(got[0, 0] - float(x.astype(np.int64).sum()) ** 2) <= _power_tol(x)


def test_power_spectrum_2d_closed_forms(lz, ctx):
    H, W = 96, 70
    xx, yy = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    chk = ((xx + yy) % 2).astype(np.uint8)
    got = host(lz.power_spectrum_2d(ctx, to_dev(chk.ravel()).view(H, W)))
    want = np.zeros((H, W))
    want[0, 0] = want[H // 2, W // 2] = (H * W / 2) ** 2
    assert np.max(np.abs(got - want)) <= _power_tol(chk)
    imp = np.zeros((H, W), np.uint8)
    imp[5, 9] = 200
    got = host(lz.power_spectrum_2d(ctx, to_dev(imp.ravel()).view(H, W)))
    assert np.max(np.abs(got - 40000.0)) <= _power_tol(imp)


def _acf2_tol(x):
    """A = G / den, G the inverse DFT of P' (the spectrum with the zero frequency removed) and
    den = n S2 - S1^2, which is also sum P' (Parseval).  Errors entering G:
      from dP': sum |dP'| <= 2 dZ sum|Z| + n dZ^2 + 2 eps sum|Z|^2, with sum|Z| <= n sqrt(S2)
                (Cauchy-Schwarz and Parseval: sum|Z|^2 = n S2);
      from the inverse passes: 4 (h + w + 4) eps sum|P'| = 4 (h + w + 4) eps den;
    and the final division adds eps."""
    h, w = x.shape
    n = h * w
    xs = x.astype(np.int64)
    S1, S2 = int(xs.sum()), int((xs * xs).sum())
    den = float(n * S2 - S1 * S1)
    dz = _dz_max(x)
    from_p = 2 * dz * n * np.sqrt(S2) + n * dz * dz + 2 * EPS * n * S2
    return from_p / den + 4 * (h + w + 4) * EPS + 2 * EPS


@pytest.mark.parametrize("h,w", [(1, 2), (2, 1), (5, 7), (16, 16), (24, 40), (33, 17), (1, 300)])
def test_autocorrelation_2d_full(lz, ctx, h, w):
    rng = np.random.default_rng(110 + h * 5 + w)
    x = rng.integers(0, 256, (h, w), dtype=np.uint8)
    got = host(lz.autocorrelation_2d(ctx, to_dev(x.ravel()).view(h, w)))
    want = dg.autocorrelation_2d(x)
    err = np.max(np.abs(got - want))
    assert err <= _acf2_tol(x), (err, _acf2_tol(x))


def test_autocorrelation_2d_closed_forms_and_constant(lz, ctx):
    H, W = 40, 64
    xx, yy = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    chk = (100 + 50 * ((xx + yy) % 2)).astype(np.uint8)
    got = host(lz.autocorrelation_2d(ctx, to_dev(chk.ravel()).view(H, W)))
    assert np.max(np.abs(got - (-1.0) ** (xx + yy))) <= _acf2_tol(chk)
    # a constant matrix has no coefficient, whichever route its first pass takes (direct DFT, the
    # 1024-point pass, radix-4 and mixed-radix FFTs): n S2 = S1^2 exactly in the moment sums
    for shape in ((9, 13), (1024, 1024), (64, 64), (40, 24)):
        const = np.full(shape, 42, np.uint8)
        assert np.isnan(host(lz.autocorrelation_2d(ctx, to_dev(const.ravel()).view(*shape)))).all(), shape
    one = np.full((1, 1), 3, np.uint8)
    assert np.isnan(host(lz.autocorrelation_2d(ctx, to_dev(one.ravel()).view(1, 1)))).all()


def test_autocorrelation_2d_sampled_large(lz, ctx):
    """A 512 x 768 image-like matrix (smooth gradient + noise), checked at sampled lags."""
    rng = np.random.default_rng(120)
    H, W = 512, 768
    xx, yy = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    img = ((xx * 255 // H + yy * 255 // W) // 2 + rng.integers(0, 40, (H, W))).clip(0, 255).astype(np.uint8)
    got = host(lz.autocorrelation_2d(ctx, to_dev(img.ravel()).view(H, W)))
    tol = _acf2_tol(img)
    lags = [(0, 0), (1, 0), (0, 1), (1, 1), (7, 300), (H - 1, W - 1), (256, 384), (100, 5)]
    lags += [tuple(v) for v in rng.integers(0, [H, W], (8, 2))]
    for dx, dy in lags:
        want = dg.autocorrelation_2d_at(img, int(dx), int(dy))
        assert abs(got[dx, dy] - want) <= tol, (dx, dy, got[dx, dy], want, tol)
    assert abs(got[0, 0] - 1.0) <= tol


def test_autocorrelation_2d_sampled_direct(lz, ctx):
    """1009 x 1013 (both prime: all four passes are direct DFTs on the matrix cores), at sampled lags,
    the mirror rows included (dx above h/2)."""
    rng = np.random.default_rng(122)
    H, W = 1009, 1013
    img = rng.integers(0, 256, (H, W), dtype=np.uint8)
    img[::4, ::7] = 255
    got = host(lz.autocorrelation_2d(ctx, to_dev(img.ravel()).view(H, W)))
    tol = _acf2_tol(img)
    lags = [(0, 0), (1, 0), (0, 1), (4, 7), (504, 506), (505, 3), (H - 1, W - 1), (H - 4, 7)]
    lags += [tuple(v) for v in rng.integers(0, [H, W], (6, 2))]
    for dx, dy in lags:
        want = dg.autocorrelation_2d_at(img, int(dx), int(dy))
        assert abs(got[dx, dy] - want) <= tol, (dx, dy, got[dx, dy], want, tol)
    # an even matrix: A[-dx][-dy] = A[dx][dy], bit for bit for the mirrored rows
    assert np.array_equal(got[1:], got[:0:-1, np.r_[0, W - 1:0:-1]])


def test_autocorrelation_2d_sampled_fft_sizes(lz, ctx):
    """1024 x 1024 (all four passes by FFT), checked at sampled lags against exact ratios."""
    rng = np.random.default_rng(121)
    H = W = 1024
    img = rng.integers(0, 256, (H, W), dtype=np.uint8)
    img[::3, ::5] = 0  # some structure, so the coefficients are not all near zero
    got = host(lz.autocorrelation_2d(ctx, to_dev(img.ravel()).view(H, W)))
    tol = _acf2_tol(img)
    lags = [(0, 0), (1, 0), (0, 1), (3, 5), (6, 10), (512, 512), (H - 1, W - 1)]
    lags += [tuple(v) for v in rng.integers(0, [H, W], (6, 2))]
    for dx, dy in lags:
        want = dg.autocorrelation_2d_at(img, int(dx), int(dy))
        assert abs(got[dx, dy] - want) <= tol, (dx, dy, got[dx, dy], want, tol)


def test_diagnostics_of_a_ciphertext(lz, ctx):
    """Sanity (Section 4): a structured plaintext's ciphertext has a flat histogram, near-zero
    autocorrelation and a spectrum with no dominant frequency.  Not a security claim."""
    H, W = 128, 128
    xx, yy = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    img = ((xx + yy) % 64 + 96).astype(np.uint8)
    C = ctx.encrypt(to_dev(img.ravel()), b"123456")[:-24].contiguous()
    assert np.array_equal(host(C), oracle.encrypt(b"123456", img.ravel(), nthreads=8)[:-24])
    S = lz.entropy(ctx, lz.histogram(ctx, C))
    assert S > 7.98
    r = host(lz.autocorrelation(ctx, C, 64))
    assert abs(r[0] - 1.0) < 1e-12 and np.max(np.abs(r[1:])) < 0.05
    A = host(lz.autocorrelation_2d(ctx, C.view(H, W)))
    assert np.max(np.abs(A.ravel()[1:])) < 0.05
    P = host(lz.power_spectrum_2d(ctx, C.view(H, W)))
    Pp = host(lz.power_spectrum_2d(ctx, to_dev(img.ravel()).view(H, W)))
    ac_c = P.ravel()[1:]
    ac_p = Pp.ravel()[1:]
    assert ac_c.max() / ac_c.mean() < 30 < ac_p.max() / ac_p.mean()


def test_invalid_arguments(lz, ctx):
    import torch

    x = torch.zeros((4, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(lz.LorenzError):
        lz.power_spectrum_2d(ctx, torch.zeros((0, 4), dtype=torch.uint8, device="cuda"))
    with pytest.raises(lz.LorenzError):
        lz.autocorrelation_2d(ctx, torch.zeros((1, 1 << 17), dtype=torch.uint8, device="cuda"))
    with pytest.raises(lz.LorenzError):
        lz.autocorrelation(ctx, x.view(-1), 16385)
    with pytest.raises(lz.LorenzError):
        lz.power_spectrum_2d(ctx, x.view(-1))
