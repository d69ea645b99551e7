"""Pins of the CPU oracle against what the paper and mathematics fix (no GPU).

Each test names the passage it checks.  None of the expected values below
comes from the GPU library: they are hand-derived (tests/golden), closed forms,
library routines (hashlib, fractions, scipy) or properties of the method.
"""
import hashlib
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import pyref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pw(rng, n):
    return bytes(rng.integers(32, 127, n, dtype=np.uint8))


# ---- Section 3.1: password -> a, a', r0, mu ---------------------------------

def test_keysetup_hand_values():
    """Hand-derived a, D, a', mu for the paper's example passwords (Section 3.1, Section 4)."""
    cases = json.load(open(os.path.join(GOLDEN, "keysetup_hand.json")))["cases"]
    for c in cases:
        k = oracle.key_setup(c["pw"].encode())
        assert k["a"] == c["a"], c["pw"]
        assert k["D"] == c["D"], c["pw"]
        assert k["mu"] == c["mu"], c["pw"]
        # a' = a / 10^D: D <= 15 here so the quotient of two exact doubles is correctly rounded
        assert k["a_prime"] == [a / 10.0 ** c["D"] for a in c["a"]]
        assert k["r0"] == [ap + 1.0 for ap in k["a_prime"]]


def test_keysetup_a_prime_correctly_rounded_all_lengths():
    """a' = g(a) is the correctly rounded rational a / 10^D, 0 <= a' <= 1 (Section 3.1)."""
    rng = np.random.default_rng(1)
    for n in range(1, 65):
        for _ in range(3):
            pw = _pw(rng, n)
            k = oracle.key_setup(pw)
            a = pyref.pack(pw)
            assert k["a"] == list(a)
            assert k["D"] == len(str(2 ** (8 * (n // 3 + 1))))
            for j in range(3):
                assert k["a_prime"][j] == float(Fraction(a[j], 10 ** k["D"]))
                assert 0.0 <= k["a_prime"][j] < 1.0
                assert a[j] < 2 ** (8 * (n // 3 + 1))


def test_keysetup_mu_omega_independent():
    """mu by exact big-integer arithmetic and Omega = SHA-256(i a) mod k_i via hashlib (Section 3.1)."""
    rng = np.random.default_rng(2)
    for n in list(range(1, 65)) * 2:
        pw = _pw(rng, n)
        k = oracle.key_setup(pw)
        a1, a2, a3 = pyref.pack(pw)
        assert k["mu"] == [(a1 + a2 + a3) % 3, (a1 * a2 + a3) % 3, (a1 + a2 * a3) % 3]
        for i in (1, 2, 3):
            msg = b"".join((i * a).to_bytes(32, "little") for a in (a1, a2, a3))
            h = int.from_bytes(hashlib.sha256(msg).digest(), "big")
            assert k["omega"][i - 1] == h % 4
    # modulus 3 (k_i = 3 is the other value allowed by 2 < k_i <= 4)
    pw = b"modulus three"
    k3 = oracle.key_setup(pw, k=(3, 3, 3))
    a = pyref.pack(pw)
    for i in (1, 2, 3):
        msg = b"".join((i * x).to_bytes(32, "little") for x in a)
        assert k3["omega"][i - 1] == int.from_bytes(hashlib.sha256(msg).digest(), "big") % 3


def test_keysetup_matches_pyref():
    """C oracle (strtod, OpenSSL, byte bignums) equals the Python reference (Fraction, hashlib, int)."""
    rng = np.random.default_rng(3)
    for n in range(1, 65):
        pw = _pw(rng, n)
        k1, k2 = oracle.key_setup(pw), pyref.key_setup(pw)
        for f in ("D", "a_prime", "r0", "mu", "omega"):
            assert k1[f] == (list(k2[f]) if isinstance(k2[f], (list, tuple)) else k2[f]), (n, f)


# ---- Eq. R_nu -----------------------------------------------------------------

def test_R_byte_extraction():
    """R_nu(alpha, Omega) = byte Omega of floor(alpha 10^13), two's complement (Eq. R_nu)."""
    rng = np.random.default_rng(4)
    alphas = list(rng.uniform(-60, 60, 4000))
    # adversarial: products that land on or next to integers, negatives, zero
    for m in rng.integers(-5 * 10 ** 14, 5 * 10 ** 14, 500):
        v = float(m) / 1e13
        alphas += [v, math.nextafter(v, -math.inf), math.nextafter(v, math.inf)]
    alphas += [0.0, -0.0, 1e-14, -1e-14, 53.6, -53.6]
    for a in alphas:
        N = math.floor(a * 1e13)
        for om in range(4):
            want = (N % 2 ** 64 >> (8 * om)) & 255
            assert oracle.R(a, om) == want, (a, om)
            assert pyref.R(a, om) == want


# ---- Step 2: Theta --------------------------------------------------------------

def test_theta_exhaustive():
    """Theta = P_i / 10^(3+Omega_3) correctly rounded; bound 0 <= m_i <= 0.255 (Section 2, Step 2)."""
    mx = 0.0
    for p in range(256):
        for om in range(4):
            t = oracle.theta(p, om)
            assert t == float(Fraction(p, 10 ** (3 + om)))
            assert 0.0 <= t <= 0.255
            mx = max(mx, t)
    assert mx == 0.255


# ---- Section 3.1: the Euler-discretised Lorenz system F --------------------------

def test_euler_fixed_points():
    """The origin and C+- = (+-sqrt(beta(rho-1)), +-sqrt(beta(rho-1)), rho-1) are fixed points of F."""
    c = math.sqrt(72.0)  # beta (rho - 1) = (8/3) 27 = 72
    for r in ([0.0, 0.0, 0.0], [c, c, 27.0], [-c, -c, 27.0]):
        assert oracle.lorenz(r, 0.01, 3000) == r
        assert pyref.euler(r, 0.01, 3000) == r


def test_euler_converges_to_lorenz_ode():
    """F is forward Euler of the Lorenz equations: first-order convergence to the ODE solution."""
    from scipy.integrate import solve_ivp

    def f(t, r):
        x, y, z = r
        return [10.0 * (y - x), x * (28.0 - z) - y, x * y - 8.0 / 3.0 * z]

    r0, T = [1.0, 1.0, 1.0], 1.0
    ref = solve_ivp(f, (0, T), r0, rtol=1e-12, atol=1e-12, method="DOP853").y[:, -1]
    errs = []
    for dt in (1e-3, 5e-4, 2.5e-4):
        r = oracle.lorenz(r0, dt, int(round(T / dt)))
        errs.append(float(np.max(np.abs(np.array(r) - ref))))
    assert errs[-1] < 0.2
    for e1, e2 in zip(errs, errs[1:]):
        assert 1.8 < e1 / e2 < 2.2, errs


def test_euler_matches_pyref_bitwise():
    rng = np.random.default_rng(5)
    for _ in range(20):
        r = list(rng.uniform(-20, 20, 3))
        r[2] = abs(r[2]) + 5
        assert oracle.lorenz(r, 0.01, 500) == pyref.euler(r, 0.01, 500)


def test_dt_bound_reading():
    """Reading of 0 < dt <= 0.027: forward Euler from (1,1,1) overflows for dt >= 0.025, stays bounded at 0.024."""
    r = oracle.lorenz([1.0, 1.0, 1.0], 0.025, 200)
    assert not all(math.isfinite(v) for v in r)
    r = oracle.lorenz([1.0, 1.0, 1.0], 0.024, 200000)
    assert all(abs(v) < 100 for v in r)


def test_escape_inside_the_paper_ranges_is_reported():
    """At dt = 0.024 a start inside the lambda ranges of Section 3.1 leaves the attractor and overflows; the
    oracle reports it (floor(v 10^13) is then no 64-bit integer) instead of producing bytes.  The same holds
    for a block index whose start r0 + b 2^-24 lies 64 away from r0."""
    r = oracle.lorenz([0.0, 16.0, 0.091], 0.024, 3000)
    assert not all(math.isfinite(v) for v in r)
    P = np.zeros(64, np.uint8)
    with pytest.raises(oracle.TrajectoryEscaped):
        oracle.encrypt(b"123456", P, dt=0.024, lam=(0.0, 16.0, 0.091), n_it=3000)
    with pytest.raises(oracle.TrajectoryEscaped):
        oracle.crypt_block(b"123456", 64 << 24, P, n_it=3000)
    C = oracle.encrypt(b"123456", P, n_it=3000)
    Q, ok = oracle.decrypt(b"123456", C, n_it=3000)
    assert ok and not Q.any()
    with pytest.raises(oracle.TrajectoryEscaped):
        oracle.decrypt(b"123456", C, dt=0.024, lam=(0.0, 16.0, 0.091), n_it=3000)


@pytest.mark.parametrize("integrator", ["euler", "euler_fma", "rk4"])
def test_largest_accepted_dt_stays_on_the_attractor(integrator):
    """dt = 0.015 (the largest the library accepts): starts on a 5 x 5 x 5 grid over the closure of the lambda
    ranges shifted by a' and the block offset (each in [0, 1]) stay bounded for 2 x 10^5 steps, and so do
    points of the attractor moved by up to 1.5 in every coordinate (Theta <= 0.255 plus a' < 1 per byte)."""
    lo = np.array([-15.67, -11.28, 0.090])
    hi = np.array([16.01, 16.01, 62.0]) + 2.0
    g = [np.linspace(lo[j], hi[j], 5) for j in range(3)]
    starts = np.array(np.meshgrid(*g, indexing="ij")).reshape(3, -1).T
    end = oracle.lorenz_many(starts, 0.015, 200_000, integrator, nthreads=8)
    assert np.all(np.abs(end) < 100), starts[np.any(~(np.abs(end) < 100), axis=1)][:3]
    path = [oracle.lorenz([1.0, 1.0, 1.0], 0.015, 5000, integrator)]
    for _ in range(63):
        path.append(oracle.lorenz(path[-1], 0.015, 97, integrator))
    corners = np.array([[sx, sy, sz] for sx in (-1.5, 1.5) for sy in (-1.5, 1.5) for sz in (-1.5, 1.5)])
    moved = (np.array(path)[:, None, :] + corners[None, :, :]).reshape(-1, 3)
    end = oracle.lorenz_many(moved, 0.015, 20_000, integrator, nthreads=8)
    assert np.all(np.abs(end) < 100)


def test_cipher_at_the_corners_of_the_parameter_domain():
    """The whole cipher at dt = 0.015 with lambda near each corner of its ranges, on the first block and on the
    last block a message may have (2^24 - 1), runs without leaving the attractor and round-trips."""
    rng = np.random.default_rng(40)
    P = rng.integers(0, 256, 600, dtype=np.uint8)
    for lam in [(-15.66, -11.27, 0.0901), (16.0, 16.0, 61.99), (-15.66, 16.0, 0.0901), (16.0, -11.27, 61.99)]:
        kw = dict(dt=0.015, lam=lam, n_it=3000)
        C = oracle.encrypt(b"corner", P, nthreads=4, block_len=600, **kw)
        Q, ok = oracle.decrypt(b"corner", C, nthreads=4, block_len=600, **kw)
        assert ok and np.array_equal(Q, P)
        out, _ = oracle.crypt_block(b"corner", (1 << 24) - 1, P[:256], **kw)
        assert len(out) == 256


def test_literal_printed_map_is_degenerate():
    """Reading of the garbled Euler equations: taken literally they contract to the origin."""
    x, y, z, s, rho, b, dt = 1.5, 1.2, 1.3, 10.0, 28.0, 8.0 / 3.0, 0.01
    for _ in range(3000):
        x, y, z = ((1 - s) * x + s * y) * dt, (rho * x - 2 * y - x * z) * dt, (x * y + (1 - b) * z) * dt
    assert (x, y, z) == (0.0, 0.0, 0.0)


# ---- Steps 1-3 (Section 3.2) and the parallel version (Section 5) ---------------

def test_first_byte_closed_form():
    """Step 1 at i = 1: C_1 = (P_1 + R(alpha_1, Omega_1) + R(alpha_2, Omega_2)) mod 256, alpha_i = r^(b)[mu_i]."""
    rng = np.random.default_rng(6)
    for n in (1, 2, 3, 7, 16, 33, 64):
        pw = _pw(rng, n)
        k = oracle.key_setup(pw)
        P = rng.integers(0, 256, 5 * 256, dtype=np.uint8)
        C = oracle.encrypt(pw, P, n_it=5)
        for b in range(5):
            r = [k["r0"][j] + b * 2.0 ** -24 for j in range(3)]
            al = [r[k["mu"][i]] for i in range(3)]
            want = (int(P[256 * b]) + pyref.R(al[0], k["omega"][0]) + pyref.R(al[1], k["omega"][1])) % 256
            assert C[256 * b] == want


def test_one_byte_message_tag_closed_form():
    """One-byte message: final state = F^(n_it)(r0 + Theta e_(mu_3)) + a', tag = N of it (Steps 2-3)."""
    rng = np.random.default_rng(7)
    for n in (3, 5, 16):
        pw = _pw(rng, n)
        k = oracle.key_setup(pw)
        for p in (0, 1, 200, 255):
            C = oracle.encrypt(pw, bytes([p]), n_it=40)
            r = list(k["r0"])
            r[k["mu"][2]] = r[k["mu"][2]] + p / 10.0 ** (3 + k["omega"][2])
            r = oracle.lorenz(r, 0.01, 40)
            r = [r[j] + k["a_prime"][j] for j in range(3)]
            want = b"".join((math.floor(v * 1e13) % 2 ** 64).to_bytes(8, "little") for v in r)
            assert bytes(C[1:]) == want


def test_roundtrip_and_empty():
    rng = np.random.default_rng(8)
    for n in (0, 1, 255, 256, 257, 1000):
        P = rng.integers(0, 256, n, dtype=np.uint8)
        C = oracle.encrypt(b"roundtrip pw", P, n_it=20)
        assert len(C) == n + 24
        Q, ok = oracle.decrypt(b"roundtrip pw", C, n_it=20)
        assert ok and np.array_equal(Q, P)


def test_codec_exhaustive_inverse():
    """Eqs. encode/decode: D(E(x)) = x for every byte x and every keystream sum (mod 2^8)."""
    for s in range(511):
        for x in range(256):
            y = (x + s) % 256
            assert (y - s) % 256 == x
    # and through the oracle: every plaintext byte value, first byte of a block
    P = np.arange(256, dtype=np.uint8).repeat(1)
    C = oracle.encrypt(b"codec", P, n_it=3, block_len=1)
    Q, ok = oracle.decrypt(b"codec", C, n_it=3, block_len=1)
    assert ok and np.array_equal(Q, P)


def test_tamper_any_byte_detected():
    """Integrity (Abstract, end of Section 2): altering any ciphertext byte, tag included, is detected."""
    rng = np.random.default_rng(9)
    P = rng.integers(0, 256, 300, dtype=np.uint8)
    C = oracle.encrypt(b"tamper", P, n_it=30)
    for off in range(len(C)):
        D = C.copy()
        D[off] ^= int(rng.integers(1, 256))
        Q, ok = oracle.decrypt(b"tamper", D, n_it=30)
        assert not ok, off
        assert not Q.any()


def test_tamper_full_iterations_and_wrong_password():
    rng = np.random.default_rng(10)
    P = rng.integers(0, 256, 600, dtype=np.uint8)
    C = oracle.encrypt(b"pw-3000", P)
    for off in (0, 255, 256, 599, 600, 623):
        D = C.copy()
        D[off] ^= 0x01
        assert not oracle.decrypt(b"pw-3000", D)[1]
    assert not oracle.decrypt(b"pw-3001", C)[1]
    assert oracle.decrypt(b"pw-3000", C)[1]


def test_block_independence():
    """Parallel version (Section 5): blocks are independent chains; a change stays in its block."""
    rng = np.random.default_rng(11)
    P = rng.integers(0, 256, 1024, dtype=np.uint8)
    C = oracle.encrypt(b"indep", P, n_it=20)
    P2 = P.copy()
    P2[300] ^= 0x55
    C2 = oracle.encrypt(b"indep", P2, n_it=20)
    diff = np.nonzero(C[:1024] != C2[:1024])[0]
    assert diff.min() == 300 and diff.max() < 512
    assert (C[1024:] != C2[1024:]).any()


def test_sequential_version_is_block_zero():
    """Sequential strong version = one block: equals block mode whenever block_len >= n."""
    rng = np.random.default_rng(12)
    P = rng.integers(0, 256, 700, dtype=np.uint8)
    a = oracle.encrypt(b"seq", P, n_it=15, block_len=700)
    b = oracle.encrypt(b"seq", P, n_it=15, block_len=4096)
    c = oracle.encrypt(b"seq", P, n_it=15, block_len=256)
    assert np.array_equal(a, b)
    assert np.array_equal(a[:256], c[:256]) and not np.array_equal(a[256:700], c[256:700])


@pytest.mark.parametrize("n_it", [1, 7, 30])
@pytest.mark.parametrize("B", [1, 3, 64, 1 << 20])
def test_c_oracle_equals_python_reference(n_it, B):
    rng = np.random.default_rng(100 + n_it * 7 + B % 97)
    for n_pw in (1, 2, 3, 4, 5, 6, 17, 64):
        pw = _pw(rng, n_pw)
        P = rng.integers(0, 256, int(rng.integers(0, 90)), dtype=np.uint8)
        C = oracle.encrypt(pw, P, n_it=n_it, block_len=B)
        assert bytes(C) == pyref.encrypt(pw, bytes(P), n_it=n_it, B=B)
        Q, ok = pyref.decrypt(pw, bytes(C), n_it=n_it, B=B)
        assert ok and Q == bytes(P)


def test_c_oracle_equals_python_reference_full_iterations():
    P = bytes(range(40))
    C = oracle.encrypt(b"123456", P)
    assert bytes(C) == pyref.encrypt(b"123456", P)


# ---- sanity only (Section 4): a degenerate keystream would fail these -------------

def test_ciphertext_entropy_sanity():
    """Ciphertext byte entropy reaches S_max = 8 for a low-entropy plaintext (Section 4).

    Two properties of the method as read shape the keystream: the three (mu_i, Omega_i)
    channels share one update rule, so once they coincide they stay merged and the keystream
    byte is 2 R (even: the ciphertext keeps the plaintext's parity); and the next Step 1 reads
    the same alpha that just moved Omega, so R = 0 mod 4 occurs with probability 7/16.  The
    plaintext here is 5-bit (32 symbols, balanced parity).  A degenerate keystream (the literal
    printed map, a constant or short cycle) fails both checks.
    """
    rng = np.random.default_rng(15)
    P = rng.integers(64, 96, 1 << 16, dtype=np.uint8)
    C = oracle.encrypt(b"123456", P, nthreads=8)[:-24]
    p = np.bincount(C, minlength=256) / len(C)
    assert -np.sum(p[p > 0] * np.log2(p[p > 0])) > 7.99
    Z = oracle.encrypt(b"123456", np.zeros(1 << 16, dtype=np.uint8), nthreads=8)[:-24]
    q = np.bincount(Z >> 1, minlength=128) / len(Z)
    assert (q > 0).sum() == 128
    assert -np.sum(q[q > 0] * np.log2(q[q > 0])) > 6.8
    # 2R mod 256 = 0 mod 8 exactly when R = 0 mod 4: 7/16 of the keystream, vs 1/4 for uniform R
    assert abs(np.mean(Z % 8 == 0) - 7 / 16) < 0.03


def test_password_sensitivity_sanity():
    """Passwords 123456 and 123457 (Section 4, Fig. 2) give ciphertexts that differ almost everywhere.

    Both keystreams are mostly even (merged channels), so a byte differs when its upper seven
    bits do; with the R = 0 mod 4 excess the expected collision rate is about 1%.
    """
    P = np.random.default_rng(13).integers(0, 256, 8192, dtype=np.uint8)
    a = oracle.encrypt(b"123456", P, nthreads=8)
    b = oracle.encrypt(b"123457", P, nthreads=8)
    assert np.mean(a != b) > 0.98


def test_threads_do_not_change_output():
    P = np.random.default_rng(14).integers(0, 256, 5000, dtype=np.uint8)
    a = oracle.encrypt(b"threads", P, n_it=50, nthreads=1)
    b = oracle.encrypt(b"threads", P, n_it=50, nthreads=8)
    assert np.array_equal(a, b)


# ---- integrator variants (Section 3.1 leaves the integrator open to other schemes) --------

def test_variant_fixed_points():
    c = math.sqrt(72.0)
    for integ in ("euler_fma", "rk4"):
        for r in ([0.0, 0.0, 0.0], [c, c, 27.0], [-c, -c, 27.0]):
            assert oracle.lorenz(r, 0.01, 3000, integ) == r, integ
            assert pyref.INTEGRATORS[integ](r, 0.01, 300) == r, integ


def test_rk4_fourth_order_convergence():
    """RK4 reaches the DOP853 solution of the Lorenz ODE with error ratio ~16 per halving of dt."""
    from scipy.integrate import solve_ivp

    def f(t, r):
        x, y, z = r
        return [10.0 * (y - x), x * (28.0 - z) - y, x * y - 8.0 / 3.0 * z]

    r0, T = [1.0, 1.0, 1.0], 0.5
    ref = solve_ivp(f, (0, T), r0, rtol=1e-13, atol=1e-13, method="DOP853").y[:, -1]
    errs = [float(np.max(np.abs(np.array(oracle.lorenz(r0, dt, int(round(T / dt)), "rk4")) - ref)))
            for dt in (0.01, 0.005, 0.0025)]
    for e1, e2 in zip(errs, errs[1:]):
        assert 14.0 < e1 / e2 < 20.0, errs


def test_euler_fma_first_order_and_close_to_euler():
    """Fused Euler converges at first order and differs from the 14-rounding Euler only by rounding."""
    from scipy.integrate import solve_ivp

    def f(t, r):
        x, y, z = r
        return [10.0 * (y - x), x * (28.0 - z) - y, x * y - 8.0 / 3.0 * z]

    r0, T = [1.0, 1.0, 1.0], 1.0
    ref = solve_ivp(f, (0, T), r0, rtol=1e-12, atol=1e-12, method="DOP853").y[:, -1]
    errs = [float(np.max(np.abs(np.array(oracle.lorenz(r0, dt, int(round(T / dt)), "euler_fma")) - ref)))
            for dt in (1e-3, 5e-4, 2.5e-4)]
    for e1, e2 in zip(errs, errs[1:]):
        assert 1.8 < e1 / e2 < 2.2, errs
    rng = np.random.default_rng(16)
    for _ in range(200):
        r = [float(v) for v in rng.uniform(-20, 20, 3)]
        a = oracle.lorenz(r, 0.01, 1, "euler")
        b = oracle.lorenz(r, 0.01, 1, "euler_fma")
        for u, v in zip(a, b):
            assert abs(u - v) <= 8 * math.ulp(max(abs(u), 1.0))


def test_variants_match_python_reference_bitwise():
    rng = np.random.default_rng(17)
    for integ in ("euler_fma", "rk4"):
        for _ in range(10):
            r = [float(v) for v in rng.uniform(-15, 15, 3)]
            r[2] = abs(r[2]) + 5
            assert oracle.lorenz(r, 0.01, 200, integ) == pyref.INTEGRATORS[integ](r, 0.01, 200), integ
        P = bytes(rng.integers(0, 256, 50, dtype=np.uint8))
        for B in (7, 1 << 20):
            C = oracle.encrypt(b"variant", P, n_it=11, block_len=B, integrator=integ)
            assert bytes(C) == pyref.encrypt(b"variant", P, n_it=11, B=B, integrator=integ)
            Q, ok = oracle.decrypt(b"variant", C, n_it=11, block_len=B, integrator=integ)
            assert ok and bytes(Q) == P


def test_variants_are_distinct_formats():
    P = np.random.default_rng(18).integers(0, 256, 512, dtype=np.uint8)
    outs = {i: oracle.encrypt(b"formats", P, integrator=i, nthreads=2) for i in ("euler", "euler_fma", "rk4")}
    assert np.mean(outs["euler"] != outs["euler_fma"]) > 0.5
    assert np.mean(outs["euler"] != outs["rk4"]) > 0.9
    for i, C in outs.items():
        Q, ok = oracle.decrypt(b"formats", C, integrator=i, nthreads=2)
        assert ok and np.array_equal(Q, P)
