"""Pure-Python mini-reference of the Lorenz chaotic cipher (arXiv:1201.3114).

TEST INFRASTRUCTURE ONLY: a second, independent implementation of the same
reading as ``lz_oracle.c``, written with Python integers (exact), fractions
(exact rational rounding of a'), ``hashlib`` and Python floats (IEEE binary64,
round to nearest even, never contracted).  It is slow (about 10^6 Euler steps
per second), so it is meant for tiny messages and small ``n_it``.

Every function names the passage of the paper it follows.
"""
from __future__ import annotations

import hashlib
import math
from fractions import Fraction

SIGMA = 10.0
RHO = 28.0
BETA = 8.0 / 3.0          # Python evaluates the correctly rounded quotient
NU = 13                   # floor(log10 2^(xi - 6)) with xi = 52 (Eq. R_nu)
SCALE = 10.0 ** NU        # 1e13, exact in binary64


def pack(pw: bytes) -> tuple[int, int, int]:
    """Section 3.1, equations for a1, a2, a3 (pi is 1-based in the paper)."""
    n = len(pw)
    L = n // 3
    pi = lambda i: pw[i - 1]
    if n % 3 == 0:
        a1 = sum(pi(i) * 2 ** (8 * (i - 1)) for i in range(1, L + 1))
    else:
        a1 = sum(pi(i) * 2 ** (8 * i) for i in range(1, L + 1)) + pi(3 * L + 1)
    if n % 3 != 2:
        a2 = sum(pi(i) * 2 ** (8 * (-L + (i - 1))) for i in range(L + 1, 2 * L + 1))
    else:
        a2 = sum(pi(i) * 2 ** (8 * (-L + i)) for i in range(L + 1, 2 * L + 1)) + pi(3 * L + 2)
    a3 = sum(pi(i) * 2 ** (8 * (-2 * L + (i - 1))) for i in range(2 * L + 1, 3 * L + 1))
    return a1, a2, a3


def digits_D(L: int) -> int:
    """Section 3.1, g(x): exponent ceil(log10 2^(8(L+1))), as an exact digit count."""
    return len(str(2 ** (8 * (L + 1))))


def key_setup(pw: bytes, lam=(1.0, 1.0, 1.0), k=(4, 4, 4)) -> dict:
    """Section 3.1: a, a', r0 = a' + lambda, mu, Omega = hash(i a) mod k_i."""
    a = pack(pw)
    L = len(pw) // 3
    D = digits_D(L)
    a_prime = [float(Fraction(aj, 10 ** D)) for aj in a]      # correctly rounded
    r0 = [a_prime[j] + lam[j] for j in range(3)]
    a1, a2, a3 = a
    mu = [(a1 + a2 + a3) % 3, (a1 * a2 + a3) % 3, (a1 + a2 * a3) % 3]
    omega = []
    for i in (1, 2, 3):
        msg = b"".join((i * aj).to_bytes(32, "little") for aj in a)
        h = int.from_bytes(hashlib.sha256(msg).digest(), "big")
        omega.append(h % k[i - 1])
    return dict(a=a, L=L, D=D, a_prime=a_prime, r0=r0, mu=mu, omega=omega, k=list(k))


def euler(r, dt, steps):
    """Section 3.1, F: forward Euler of the Lorenz system, fixed evaluation order."""
    x, y, z = r
    for _ in range(steps):
        dx = SIGMA * (y - x)
        dy = (x * (RHO - z)) - y
        dz = (x * y) - (BETA * z)
        x, y, z = x + dt * dx, y + dt * dy, z + dt * dz
    return [x, y, z]


def fma(a: float, b: float, c: float) -> float:
    """a*b + c with one rounding (exact rational arithmetic, then nearest-even)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def euler_fma(r, dt, steps):
    """Euler with each update fused into one rounding (variant format of Section 3.1's F)."""
    x, y, z = r
    for _ in range(steps):
        dx = SIGMA * (y - x)
        dy = fma(x, RHO - z, -y)
        dz = fma(x, y, -(BETA * z))
        x, y, z = fma(dt, dx, x), fma(dt, dy, y), fma(dt, dz, z)
    return [x, y, z]


def _field(x, y, z):
    return SIGMA * (y - x), (x * (RHO - z)) - y, (x * y) - (BETA * z)


def rk4(r, dt, steps):
    """Classical Runge-Kutta 4 of the Lorenz system (a format variant; Section 3.1 leaves the integrator open)."""
    x, y, z = r
    h2, h6 = dt * 0.5, dt / 6.0
    for _ in range(steps):
        k1 = _field(x, y, z)
        k2 = _field(x + h2 * k1[0], y + h2 * k1[1], z + h2 * k1[2])
        k3 = _field(x + h2 * k2[0], y + h2 * k2[1], z + h2 * k2[2])
        k4 = _field(x + dt * k3[0], y + dt * k3[1], z + dt * k3[2])
        x = x + h6 * ((k1[0] + k4[0]) + 2.0 * (k2[0] + k3[0]))
        y = y + h6 * ((k1[1] + k4[1]) + 2.0 * (k2[1] + k3[1]))
        z = z + h6 * ((k1[2] + k4[2]) + 2.0 * (k2[2] + k3[2]))
    return [x, y, z]


INTEGRATORS = {"euler": euler, "euler_fma": euler_fma, "rk4": rk4}


def R(alpha: float, omega: int) -> int:
    """Eq. R_nu: byte Omega of floor(alpha 10^nu), two's complement."""
    return (math.floor(alpha * SCALE) >> (8 * omega)) & 255


def digest(v: float) -> int:
    """Integrity word N(v) = floor(v 10^nu) as an unsigned 64-bit pattern."""
    return math.floor(v * SCALE) & (2 ** 64 - 1)


def crypt_block(key, b, data: bytes, decrypt: bool, dt=0.01, n_it=3000, integrator="euler"):
    """Steps 1-3 of Section 3.2 over block b of the parallel version (Section 5)."""
    r = [key["r0"][j] + b * 2.0 ** -24 for j in range(3)]
    mu = list(key["mu"])
    om = list(key["omega"])
    k = key["k"]
    alpha = [r[mu[i]] for i in range(3)]
    out = bytearray()
    for byte in data:
        R1, R2 = R(alpha[0], om[0]), R(alpha[1], om[1])
        if decrypt:
            p = (byte - R1 - R2) % 256
            out.append(p)
        else:
            p = byte
            out.append((p + R1 + R2) % 256)
        theta = p / 10.0 ** (3 + om[2])
        r[mu[2]] = r[mu[2]] + theta
        r = INTEGRATORS[integrator](r, dt, n_it)
        R3 = R(alpha[2], om[2])
        mu = [(mu[i] + (R1, R2, R3)[i]) % 3 for i in range(3)]
        alpha = [r[mu[i]] for i in range(3)]
        om = [(om[i] + R(alpha[((i + 1 + 2) % 3)], om[i])) % k[i] for i in range(3)]
        r = [r[j] + key["a_prime"][j] for j in range(3)]
    return bytes(out), tuple(digest(v) for v in r)


def _blocks(n, B):
    if n == 0:
        return [(0, 0, 0)]
    return [(b, b * B, min(n, (b + 1) * B)) for b in range((n + B - 1) // B)]


def encrypt(pw: bytes, P: bytes, dt=0.01, n_it=3000, B=256, lam=(1.0, 1.0, 1.0), k=(4, 4, 4), integrator="euler"):
    key = key_setup(pw, lam, k)
    body = bytearray()
    T = [0, 0, 0]
    for b, s, e in _blocks(len(P), B):
        c, d = crypt_block(key, b, P[s:e], False, dt, n_it, integrator)
        body += c
        T = [T[j] ^ d[j] for j in range(3)]
    return bytes(body) + b"".join(t.to_bytes(8, "little") for t in T)


def decrypt(pw: bytes, C: bytes, dt=0.01, n_it=3000, B=256, lam=(1.0, 1.0, 1.0), k=(4, 4, 4), integrator="euler"):
    """Returns (plaintext, ok); on a tag mismatch the plaintext is all zeros."""
    key = key_setup(pw, lam, k)
    n = len(C) - 24
    body = bytearray()
    T = [0, 0, 0]
    for b, s, e in _blocks(n, B):
        p, d = crypt_block(key, b, C[s:e], True, dt, n_it, integrator)
        body += p
        T = [T[j] ^ d[j] for j in range(3)]
    stored = [int.from_bytes(C[n + 8 * j:n + 8 * j + 8], "little") for j in range(3)]
    if stored != T:
        return bytes(n), False
    return bytes(body), True
