"""Pins of Step 3 of Section 3.2 (the update between bytes) in the CPU oracle, no GPU.

Step 3 moves the selectors mu, the coordinates alpha and the byte indices Omega
between two bytes and adds a' to the trajectory.  Its effect first shows in the
second byte of a block and in the tag of a message of two or more bytes.  The
derivation below builds those values from primitives that are pinned elsewhere,
and only from them:

* the key setup (hand values, exact fractions, hashlib);
* R (Python integer floor and shift);
* Theta (exact rationals, all 1,024 inputs);
* the Euler map F (fixed points, first-order convergence to the ODE).

It takes the sub-steps in the order the text of Steps 1-3 gives them:

1. R3 from the old alpha_3 and Omega_3;
2. mu_i' = (mu_i + R_i) mod 3, with R1 and R2 of Step 1 (old alpha, old Omega);
3. alpha_i = r[mu_i'], r being the trajectory after Step 2 (before a' is added);
4. Omega_i' = (Omega_i + R(alpha_[(i+2) mod 3]+1, Omega_i)) mod k_i, with the new
   alpha and the old Omega.  The index read 1-based is i itself;
5. r = r + a'.

Each of five plausible slips in that order, planted in a copy of the block
routine, changes the derived bytes or tags.  So every slip fails this pin
whatever the Python reference says.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import pyref

N_IT = 30
DT = 0.01
BLOCK = 4  # short blocks: a 12-byte message has three blocks of four bytes


def _digest(v: float) -> int:
    """N(v) = floor(v 10^13) as an unsigned 64-bit pattern (the integrity reading)."""
    return math.floor(v * 1e13) % 2 ** 64


def _derive_block(key: dict, b: int, P: bytes):
    """Ciphertext bytes and final state of block b for the plaintext P (1 to 3 bytes),
    from the key setup, R, Theta and F only, sub-step by sub-step."""
    r = [key["r0"][j] + b * 2.0 ** -24 for j in range(3)]       # block start (Section 5)
    mu = list(key["mu"])
    om = list(key["omega"])
    alpha = [r[mu[0]], r[mu[1]], r[mu[2]]]                        # Eq. alpha with n = 0
    C = []
    for p in P:
        # Step 1: encode with R(alpha_1, Omega_1) + R(alpha_2, Omega_2)
        R1 = oracle.R(alpha[0], om[0])
        R2 = oracle.R(alpha[1], om[1])
        C.append((p + R1 + R2) % 256)
        # Step 2: Theta into coordinate mu_3, then n_it steps of F
        r[mu[2]] = r[mu[2]] + oracle.theta(p, om[2])
        r = oracle.lorenz(r, DT, N_IT)
        # Step 3, sub-step 1: R3 from the old alpha_3 and Omega_3
        R3 = oracle.R(alpha[2], om[2])
        # sub-step 2: new selectors from the old ones and R1, R2, R3
        mu_new = [(mu[0] + R1) % 3, (mu[1] + R2) % 3, (mu[2] + R3) % 3]
        # sub-step 3: new alpha from the trajectory after Step 2 and the new selectors
        alpha_new = [r[mu_new[0]], r[mu_new[1]], r[mu_new[2]]]
        # sub-step 4: new Omega from the new alpha (index [(i+2) mod 3]+1 = i) and the old Omega
        om_new = [(om[i] + oracle.R(alpha_new[i], om[i])) % key["k"][i] for i in range(3)]
        # sub-step 5: r = r + a'
        r = [r[j] + key["a_prime"][j] for j in range(3)]
        mu, alpha, om = mu_new, alpha_new, om_new
    return C, r


def _cases():
    """Passwords covering every n_pi mod 3 class (the paper's example passwords among them), with
    plaintexts whose bytes are nonzero, so Theta moves the trajectory at every byte."""
    rng = np.random.default_rng(31)
    pws = [b"123456", b"123457", b"a", b"ab", b"abcd"]
    pws += [bytes(rng.integers(32, 127, n, dtype=np.uint8)) for n in (5, 8, 16, 33, 64)]
    return [(pw, bytes(rng.integers(1, 256, 3 * BLOCK, dtype=np.uint8))) for pw in pws]


def _step3_mismatches(encrypt) -> list:
    """Cases where encrypt(pw, P, n_it, block_len) differs from the derivation: bytes 2 and 3 of
    each of three blocks, and the tags of 2- and 3-byte messages.  Empty when it agrees."""
    bad = []
    for pw, P in _cases():
        key = oracle.key_setup(pw)
        C = encrypt(pw, P, N_IT, BLOCK)
        for b in range(3):
            want, _ = _derive_block(key, b, P[BLOCK * b:BLOCK * b + 3])
            got = [int(v) for v in C[BLOCK * b:BLOCK * b + 3]]
            if got[1:] != want[1:]:
                bad.append((pw, "bytes 2-3 of block", b))
        for n in (2, 3):
            want_c, r = _derive_block(key, 0, P[:n])
            tag = b"".join(_digest(v).to_bytes(8, "little") for v in r)
            Cn = bytes(encrypt(pw, P[:n], N_IT, 1 << 20))
            if list(Cn[:n]) != want_c or Cn[n:] != tag:
                bad.append((pw, "tag of an n-byte message", n))
    return bad


def _oracle_encrypt(pw, P, n_it, B):
    return oracle.encrypt(pw, np.frombuffer(P, np.uint8), n_it=n_it, block_len=B)


def _pyref_encrypt(pw, P, n_it, B):
    return pyref.encrypt(pw, P, n_it=n_it, B=B)


def test_step3_closed_form_c_oracle():
    """Bytes 2 and 3 of a block and the tags of 2- and 3-byte messages follow Step 3 (C oracle)."""
    assert _step3_mismatches(_oracle_encrypt) == []


def test_step3_closed_form_python_reference():
    assert _step3_mismatches(_pyref_encrypt) == []


def test_step3_decrypt_recovers_bytes_two_and_three():
    """Decryption runs the same Step 3 on the decoded bytes: the derived ciphertext decrypts back."""
    for pw, P in _cases()[:4]:
        key = oracle.key_setup(pw)
        C, r = _derive_block(key, 0, P[:3])
        tag = b"".join(_digest(v).to_bytes(8, "little") for v in r)
        Q, ok = oracle.decrypt(pw, bytes(C) + tag, n_it=N_IT)
        assert ok and bytes(Q) == P[:3]


# ---- planted slips: each must fail the pin above ----------------------------------------------

SLIPS = {
    "R3_from_new_alpha3": "R3 taken from the new alpha_3 instead of the old one",
    "mu_from_new_alpha": "mu updated with R of the new alpha",
    "a_prime_before_alpha": "a' added to r before alpha is re-read",
    "cyclic_alpha_index": "the alpha index of the Omega update read cyclically (alpha_3, alpha_1, alpha_2)",
    "omega_from_old_alpha": "Omega moved by R of the old alpha",
}


def _slipped_block(key, b, data, slip, n_it):
    """A copy of the block routine with one slip planted (slip None: no slip)."""
    r = [key["r0"][j] + b * 2.0 ** -24 for j in range(3)]
    mu, om = list(key["mu"]), list(key["omega"])
    alpha = [r[m] for m in mu]
    out = []
    for p in data:
        R1, R2 = oracle.R(alpha[0], om[0]), oracle.R(alpha[1], om[1])
        out.append((p + R1 + R2) % 256)
        r[mu[2]] = r[mu[2]] + oracle.theta(p, om[2])
        r = oracle.lorenz(r, DT, n_it)
        old_alpha = list(alpha)
        if slip == "a_prime_before_alpha":
            r = [r[j] + key["a_prime"][j] for j in range(3)]
        if slip == "R3_from_new_alpha3":
            R3 = oracle.R(r[mu[2]], om[2])
        else:
            R3 = oracle.R(alpha[2], om[2])
        Rs = [R1, R2, R3]
        if slip == "mu_from_new_alpha":
            Rs = [oracle.R(r[mu[i]], om[i]) for i in range(3)]
        mu = [(mu[i] + Rs[i]) % 3 for i in range(3)]
        alpha = [r[m] for m in mu]
        if slip == "cyclic_alpha_index":
            src = [alpha[(i + 2) % 3] for i in range(3)]
        elif slip == "omega_from_old_alpha":
            src = old_alpha
        else:
            src = alpha
        om = [(om[i] + oracle.R(src[i], om[i])) % key["k"][i] for i in range(3)]
        if slip != "a_prime_before_alpha":
            r = [r[j] + key["a_prime"][j] for j in range(3)]
    return out, r


def _slipped_encrypt(slip):
    def enc(pw, P, n_it, B):
        key = oracle.key_setup(pw)
        body, T = [], [0, 0, 0]
        nb = max(1, (len(P) + B - 1) // B)
        for b in range(nb):
            c, r = _slipped_block(key, b, P[B * b:B * (b + 1)], slip, n_it)
            body += c
            T = [T[j] ^ _digest(r[j]) for j in range(3)]
        return bytes(body) + b"".join(t.to_bytes(8, "little") for t in T)
    return enc


def test_slip_harness_without_slip_equals_oracle():
    """The copy used for planting slips equals the oracle when no slip is planted, so a failure
    below comes from the slip alone."""
    enc = _slipped_encrypt(None)
    for pw, P in _cases()[:5]:
        assert enc(pw, P, N_IT, BLOCK) == bytes(_oracle_encrypt(pw, P, N_IT, BLOCK))
    assert _step3_mismatches(enc) == []


@pytest.mark.parametrize("slip", sorted(SLIPS))
def test_planted_step3_slip_fails_the_pin(slip):
    """Each plausible misreading of Step 3's order is caught by the derivation."""
    assert _step3_mismatches(_slipped_encrypt(slip)), SLIPS[slip]
