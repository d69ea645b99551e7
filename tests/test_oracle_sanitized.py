"""The oracle under host sanitizers: AddressSanitizer + UndefinedBehaviorSanitizer, and ThreadSanitizer (its
block and Lorenz-state threads).  tests/native/oracle_sanitize.c compiles the oracle's source into one program
with gcc; the test feeds it seeded cases (every password length 1..64, messages empty to several blocks, block
lengths 1 to sequential, all three integrators, k in {3, 4}, 1 or 4 threads), fails on any sanitizer report, and
requires every result to equal the oracle's ordinary build byte for byte."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "native", "oracle_sanitize.c")
SAN = {
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
    "tsan": ["-fsanitize=thread"],
}
ENV = {
    "asan_ubsan": {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:exitcode=66",
                   "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1:exitcode=67"},
    "tsan": {"TSAN_OPTIONS": "halt_on_error=1:exitcode=68"},
}
REPORTS = ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:", "WARNING: ThreadSanitizer")


def _hex(b) -> str:
    b = bytes(b)
    return b.hex() if b else "-"


def _cases(rng):
    """(line, expected output) pairs; expected values come from the oracle's ordinary build."""
    cases = []
    lengths = list(range(1, 65))
    rng.shuffle(lengths)
    sizes = [0, 1, 2, 23, 24, 25, 255, 256, 257, 700]
    for i, n_pw in enumerate(lengths):
        pw = bytes(rng.integers(0, 256, n_pw, dtype=np.uint8))
        n = sizes[i % len(sizes)]
        P = rng.integers(0, 256, n, dtype=np.uint8)
        n_it = int(rng.integers(3, 30))
        block_len = [1, 5, 64, 256, 100_000][i % 5]
        integrator = i % 3
        nthreads = 4 if i % 2 else 1
        k = tuple(int(v) for v in rng.integers(3, 5, 3))
        C = oracle.encrypt(pw, P, nthreads=1, n_it=n_it, block_len=block_len, integrator=integrator, k=k)
        line = f"E {_hex(pw)} {n_it} {block_len} {integrator} {nthreads} {k[0]} {k[1]} {k[2]} {_hex(P)}"
        cases.append((line, f"{_hex(C)} rt=1 tamper=-2"))
    for integrator in range(3):
        r = rng.uniform(-20, 20, (37, 3))
        r[:, 2] = rng.uniform(1, 45, 37)
        out = oracle.lorenz_many(r, 0.01, 250, integrator=integrator, nthreads=1)
        cases.append((f"L 37 250 {integrator} 4 {_hex(r.tobytes())}", _hex(out.tobytes())))
    alpha = rng.uniform(-60, 60, 500)
    omega = rng.integers(0, 4, 500, dtype=np.uint8)
    p = rng.integers(0, 256, 300, dtype=np.uint8)
    omega3 = rng.integers(0, 4, 300, dtype=np.uint8)
    expect = f"{_hex(oracle.R_many(alpha, omega))} {_hex(oracle.theta_many(p, omega3).tobytes())}"
    cases.append((f"U 500 300 {_hex(alpha.tobytes())} {_hex(omega)} {_hex(p)} {_hex(omega3)}", expect))
    return cases


@pytest.mark.parametrize("kind", sorted(SAN))
def test_oracle_under_sanitizers(kind, tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not found")
    exe = tmp_path / f"oracle_{kind}"
    cmd = [gcc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math",
           *SAN[kind], DRIVER, "-o", str(exe), "-lcrypto", "-lpthread", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "cannot find" in r.stderr and "san" in r.stderr:
        pytest.skip(f"{kind} runtime not installed: {r.stderr.strip()[:200]}")
    assert r.returncode == 0, r.stderr
    cases = _cases(np.random.default_rng(2024))
    env = dict(os.environ, **ENV[kind])
    run = subprocess.run([str(exe)], input="\n".join(c[0] for c in cases) + "\n", capture_output=True, text=True,
                         env=env, timeout=300)
    for rep in REPORTS:
        assert rep not in run.stderr, run.stderr[-4000:]
    assert run.returncode == 0, (run.returncode, run.stderr[-4000:])
    got = run.stdout.splitlines()
    assert len(got) == len(cases)
    for (line, want), out in zip(cases, got):
        assert out == want, line[:120]
