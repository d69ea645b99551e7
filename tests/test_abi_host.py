"""C-ABI library: loads, exports the header's symbols, host-side logic (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lorenz_cipher.h")


@pytest.fixture(scope="module")
def B():
    from paper_1201_3114_amd import binding

    return binding


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lz_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_binding_surface(B):
    decl = declared_functions()
    assert decl == sorted(B.SIGNATURES), set(decl) ^ set(B.SIGNATURES)


def test_library_exports_every_declared_symbol(B):
    lib = ctypes.CDLL(B.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_struct_layouts(B):
    assert ctypes.sizeof(B.Key) == 64
    assert ctypes.sizeof(B.Params) == 48
    assert ctypes.sizeof(B.Launch) == 16
    assert ctypes.sizeof(B.Completion) == 40


def test_params_default_and_check(B):
    p = B.Params()
    assert B.lib.lz_params_default(ctypes.byref(p)) == 0
    assert (p.dt, p.n_it, p.block_len, list(p.k), list(p.lam)) == (0.01, 3000, 256, [4, 4, 4], [1.0, 1.0, 1.0])
    assert B.lib.lz_params_check(ctypes.byref(p)) == 0
    for field, bad in [("dt", 0.0), ("dt", 0.0150000001), ("dt", 0.024), ("dt", -1.0), ("dt", float("nan")),
                       ("n_it", 0), ("block_len", 0), ("integrator", 3)]:
        q = B.Params()
        B.lib.lz_params_default(ctypes.byref(q))
        setattr(q, field, bad)
        assert B.lib.lz_params_check(ctypes.byref(q)) == B.LZ_E_INVAL, (field, bad)
        assert B.lib.lz_last_error()
    for k in (2, 5, 0):
        q = B.Params()
        B.lib.lz_params_default(ctypes.byref(q))
        q.k[1] = k
        assert B.lib.lz_params_check(ctypes.byref(q)) == B.LZ_E_INVAL
    for ok_field, ok in [("block_len", (1 << 32) - 1), ("integrator", 1), ("integrator", 2), ("dt", 0.015)]:
        q = B.Params()
        B.lib.lz_params_default(ctypes.byref(q))
        setattr(q, ok_field, ok)
        assert B.lib.lz_params_check(ctypes.byref(q)) == 0, (ok_field, ok)
    q = B.Params()
    B.lib.lz_params_default(ctypes.byref(q))
    q.lam[2] = 0.05  # outside 0.090 < lambda_3 < 62
    assert B.lib.lz_params_check(ctypes.byref(q)) == B.LZ_E_INVAL
    assert B.lib.lz_params_check(None) == B.LZ_E_INVAL
    assert B.lib.lz_ciphertext_len(1000) == 1024


def test_block_count_limits(B):
    """Block b starts at r0 + b 2^-24: at most 2^24 blocks per message, and at most 2^32 bytes."""
    def count(n, block_len=256):
        p = B.Params()
        B.lib.lz_params_default(ctypes.byref(p))
        p.block_len = block_len
        nb = ctypes.c_uint64(0)
        rc = B.lib.lz_block_count(ctypes.byref(p), n, ctypes.byref(nb))
        return rc, nb.value

    assert count(0) == (0, 1)
    assert count(1) == (0, 1)
    assert count(257) == (0, 2)
    assert count(1 << 32) == (0, 1 << 24)
    assert count((1 << 32) + 1)[0] == B.LZ_E_INVAL
    assert count((1 << 32), 255)[0] == B.LZ_E_INVAL
    assert count(1 << 24, 1) == (0, 1 << 24)
    assert count((1 << 24) + 1, 1)[0] == B.LZ_E_INVAL
    assert count(3 << 24, 3) == (0, 1 << 24)
    assert count((3 << 24) + 1, 3)[0] == B.LZ_E_INVAL
    assert b"2^24" in B.lib.lz_last_error()
    assert B.lib.lz_block_count(None, 5, None) == B.LZ_E_INVAL


def _lib_key(B, pw, k=(4, 4, 4)):
    p = B.Params()
    B.lib.lz_params_default(ctypes.byref(p))
    p.k[:] = list(k)
    key = B.Key()
    buf, n = B.pw_buf(pw)
    assert B.lib.lz_key_setup(buf, n, ctypes.byref(p), ctypes.byref(key)) == 0
    return key


def test_key_setup_matches_oracle_all_lengths(B):
    """Host key setup (own bignum division, own SHA-256) equals the oracle (strtod, OpenSSL)."""
    rng = np.random.default_rng(21)
    for n in list(range(1, 65)) * 3:
        pw = bytes(rng.integers(0, 256, n, dtype=np.uint8))  # any byte values
        for k in ((4, 4, 4), (3, 4, 3)):
            got = _lib_key(B, pw, k)
            want = oracle.key_setup(pw, k=k)
            assert list(got.a_prime) == want["a_prime"], (n, pw)
            assert list(got.r0) == want["r0"]
            assert list(got.mu) == want["mu"]
            assert list(got.omega) == want["omega"]
            assert list(got.k) == list(k)


def test_key_setup_hand_values(B):
    import json

    cases = json.load(open(os.path.join(ROOT, "tests", "golden", "keysetup_hand.json")))["cases"]
    for c in cases:
        key = _lib_key(B, c["pw"].encode())
        assert list(key.mu) == c["mu"]
        assert list(key.a_prime) == [a / 10.0 ** c["D"] for a in c["a"]]


def test_key_setup_rejects_bad_lengths(B):
    p = B.Params()
    B.lib.lz_params_default(ctypes.byref(p))
    key = B.Key()
    buf, _ = B.pw_buf(b"x" * 65)
    assert B.lib.lz_key_setup(buf, 0, ctypes.byref(p), ctypes.byref(key)) == B.LZ_E_INVAL
    assert B.lib.lz_key_setup(buf, 65, ctypes.byref(p), ctypes.byref(key)) == B.LZ_E_INVAL
    assert B.lib.lz_key_setup(None, 3, ctypes.byref(p), ctypes.byref(key)) == B.LZ_E_INVAL
    assert B.lib.lz_key_setup(buf, 64, ctypes.byref(p), ctypes.byref(key)) == 0


def test_null_handles_rejected_without_gpu(B):
    assert B.lib.lz_context_create(0, None, None) == B.LZ_E_INVAL
    assert B.lib.lz_encrypt(None, None, 0, None, 0, None, None) == B.LZ_E_INVAL
    assert B.lib.lz_decrypt(None, None, 0, None, 0, None, None, None) == B.LZ_E_INVAL
    assert B.lib.lz_batch_launch(None, None) == B.LZ_E_INVAL
    assert B.lib.lz_encrypt_batch(None, None, None) == B.LZ_E_INVAL
    assert B.lib.lz_decrypt_batch(None, None, None, None) == B.LZ_E_INVAL
    assert B.lib.lz_server_submit(None, 0, 0, None, 0, None, 0, None, 0) == B.LZ_E_INVAL
    assert B.lib.lz_context_destroy(None) == 0
    assert B.lib.lz_batch_destroy(None) == 0
    assert B.lib.lz_server_destroy(None) == 0


def test_sha256_via_key_setup_hashlib(B):
    """Omega = SHA-256(i a) mod 4 recomputed with hashlib from the packed integers."""
    import hashlib

    from oracle import pyref

    rng = np.random.default_rng(22)
    for n in range(1, 65):
        pw = bytes(rng.integers(32, 127, n, dtype=np.uint8))
        a = pyref.pack(pw)
        key = _lib_key(B, pw)
        for i in (1, 2, 3):
            msg = b"".join((i * x).to_bytes(32, "little") for x in a)
            assert key.omega[i - 1] == int.from_bytes(hashlib.sha256(msg).digest(), "big") % 4


def test_header_is_plain_c_and_links(tmp_path):
    """The header compiles as C99 and C++17 with no HIP or torch headers, and a C program that
    calls only host-side entry points links against the library and runs (no GPU needed)."""
    import os
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    inc = os.path.join(root, "include")
    libdir = os.path.join(root, "paper_1201_3114_amd")
    src = tmp_path / "use.c"
    src.write_text(r'''
#include <stdio.h>
#include <string.h>
#include "lorenz_cipher.h"
int main(void) {
    lz_params p;
    lz_key k;
    if (lz_params_default(&p) != LZ_OK || lz_params_check(&p) != LZ_OK) return 1;
    if (lz_ciphertext_len(100) != 100 + LZ_TAG_BYTES) return 2;
    if (lz_key_setup((const uint8_t *)"123456", 6, &p, &k) != LZ_OK) return 3;
    if (k.mu[0] != 0 || k.mu[1] != 2 || k.mu[2] != 2) return 4;
    if (lz_key_setup((const uint8_t *)"", 0, &p, &k) != LZ_E_INVAL || strlen(lz_last_error()) == 0) return 5;
    uint64_t nb = 0;
    if (lz_block_count(&p, LZ_MAX_MESSAGE, &nb) != LZ_OK || nb != LZ_MAX_BLOCKS) return 6;
    /* the batch calls of the problem statement, over a batch handle; no GPU here, so NULL handles */
    if (lz_encrypt_batch(NULL, NULL, NULL) != LZ_E_INVAL) return 7;
    if (lz_decrypt_batch(NULL, NULL, NULL, NULL) != LZ_E_INVAL) return 8;
    p.dt = LZ_MAX_DT * 1.0000001;
    if (lz_params_check(&p) != LZ_E_INVAL) return 9;
    /* the entry point without allocation rejects a missing status word before any HIP call */
    if (lz_decrypt_noalloc(NULL, (const uint8_t *)"pw", 2, (const uint8_t *)&k, 64, (uint8_t *)&k, NULL, NULL)
        != LZ_E_INVAL) return 10;
    if (lz_autotune_cached(NULL, NULL, 0.0, NULL, NULL) != LZ_E_INVAL) return 11;
    if (sizeof(lz_server_config) != 24 || LZ_SERVE_ADAPTIVE != 0 || LZ_SERVE_ALL_CHAINS != 1) return 12;
    if (LZ_NOALLOC_SCRATCH_BYTES < 3 * sizeof(uint64_t)) return 13;
    printf("ok\n");
    return 0;
}
''')
    for std, comp, name in (("-std=c99", "gcc", "use.c"), ("-std=c++17", "g++", "use.c")):
        cmd = [comp, std, "-Wall", "-Werror", "-I", inc, "-fsyntax-only"] + (["-x", "c++"] if comp == "g++" else []) + [str(src)]
        subprocess.run(cmd, check=True)
    exe = tmp_path / "use"
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-L", libdir, "-llorenz_cipher",
                    f"-Wl,-rpath,{libdir}", "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", (out.returncode, out.stdout, out.stderr)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus above 1 exits with status 2 and a JSON message, before any GPU work."""
    import json
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and "--gpus must be 1" in msg["error"]


def test_decrypt_noalloc_rejects_bad_arguments_on_the_host(B):
    """lz_decrypt_noalloc checks its arguments before any HIP call: the stand-in pointers below are
    never dereferenced (no GPU is needed)."""
    p = B.Params()
    B.lib.lz_params_default(ctypes.byref(p))
    buf, npw = B.pw_buf(b"password")
    fake = ctypes.c_void_p(4096)
    cases = [
        (ctypes.byref(p), buf, npw, fake, 23, fake, fake, "shorter than the 24-byte tag"),
        (ctypes.byref(p), buf, npw, fake, 100, fake, None, "d_status"),
        (ctypes.byref(p), buf, 0, fake, 100, fake, fake, "password length"),
        (ctypes.byref(p), buf, 65, fake, 100, fake, fake, "password length"),
        (ctypes.byref(p), None, npw, fake, 100, fake, fake, "NULL"),
        (ctypes.byref(p), buf, npw, None, 100, fake, fake, "NULL"),
        (ctypes.byref(p), buf, npw, fake, 100, None, fake, "NULL plaintext"),
        (ctypes.byref(p), buf, npw, fake, (1 << 32) + 25, fake, fake, "2^32"),
    ]
    for *args, msg in cases:
        assert B.lib.lz_decrypt_noalloc(*args, None) == B.LZ_E_INVAL, msg
        assert msg.encode() in B.lib.lz_last_error(), (msg, B.lib.lz_last_error())
    q = B.Params()
    B.lib.lz_params_default(ctypes.byref(q))
    q.block_len = 16
    assert B.lib.lz_decrypt_noalloc(ctypes.byref(q), buf, npw, fake, (1 << 28) + 25, fake, fake, None) == B.LZ_E_INVAL
    assert b"blocks" in B.lib.lz_last_error()
    q.dt = 0.02
    assert B.lib.lz_decrypt_noalloc(ctypes.byref(q), buf, npw, fake, 100, fake, fake, None) == B.LZ_E_INVAL
