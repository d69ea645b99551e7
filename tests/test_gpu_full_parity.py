"""Full-size parity: every byte and every tag of the large workloads against the CPU oracle.

* the 64 MiB message (262,144 blocks, 1,024 workgroups of the plain kernel) at the method's
  n_it = 3000, in the benchmark's launch configuration: every ciphertext byte and the tag;
* a 4 MiB message (16,384 blocks, 64 workgroups) at n_it = 30: every byte and the tag, both
  directions;
* the 4,096-message batch (log-uniform 1 KiB..1 MiB, own passwords) at n_it = 30: every
  message's ciphertext and tag, one persistent launch;
* its integrity variant: 409 ciphertexts with one altered byte; every status against the
  oracle's decrypt, every released plaintext against the oracle's;
* the same batch under every launch shape the autotuner can choose (the benchmark times the
  shape it picks on the device at hand): each shape's ciphertexts equal the ones checked
  against the oracle, and its decrypt returns the plaintexts.

The oracle runs block ranges on up to 16 host threads and the tests print a line per slice.
"""
import time

import numpy as np
import pytest

import oracle
from gpu_util import ORACLE_THREADS, host, need_gpu, say, to_dev

B = 256


@pytest.fixture(scope="module")
def lz():
    need_gpu()
    import paper_1201_3114_amd as lz

    return lz


def _oracle_sliced(pw, P, slices, **kw):
    """The oracle's ciphertext of P (body and tag) computed slice by slice over whole blocks."""
    n = len(P)
    nb = max(1, -(-n // B))
    per = -(-nb // slices)
    body = np.empty(n, dtype=np.uint8)
    tag = [0, 0, 0]
    t0 = time.time()
    for s, b0 in enumerate(range(0, nb, per)):
        lo, hi = b0 * B, min(n, (b0 + per) * B)
        out, part = oracle.crypt_range(pw, b0, P[lo:hi], nthreads=ORACLE_THREADS, **kw)
        body[lo:hi] = out
        tag = [t ^ p for t, p in zip(tag, part)]
        say(f"  oracle slice {s + 1}: blocks {b0}..{min(nb, b0 + per) - 1} ({time.time() - t0:.0f} s)")
    tag_bytes = np.frombuffer(b"".join(int(t).to_bytes(8, "little") for t in tag), dtype=np.uint8)
    return np.concatenate([body, tag_bytes])


def test_oracle_slices_equal_whole_message():
    """The sliced oracle equals its whole-message call (CPU only: guards the helper above)."""
    rng = np.random.default_rng(501)
    P = rng.integers(0, 256, 37 * B + 101, dtype=np.uint8)
    want = oracle.encrypt(b"slices", P, nthreads=4, n_it=5)
    assert np.array_equal(_oracle_sliced(b"slices", P, 5, n_it=5), want)


@pytest.mark.gpu
def test_plain_64m_every_byte_and_tag(lz):
    """64 MiB, 32-byte password, n_it = 3000, the benchmark's shape: the whole ciphertext
    (67,108,864 body bytes and the 24-byte tag) equals the oracle's; decryption returns P."""
    import torch

    from paper_1201_3114_amd import workloads

    P, pw = workloads.plain("plain_64m")
    say("plain_64m full parity:", len(P), "bytes, oracle threads", ORACLE_THREADS)
    ctx = lz.Context(0)
    dP = to_dev(P)
    C = ctx.encrypt(dP, pw)
    got = host(C)
    want = _oracle_sliced(pw, P, 8)
    diff = np.flatnonzero(got != want)
    assert diff.size == 0, f"{diff.size} bytes differ, first at {diff[:8]}"
    Q = ctx.decrypt(C, pw)
    assert torch.equal(Q, dP)
    ctx.close()


@pytest.mark.gpu
def test_64_workgroups_every_byte_and_tag(lz):
    """4 MiB (16,384 blocks = 64 workgroups of 256 lanes) at n_it = 30: every byte and the tag,
    encrypt and decrypt, and a flipped tag byte fails on both sides."""
    rng = np.random.default_rng(502)
    n = 4 << 20
    P = rng.integers(0, 256, n, dtype=np.uint8)
    pw = bytes(rng.integers(32, 127, 29, dtype=np.uint8))
    say("4 MiB at n_it 30")
    ctx = lz.Context(0, lz.params(n_it=30))
    C = ctx.encrypt(to_dev(P), pw)
    got = host(C)
    want = _oracle_sliced(pw, P, 4, n_it=30)
    assert np.array_equal(got, want)
    assert np.array_equal(host(ctx.decrypt(C, pw)), P)
    Po, ok = oracle.decrypt(pw, want, nthreads=ORACLE_THREADS, n_it=30)
    assert ok and np.array_equal(Po, P)
    C[n + 11] ^= 0x40
    with pytest.raises(lz.IntegrityError):
        ctx.decrypt(C, pw)
    bad = want.copy()
    bad[n + 11] ^= 0x40
    assert not oracle.decrypt(pw, bad, nthreads=ORACLE_THREADS, n_it=30)[1]
    ctx.close()


@pytest.fixture(scope="module")
def batch_n30(lz):
    """The 4,096-message batch encrypted on the GPU at n_it = 30 in one persistent launch."""
    import torch

    from paper_1201_3114_amd import workloads

    wl = workloads.batch()
    say("batch at n_it 30:", len(wl.sizes), "messages,", int(wl.sizes.sum()), "bytes")
    ctx = lz.Context(0, lz.params(n_it=30))
    in_off = wl.offsets.astype(np.uint64)
    out_off, out_tot = lz.packed_offsets(wl.sizes, 24)
    d_out = torch.empty(out_tot, dtype=torch.uint8, device="cuda")
    b = lz.Batch(ctx, False, wl.sizes, wl.passwords, to_dev(wl.data), in_off, d_out, out_off)
    b.encrypt()
    C = host(d_out)
    b.close()
    yield ctx, wl, in_off, out_off, C
    ctx.close()


@pytest.mark.gpu
def test_batch_every_message(lz, batch_n30):
    """Every one of the 4,096 ciphertexts (body and tag) equals the oracle's."""
    ctx, wl, in_off, out_off, C = batch_n30
    t0, bad = time.time(), []
    for i, n in enumerate(wl.sizes):
        n = int(n)
        P = wl.data[int(in_off[i]):int(in_off[i]) + n]
        want = oracle.encrypt(wl.passwords[i], P, nthreads=ORACLE_THREADS, n_it=30)
        if not np.array_equal(C[int(out_off[i]):int(out_off[i]) + n + 24], want):
            bad.append(i)
        if i % 1024 == 1023:
            say(f"  {i + 1} messages checked, {len(bad)} differ ({time.time() - t0:.0f} s)")
    assert not bad, f"{len(bad)} messages differ, first {bad[:8]}"


@pytest.mark.gpu
def test_batch_integrity_every_status(lz, batch_n30):
    """409 of the 4,096 ciphertexts get one altered byte (tag included); the batched decrypt's
    4,096 statuses equal the oracle's decrypt results, released plaintexts equal the oracle's
    and the rejected ones are zero."""
    import torch

    from paper_1201_3114_amd import workloads

    ctx, wl, in_off, out_off, C = batch_n30
    sizes = wl.sizes
    n_msg = len(sizes)
    C = C.copy()
    idx, offs, vals = workloads.tamper_plan(sizes + 24)
    for i, o, v in zip(idx, offs, vals):
        C[int(out_off[i]) + int(o)] ^= v
    d_pout = torch.empty(int(sizes.sum()), dtype=torch.uint8, device="cuda")
    st = torch.full((n_msg,), 7, dtype=torch.int32, device="cuda")
    bd = lz.Batch(ctx, True, sizes, wl.passwords, to_dev(C), out_off, d_pout, in_off)
    bd.decrypt(st)
    status = host(st)
    Pout = host(d_pout)
    bd.close()
    t0, wrong = time.time(), []
    for i, n in enumerate(sizes):
        n = int(n)
        ct = C[int(out_off[i]):int(out_off[i]) + n + 24]
        Po, ok = oracle.decrypt(wl.passwords[i], ct, nthreads=ORACLE_THREADS, n_it=30)
        if int(status[i]) != (0 if ok else -2) or not np.array_equal(Pout[int(in_off[i]):int(in_off[i]) + n], Po):
            wrong.append(i)
        if i % 1024 == 1023:
            say(f"  {i + 1} statuses checked, {len(wrong)} differ ({time.time() - t0:.0f} s)")
    assert not wrong, f"{len(wrong)} messages differ from the oracle, first {wrong[:8]}"
    assert int((status == -2).sum()) == len(idx) and int((status == 0).sum()) == n_msg - len(idx)


def tuner_grid():
    """The launch shapes the autotuner times: chains per lane m in 1, 2, 4 and resident waves per
    SIMD w with 4 <= m * w <= 8, workgroups of 64..256 lanes, 16..128-byte tiles (the context's
    default shape is one of them)."""
    for m in (1, 2, 4):
        for w in (1, 2, 4, 8):
            if not 4 <= m * w <= 8:
                continue
            for wg in (256, 128, 64):
                for tile in (128, 64, 32, 16):
                    yield m, wg, tile, w


@pytest.mark.gpu
def test_batch_every_tuner_shape(lz, batch_n30):
    """The full 4,096-message batch at n_it = 30 under each of the 72 shapes: the ciphertexts and
    tags equal the oracle-checked ones of the default shape, byte for byte, and the batched decrypt
    returns every plaintext with status 0. A shape the device cannot hold is rejected at creation."""
    import torch

    ctx, wl, in_off, out_off, C = batch_n30
    sizes = wl.sizes
    d_in = to_dev(wl.data)
    d_want = to_dev(C)
    d_out = torch.empty_like(d_want)
    d_back = torch.empty_like(d_in)
    st = torch.empty(len(sizes), dtype=torch.int32, device="cuda")
    assert ctx.get_launch() in [lz.LaunchShape(*g) for g in tuner_grid()]
    ran, rejected, t0 = 0, [], time.time()
    for g in tuner_grid():
        sh = lz.LaunchShape(*g)
        try:
            be = lz.Batch(ctx, False, sizes, wl.passwords, d_in, in_off, d_out, out_off, shape=sh)
        except lz.LorenzError:
            rejected.append(g)
            continue
        d_out.fill_(0)
        be.encrypt()
        be.close()
        assert torch.equal(d_out, d_want), f"shape {g}: ciphertexts differ"
        d_back.fill_(0)
        st.fill_(7)
        bd = lz.Batch(ctx, True, sizes, wl.passwords, d_out, out_off, d_back, in_off, d_status=st, shape=sh)
        bd.decrypt(st)
        bd.close()
        assert torch.equal(d_back, d_in), f"shape {g}: plaintexts differ"
        assert int((st != 0).sum()) == 0, f"shape {g}: a status is not 0"
        ran += 1
        if ran % 12 == 0:
            say(f"  {ran} shapes equal ({time.time() - t0:.0f} s)")
    say(f"  {ran} shapes ran, {len(rejected)} rejected: {rejected}")
    assert ran + len(rejected) == 72 and ran >= 48
