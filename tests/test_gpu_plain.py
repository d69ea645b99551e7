"""GPU plain path vs the CPU oracle, bit for bit (Sections 3.2 and 5)."""
import numpy as np
import pytest

import oracle
from gpu_util import ORACLE_THREADS, host, need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lz():
    need_gpu()
    import paper_1201_3114_amd as lz

    return lz


def _ctx(lz, **kw):
    return lz.Context(0, lz.params(**kw))


def test_plain_64k_config_bit_exact(lz):
    """64 KiB uniform bytes, 16-byte printable password, default parameters: E and D vs oracle."""
    from paper_1201_3114_amd import workloads

    P, pw = workloads.plain("plain_64k")
    say("plain_64k", len(P), pw)
    ctx = _ctx(lz)
    C = ctx.encrypt(to_dev(P), pw)
    want = oracle.encrypt(pw, P, nthreads=ORACLE_THREADS)
    assert np.array_equal(host(C), want)
    Q = ctx.decrypt(C, pw)
    assert np.array_equal(host(Q), P)
    Qo, ok = oracle.decrypt(pw, want, nthreads=ORACLE_THREADS)
    assert ok and np.array_equal(Qo, P)


@pytest.mark.parametrize("n", [0, 1, 2, 63, 64, 65, 255, 256, 257, 1000, 3 * 256 + 77, 64 * 256, 64 * 256 + 1,
                               300 * 256 + 131])
def test_plain_sizes_ragged(lz, n):
    """Empty, sub-block, exact-block and ragged messages spanning several LDS tiles and waves."""
    rng = np.random.default_rng(1000 + n)
    P = rng.integers(0, 256, n, dtype=np.uint8)
    pw = bytes(rng.integers(32, 127, 1 + n % 64, dtype=np.uint8))
    say("ragged n", n)
    ctx = _ctx(lz, n_it=40)
    C = ctx.encrypt(to_dev(P), pw)
    want = oracle.encrypt(pw, P, nthreads=ORACLE_THREADS, n_it=40)
    assert np.array_equal(host(C), want)
    assert np.array_equal(host(ctx.decrypt(C, pw)), P)


@pytest.mark.parametrize("m", [1, 2, 4])
@pytest.mark.parametrize("wg", [64, 256])
@pytest.mark.parametrize("tile", [16, 32, 64, 128])
def test_launch_shapes_identical(lz, m, wg, tile):
    """Every launch shape gives the oracle's bytes (the schedule cannot change the result)."""
    rng = np.random.default_rng(7)
    n = 200 * 256 + 99
    P = rng.integers(0, 256, n, dtype=np.uint8)
    ctx = _ctx(lz, n_it=25)
    shape = lz.LaunchShape(m, wg, tile, 4)
    try:
        ctx.set_launch(shape)
    except lz.LorenzError:
        pytest.skip("shape over the LDS limit of this device")
    say("shape", shape)
    C = ctx.encrypt(to_dev(P), b"shapes")
    want = oracle.encrypt(b"shapes", P, nthreads=ORACLE_THREADS, n_it=25)
    assert np.array_equal(host(C), want)
    assert np.array_equal(host(ctx.decrypt(C, b"shapes")), P)


@pytest.mark.parametrize("kw", [dict(block_len=1), dict(block_len=3), dict(block_len=64), dict(block_len=1000),
                                dict(k=(3, 3, 3)), dict(k=(4, 3, 4)), dict(dt=0.015), dict(dt=0.001),
                                dict(lam=(-15.0, 15.9, 61.5)), dict(n_it=1), dict(n_it=7)])
def test_parameters_vs_oracle(lz, kw):
    rng = np.random.default_rng(11)
    n = 5000
    P = rng.integers(0, 256, n, dtype=np.uint8)
    kw2 = dict(n_it=30)
    kw2.update(kw)
    say("params", kw2)
    ctx = _ctx(lz, **kw2)
    C = ctx.encrypt(to_dev(P), b"parameter sweep")
    want = oracle.encrypt(b"parameter sweep", P, nthreads=ORACLE_THREADS, **kw2)
    assert np.array_equal(host(C), want)


def test_password_lengths_and_bytes(lz):
    rng = np.random.default_rng(12)
    ctx = _ctx(lz, n_it=20)
    for npw in (1, 2, 3, 4, 5, 17, 18, 63, 64):
        pw = bytes(rng.integers(0, 256, npw, dtype=np.uint8))
        P = rng.integers(0, 256, 700, dtype=np.uint8)
        C = ctx.encrypt(to_dev(P), pw)
        assert np.array_equal(host(C), oracle.encrypt(pw, P, n_it=20)), npw


def test_degenerate_and_example_passwords(lz):
    """Passwords whose packed integers are 0 (all-zero bytes: a' = 0, so r0 = lambda on every coordinate) or
    maximal (all 0xFF), one repeated byte, and the paper's example passwords 123456 and 123457 of Section 4."""
    rng = np.random.default_rng(16)
    ctx = _ctx(lz, n_it=40)
    P = rng.integers(0, 256, 1500, dtype=np.uint8)
    pws = [b"\0" * n for n in (1, 2, 3, 6, 64)] + [b"\xff" * n for n in (1, 3, 64)]
    pws += [b"a" * 33, b"123456", b"123457"]
    outs = {}
    for pw in pws:
        C = host(ctx.encrypt(to_dev(P), pw))
        assert np.array_equal(C, oracle.encrypt(pw, P, n_it=40)), pw
        outs[pw] = C
    # the two example passwords differ in one character and give unrelated ciphertexts
    a, b = outs[b"123456"][:1500], outs[b"123457"][:1500]
    assert np.mean(a == b) < 0.02


def test_tamper_detected_and_zeroed(lz):
    """A changed ciphertext byte (body or tag) fails the tag; the plaintext comes back zeroed."""
    import torch

    rng = np.random.default_rng(13)
    P = rng.integers(0, 256, 2000, dtype=np.uint8)
    ctx = _ctx(lz, n_it=50)
    C = ctx.encrypt(to_dev(P), b"tamper")
    for off in (0, 1, 255, 256, 1999, 2000, 2023):
        bad = C.clone()
        bad[off] ^= int(rng.integers(1, 256))
        say("tamper offset", off)
        with pytest.raises(lz.IntegrityError):
            ctx.decrypt(bad, b"tamper")
        st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        out = ctx.decrypt(bad, b"tamper", status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == -2
        assert not host(out).any()
        # the oracle agrees the altered ciphertext fails
        assert not oracle.decrypt(b"tamper", host(bad), n_it=50)[1]
    with pytest.raises(lz.IntegrityError):
        ctx.decrypt(C, b"tamper!")
    st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    ctx.decrypt(C, b"tamper", status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0


def test_streams_and_async_status(lz):
    """Calls on two streams through one context stay ordered; results equal the oracle."""
    import torch

    rng = np.random.default_rng(14)
    ctx = _ctx(lz, n_it=30)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    Ps = [rng.integers(0, 256, 3000 + 17 * i, dtype=np.uint8) for i in range(6)]
    outs = []
    for i, P in enumerate(Ps):
        s = s1 if i % 2 else s2
        with torch.cuda.stream(s):
            d = to_dev(P)
            outs.append(ctx.encrypt(d, b"streams %d" % i, stream=s))
    torch.cuda.synchronize()
    for i, P in enumerate(Ps):
        assert np.array_equal(host(outs[i]), oracle.encrypt(b"streams %d" % i, P, n_it=30))


def test_invalid_arguments(lz):
    import torch

    ctx = _ctx(lz)
    with pytest.raises(lz.LorenzError):
        ctx.encrypt(torch.zeros(10, dtype=torch.uint8, device="cuda"), b"")
    with pytest.raises(lz.LorenzError):
        ctx.encrypt(torch.zeros(10, dtype=torch.uint8, device="cuda"), b"x" * 65)
    with pytest.raises(ValueError):
        ctx.decrypt(torch.zeros(10, dtype=torch.uint8, device="cuda"), b"pw")
    with pytest.raises(lz.LorenzError):
        ctx.set_launch(lz.LaunchShape(3, 256, 64, 4))
    with pytest.raises(lz.LorenzError):
        lz.Context(0, lz.params(dt=0.03))
    for bad in (dict(dt=0.0), dict(dt=-0.01), dict(n_it=0), dict(block_len=0), dict(k=(5, 4, 4)), dict(k=(4, 2, 4))):
        with pytest.raises(lz.LorenzError):
            lz.Context(0, lz.params(**bad))


def test_truncated_and_extended_ciphertexts(lz):
    """The tag is the last 24 bytes: a ciphertext cut short or with bytes appended is rejected (its tag
    and body no longer match) and the output zeroed; fewer than 24 bytes is an argument error."""
    import torch

    rng = np.random.default_rng(15)
    P = rng.integers(0, 256, 700, dtype=np.uint8)
    ctx = _ctx(lz, n_it=40)
    C = ctx.encrypt(to_dev(P), b"cut")
    variants = {"cut 1": C[:-1], "cut 24": C[:-24], "cut 300": C[:-300],
                "extended 1": torch.cat([C, C[:1]]), "extended 256": torch.cat([C, C[:256]])}
    for name, bad in variants.items():
        say(name)
        st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        out = ctx.decrypt(bad.contiguous(), b"cut", status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == -2, name
        assert not host(out).any(), name
        assert not oracle.decrypt(b"cut", host(bad), n_it=40)[1], name
    with pytest.raises(ValueError):
        ctx.decrypt(C[:23].contiguous(), b"cut")


def test_plain_64m_sampled(lz):
    """64 MiB, 32-byte password, the benchmark's launch shape: sampled blocks vs oracle,
    round trip, and tamper detection at sampled offsets."""
    import torch

    from paper_1201_3114_amd import workloads

    P, pw = workloads.plain("plain_64m")
    n = len(P)
    B = 256
    say("plain_64m", n)
    ctx = _ctx(lz)
    dP = to_dev(P)
    C = ctx.encrypt(dP, pw)
    Cg = host(C)
    rng = np.random.default_rng(99)
    nb = n // B
    blocks = sorted(set([0, 1, nb - 1] + list(rng.integers(0, nb, 45))))
    for b in blocks:
        out, _ = oracle.crypt_block(pw, int(b), P[b * B:(b + 1) * B])
        assert np.array_equal(Cg[b * B:(b + 1) * B], out), b
    Q = ctx.decrypt(C, pw)
    assert torch.equal(Q, dP)
    for off in (0, n // 2 + 3, n - 1, n + 5):
        bad = C.clone()
        bad[off] ^= 0x10
        with pytest.raises(lz.IntegrityError):
            ctx.decrypt(bad, pw)


def test_maximum_message_size(lz):
    """The largest message the format allows, 2^32 bytes (16,777,216 blocks; the last block's initial
    condition is r0 + (2^24 - 1) 2^-24): sampled blocks including the first and last equal the oracle,
    the round trip is exact, a flipped last byte or tag byte is detected, and one byte more is rejected
    before any work is queued."""
    import ctypes

    import torch

    from paper_1201_3114_amd import binding as B

    n = 1 << 32
    Bsz = 256
    nb = n // Bsz
    pw = b"maximum size"
    g = torch.Generator(device="cuda")
    g.manual_seed(109)
    say("max size: generating", n, "bytes")
    dP = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=g)
    ctx = _ctx(lz)
    say("max size: encrypt")
    C = ctx.encrypt(dP, pw)
    torch.cuda.synchronize()
    rng = np.random.default_rng(110)
    blocks = sorted(set([0, 1, nb // 2, nb - 2, nb - 1] + [int(b) for b in rng.integers(0, nb, 11)]))
    for b in blocks:
        seg = host(dP[b * Bsz:(b + 1) * Bsz])
        out, _ = oracle.crypt_block(pw, b, seg)
        assert np.array_equal(host(C[b * Bsz:(b + 1) * Bsz]), out), b
    say("max size: decrypt")
    Q = torch.empty(n, dtype=torch.uint8, device="cuda")
    st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    ctx.decrypt(C, pw, out=Q, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and torch.equal(Q, dP)
    for off in (n - 1, n + 23):
        C[off] ^= 0x01
        ctx.decrypt(C, pw, out=Q, status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == -2, off
        assert int(Q[:1 << 20].count_nonzero().item()) == 0 and int(Q[-(1 << 20):].count_nonzero().item()) == 0
        C[off] ^= 0x01
    # n = 2^32 + 1 is rejected on the host, before anything is queued
    pbuf, npw = B.pw_buf(pw)
    rc = B.lib.lz_encrypt(ctx.handle, pbuf, npw, ctypes.c_void_p(dP.data_ptr()), n + 1,
                          ctypes.c_void_p(C.data_ptr()), None)
    assert rc == -1
    del dP, C, Q
    torch.cuda.empty_cache()


def test_block_limit_rejected_on_every_path(lz):
    """A message of more than 2^24 blocks (block b starts at r0 + b 2^-24, so its start would lie 1 or more
    away from r0) is rejected on the host by the plain, batched, streamed and served paths; 2^24 blocks are
    accepted.  Buffers of the full size are passed, so the calls touch only memory they own."""
    import ctypes

    import torch

    from paper_1201_3114_amd import binding as B

    n_ok, n_bad = 1 << 24, (1 << 24) + 1
    ctx = _ctx(lz, block_len=1, n_it=1)
    dP = torch.zeros(n_bad, dtype=torch.uint8, device="cuda")
    dC = torch.zeros(n_bad + 24, dtype=torch.uint8, device="cuda")
    pbuf, npw = B.pw_buf(b"limit")
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    say("block limit: plain")
    assert B.lib.lz_encrypt(ctx.handle, pbuf, npw, vp(dP), n_bad, vp(dC), None) == -1
    assert b"2^24" in B.lib.lz_last_error()
    assert B.lib.lz_decrypt(ctx.handle, pbuf, npw, vp(dC), n_bad + 24, vp(dP), None, None) == -1
    say("block limit: batch")
    with pytest.raises(lz.LorenzError):
        lz.Batch(ctx, False, [n_bad], [b"limit"], dP, [0], dC, [0])
    say("block limit: stream")
    st = lz.Stream(ctx, False, b"limit")
    st.update(dP[:n_ok], dC[:n_ok])
    with pytest.raises(lz.LorenzError):
        st.update(dP[:1], dC[:1])
    st.finish()
    st.close()
    say("block limit: server")
    srv = lz.Server(ctx, 1 << 30)
    with pytest.raises(lz.LorenzError):
        srv.submit(1, False, b"limit", dP.data_ptr(), n_bad, dC.data_ptr())
    srv.close()
    say("block limit: 2^24 blocks accepted")
    ctx.encrypt(dP[:n_ok], b"limit", out=dC[:n_ok + 24])
    torch.cuda.synchronize()
    Q = ctx.decrypt(dC[:n_ok + 24], b"limit")
    assert torch.equal(Q, dP[:n_ok])
    ctx.close()
