"""Streaming (resumable) encryption: any chunking gives the one-shot ciphertext and tag."""
import numpy as np
import pytest

import oracle
from gpu_util import host, need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lz():
    need_gpu()
    import paper_1201_3114_amd as lz

    return lz


def _chunks(rng, n):
    cuts, pos = [], 0
    while pos < n:
        step = int(rng.choice([0, 1, 7, 100, 255, 256, 257, 600, 3000]))
        step = min(step, n - pos)
        cuts.append((pos, pos + step))
        pos += step
    return cuts


def _stream_encrypt(lz, ctx, P_dev, pw, cuts):
    import torch

    st = lz.Stream(ctx, False, pw)
    out = torch.empty(P_dev.numel(), dtype=torch.uint8, device="cuda")
    for a, b in cuts:
        if b > a:
            st.update(P_dev[a:b], out=out[a:b])
        else:
            st.update(P_dev[a:a])
    tag = st.finish()
    st.close()
    return torch.cat([out, tag])


@pytest.mark.parametrize("n", [0, 1, 100, 256, 257, 1000, 70000])
def test_stream_equals_one_shot(lz, n):
    import torch

    rng = np.random.default_rng(60 + n)
    ctx = lz.Context(0, lz.params(n_it=25))
    P = rng.integers(0, 256, n, dtype=np.uint8)
    Pd = to_dev(P) if n else torch.zeros(0, dtype=torch.uint8, device="cuda")
    one = host(ctx.encrypt(Pd, b"stream pw"))
    assert np.array_equal(one, oracle.encrypt(b"stream pw", P, n_it=25))
    for trial in range(3):
        cuts = _chunks(rng, n) if n else []
        say("n", n, "chunks", len(cuts))
        got = host(_stream_encrypt(lz, ctx, Pd, b"stream pw", cuts))
        assert np.array_equal(got, one), (n, trial)
    # decrypt as a stream with another chunking; tag verified at the end
    C = to_dev(one)
    st = lz.Stream(ctx, True, b"stream pw")
    back = torch.empty(n, dtype=torch.uint8, device="cuda")
    for a, b in (_chunks(rng, n) if n else []):
        if b > a:
            st.update(C[a:b], out=back[a:b])
    st.finish(tag=C[n:n + 24].clone())
    st.close()
    assert np.array_equal(host(back), P)


@pytest.mark.parametrize("full", [63, 64, 255, 256, 257])
def test_stream_partial_chains_at_workgroup_edges(lz, full):
    """An update's head and tail chains run as the lanes after its whole blocks: with 63..257 whole
    blocks they fall at the end of a wave or workgroup or spill into the next one.  Each case has a
    head that completes its block, whole blocks, and a tail; then a head that does not complete its
    block (a chunk shorter than the block's rest); decrypting back is checked too."""
    import torch

    rng = np.random.default_rng(70 + full)
    ctx = lz.Context(0, lz.params(n_it=25))
    B = 256
    n = 100 + (B - 100) + full * B + 50 + 30 + 10
    P = rng.integers(0, 256, n, dtype=np.uint8)
    Pd = to_dev(P)
    one = host(ctx.encrypt(Pd, b"edge pw"))
    assert np.array_equal(one, oracle.encrypt(b"edge pw", P, n_it=25))
    a = 100
    b = a + (B - 100) + full * B + 50
    cuts = [(0, a), (a, b), (b, b + 30), (b + 30, n)]  # tail; head + whole + tail; short head; rest
    say("full", full, "cuts", cuts)
    got = host(_stream_encrypt(lz, ctx, Pd, b"edge pw", cuts))
    assert np.array_equal(got, one), full
    C = to_dev(one)
    st = lz.Stream(ctx, True, b"edge pw")
    back = torch.empty(n, dtype=torch.uint8, device="cuda")
    for x, y in cuts:
        st.update(C[x:y], out=back[x:y])
    st.finish(tag=C[n:n + 24].clone())
    st.close()
    assert np.array_equal(host(back), P)


@pytest.mark.parametrize("shape", [(1, 64, 16, 4), (1, 128, 32, 2), (2, 256, 64, 4), (4, 64, 128, 8)])
def test_stream_under_launch_shapes(lz, shape):
    """An update runs one chain per lane with the context's workgroup size and tile whatever its chains-per-lane
    setting; the result equals the one-shot ciphertext made under the same shape."""
    rng = np.random.default_rng(80 + shape[1] + shape[0])
    ctx = lz.Context(0, lz.params(n_it=20))
    ctx.set_launch(lz.LaunchShape(*shape))
    n = 256 * 300 + 77
    P = rng.integers(0, 256, n, dtype=np.uint8)
    Pd = to_dev(P)
    one = host(ctx.encrypt(Pd, b"shape pw"))
    assert np.array_equal(one, oracle.encrypt(b"shape pw", P, n_it=20, nthreads=8))
    cuts = [(0, 5), (5, 5 + 256 * 129 + 3), (5 + 256 * 129 + 3, n)]
    got = host(_stream_encrypt(lz, ctx, Pd, b"shape pw", cuts))
    assert np.array_equal(got, one), shape
    cuts = _chunks(rng, n)
    assert np.array_equal(host(_stream_encrypt(lz, ctx, Pd, b"shape pw", cuts)), one), shape


def test_stream_tamper_and_wrong_tag(lz):
    import torch

    rng = np.random.default_rng(70)
    ctx = lz.Context(0, lz.params(n_it=25))
    P = rng.integers(0, 256, 5000, dtype=np.uint8)
    C = ctx.encrypt(to_dev(P), b"tamper stream")
    for flip in (10, 2599, 4999, 5003):
        bad = C.clone()
        bad[flip] ^= 0x08
        st = lz.Stream(ctx, True, b"tamper stream")
        out = torch.empty(5000, dtype=torch.uint8, device="cuda")
        st.update(bad[:3000], out=out[:3000])
        st.update(bad[3000:5000], out=out[3000:])
        status = torch.full((1,), 9, dtype=torch.int32, device="cuda")
        st.finish(tag=bad[5000:].clone(), status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == -2, flip
        st.close()
    st = lz.Stream(ctx, True, b"tamper stream")
    st.update(C[:5000], out=torch.empty(5000, dtype=torch.uint8, device="cuda"))
    with pytest.raises(lz.IntegrityError):
        st.finish(tag=torch.zeros(24, dtype=torch.uint8, device="cuda"))
    with pytest.raises(lz.LorenzError):
        st.update(C[:10])  # finished
    st.close()


@pytest.mark.parametrize("kw", [dict(block_len=1 << 20), dict(integrator="euler_fma"), dict(integrator="rk4"),
                                dict(block_len=3)])
def test_stream_sequential_and_formats(lz, kw):
    rng = np.random.default_rng(71)
    ctx = lz.Context(0, lz.params(n_it=12, **kw))
    P = rng.integers(0, 256, 2345, dtype=np.uint8)
    Pd = to_dev(P)
    one = host(ctx.encrypt(Pd, b"formats"))
    assert np.array_equal(one, oracle.encrypt(b"formats", P, n_it=12, **kw))
    got = host(_stream_encrypt(lz, ctx, Pd, b"formats", _chunks(rng, len(P))))
    assert np.array_equal(got, one)


def test_two_streams_interleaved_on_two_streams(lz):
    import torch

    rng = np.random.default_rng(72)
    ctx = lz.Context(0, lz.params(n_it=20))
    Ps = [rng.integers(0, 256, 3333, dtype=np.uint8), rng.integers(0, 256, 1111, dtype=np.uint8)]
    devs = [to_dev(p) for p in Ps]
    torch.cuda.synchronize()
    sts = [lz.Stream(ctx, False, b"first"), lz.Stream(ctx, False, b"second")]
    tss = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty(p.numel(), dtype=torch.uint8, device="cuda") for p in devs]
    for a in range(0, 3333, 500):
        for i in (0, 1):
            b = min(a + 500, devs[i].numel())
            if b > a:
                sts[i].update(devs[i][a:b], out=outs[i][a:b], stream=tss[i])
    tags = [sts[i].finish(stream=tss[i]) for i in (0, 1)]
    torch.cuda.synchronize()
    for i, pw in enumerate((b"first", b"second")):
        got = np.concatenate([host(outs[i]), host(tags[i])])
        assert np.array_equal(got, oracle.encrypt(pw, Ps[i], n_it=20))
        sts[i].close()


def test_many_streams_random_chunks(lz):
    """Eight messages streamed at once on four HIP streams, chunk sizes drawn at random (including empty
    and one-byte chunks), encrypt and then decrypt; every ciphertext and tag equals the oracle's."""
    import torch

    rng = np.random.default_rng(73)
    ctx = lz.Context(0, lz.params(n_it=15))
    sizes = [int(x) for x in rng.integers(0, 30000, 8)]
    pws = [bytes(rng.integers(32, 127, int(rng.integers(1, 65)), dtype=np.uint8)) for _ in sizes]
    Ps = [rng.integers(0, 256, n, dtype=np.uint8) for n in sizes]
    devs = [to_dev(p) if len(p) else torch.zeros(0, dtype=torch.uint8, device="cuda") for p in Ps]
    hs = [torch.cuda.Stream() for _ in range(4)]
    outs = [torch.empty(n + 24, dtype=torch.uint8, device="cuda") for n in sizes]
    sts = [lz.Stream(ctx, False, pw) for pw in pws]
    cuts = [_chunks(rng, n) for n in sizes]
    torch.cuda.synchronize()
    for step in range(max(len(c) for c in cuts)):
        for i in range(8):
            if step < len(cuts[i]):
                a, b = cuts[i][step]
                sts[i].update(devs[i][a:b], out=outs[i][a:b], stream=hs[i % 4])
    for i in range(8):
        sts[i].finish(tag=outs[i][sizes[i]:], stream=hs[i % 4])
    torch.cuda.synchronize()
    for i in range(8):
        sts[i].close()
        assert np.array_equal(host(outs[i]), oracle.encrypt(pws[i], Ps[i], n_it=15)), i
    # decrypt every message as a stream with another random chunking, status written asynchronously
    backs = [torch.empty(max(n, 1), dtype=torch.uint8, device="cuda") for n in sizes]
    status = torch.full((8,), 9, dtype=torch.int32, device="cuda")
    # the received tags, kept alive until the asynchronous finishes have read them
    tags = [outs[i][sizes[i]:].clone() for i in range(8)]
    torch.cuda.synchronize()
    dsts = [lz.Stream(ctx, True, pw) for pw in pws]
    for i in range(8):
        for a, b in _chunks(rng, sizes[i]):
            if b > a:
                dsts[i].update(outs[i][a:b], out=backs[i][a:b], stream=hs[(i + 1) % 4])
        dsts[i].finish(tag=tags[i], status=status[i:i + 1], stream=hs[(i + 1) % 4])
    torch.cuda.synchronize()
    assert host(status).tolist() == [0] * 8
    for i in range(8):
        dsts[i].close()
        assert np.array_equal(host(backs[i])[:sizes[i]], Ps[i]), i
