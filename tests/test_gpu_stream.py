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


def _deferred_run(lz, ctx, decrypt, pw, X, cuts, rng, tag=None):
    """Runs the cuts of X through a stream with deferred updates, an immediate update now and then and
    flushes at random points; returns the output (and the tag when encrypting)."""
    import torch

    st = lz.Stream(ctx, decrypt, pw)
    out = torch.empty(sum(b - a for a, b in cuts), dtype=torch.uint8, device="cuda")
    for a, b in cuts:
        r = rng.random()
        if r < 0.1:
            st.update(X[a:b], out=out[a:b])
        else:
            st.update_deferred(X[a:b], out=out[a:b])
        if r > 0.95:
            st.flush()
        assert st.position == b
    res = st.finish(tag=tag)
    st.close()
    return out, res


@pytest.mark.parametrize("n", [0, 1, 257, 70000, 300_001])
def test_deferred_updates_equal_one_shot(lz, n):
    """Deferred updates (chunks staged and run together at a flush, before an immediate update or at the
    end) give the one-shot ciphertext and tag, and decrypt back, whatever the chunking."""
    import torch

    rng = np.random.default_rng(90 + n)
    ctx = lz.Context(0, lz.params(n_it=25))
    P = rng.integers(0, 256, n, dtype=np.uint8)
    Pd = to_dev(P) if n else torch.zeros(0, dtype=torch.uint8, device="cuda")
    one = host(ctx.encrypt(Pd, b"deferred pw"))
    if n <= 70000:
        assert np.array_equal(one, oracle.encrypt(b"deferred pw", P, n_it=25))
    for trial in range(2):
        cuts = _chunks(rng, n) if n else []
        say("n", n, "chunks", len(cuts))
        out, tag = _deferred_run(lz, ctx, False, b"deferred pw", Pd, cuts, rng)
        assert np.array_equal(np.concatenate([host(out), host(tag)]), one), (n, trial)
    C = to_dev(one)
    back, _ = _deferred_run(lz, ctx, True, b"deferred pw", C, _chunks(rng, n) if n else [], rng, tag=C[n:n + 24].clone())
    assert np.array_equal(host(back), P)


@pytest.mark.parametrize("block_len", [5, 16])
def test_deferred_runs_split_chunks_at_the_wave_boundary(lz, block_len):
    """With short blocks a run of one wave per SIMD holds only 65,536 x block_len bytes (minus the part of
    the block it continues), so the chunks of a 1.5-2 MiB message are split between many runs, at positions
    that are mostly not block-aligned: the output and tag still equal the one-shot ones, and decrypt back."""
    import torch

    rng = np.random.default_rng(140 + block_len)
    ctx = lz.Context(0, lz.params(n_it=4, block_len=block_len))
    n = int(rng.integers(1_500_000, 2_000_000))
    P = rng.integers(0, 256, n, dtype=np.uint8)
    Pd = to_dev(P)
    one = host(ctx.encrypt(Pd, b"split pw"))
    cuts, pos = [], 0
    while pos < n:
        step = int(rng.integers(1, 200_000))
        cuts.append((pos, min(n, pos + step)))
        pos += step
    say("block_len", block_len, "n", n, "chunks", len(cuts))
    out, tag = _deferred_run(lz, ctx, False, b"split pw", Pd, cuts, rng)
    assert np.array_equal(np.concatenate([host(out), host(tag)]), one)
    C = to_dev(one)
    back, _ = _deferred_run(lz, ctx, True, b"split pw", C, cuts, rng, tag=C[n:n + 24].clone())
    assert np.array_equal(host(back), P)


def test_deferred_staging_limits(lz):
    """Queued chunks run when they reach one wave on every SIMD (16 MiB on a 256-CU device): 1 MiB chunks
    that reach it exactly and one that crosses it; chunks of that size or more, up to and past the staging
    capacity (LZ_STREAM_DEFER_BYTES, 64 MiB), run at once after the queued ones; and more than
    LZ_STREAM_DEFER_CHUNKS small chunks.  The 166 MiB result equals the one-shot ciphertext (itself checked
    against the oracle at full size elsewhere)."""
    import torch

    MiB = 1 << 20
    ctx = lz.Context(0, lz.params(n_it=4))
    steps = [MiB] * 63 + [MiB + 3, 64 * MiB, MiB - 3, 16 * MiB - 5, 20 * MiB] + [7] * 4999
    n = sum(steps) + 11
    Pd = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda",
                       generator=torch.Generator(device="cuda").manual_seed(93))
    one = ctx.encrypt(Pd, b"staging pw")
    cuts, pos = [], 0
    for step in steps:
        cuts.append((pos, pos + step))
        pos += step
    cuts.append((pos, n))
    assert cuts[-1][0] <= n
    say("staging limits:", len(cuts), "chunks,", n, "bytes")
    st = lz.Stream(ctx, False, b"staging pw")
    out = torch.empty(n, dtype=torch.uint8, device="cuda")
    for a, b in cuts:
        st.update_deferred(Pd[a:b], out=out[a:b])
    tag = st.finish()
    st.close()
    assert torch.equal(torch.cat([out, tag]), one)


def test_deferred_tamper_and_calls_after_finish(lz):
    """A decrypt stream of deferred updates flags an altered byte at the end; a flush with nothing queued
    is a no-op; deferred updates and flushes after finish are rejected."""
    import torch

    rng = np.random.default_rng(94)
    ctx = lz.Context(0, lz.params(n_it=25))
    P = rng.integers(0, 256, 9000, dtype=np.uint8)
    C = ctx.encrypt(to_dev(P), b"tamper deferred")
    for flip in (0, 4444, 8999, 9010):
        bad = C.clone()
        bad[flip] ^= 0x10
        st = lz.Stream(ctx, True, b"tamper deferred")
        st.flush()
        out = torch.empty(9000, dtype=torch.uint8, device="cuda")
        for a in range(0, 9000, 1000):
            st.update_deferred(bad[a:a + 1000], out=out[a:a + 1000])
        status = torch.full((1,), 9, dtype=torch.int32, device="cuda")
        st.finish(tag=bad[9000:].clone(), status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == -2, flip
        with pytest.raises(lz.LorenzError):
            st.update_deferred(bad[:10], out=out[:10])
        with pytest.raises(lz.LorenzError):
            st.flush()
        st.close()


def test_deferred_two_streams_on_two_hip_streams(lz):
    """Two messages, each as deferred updates alternating between two HIP streams (a stream's calls are
    ordered among themselves across HIP streams), flushed midway: both equal their one-shot results."""
    import torch

    rng = np.random.default_rng(95)
    ctx = lz.Context(0, lz.params(n_it=25))
    Ps = [rng.integers(0, 256, n, dtype=np.uint8) for n in (50_000, 33_333)]
    Pds = [to_dev(P) for P in Ps]
    ones = [host(ctx.encrypt(Pd, pw)) for Pd, pw in zip(Pds, (b"one", b"two"))]
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    sts = [lz.Stream(ctx, False, pw) for pw in (b"one", b"two")]
    outs = [torch.empty(len(P), dtype=torch.uint8, device="cuda") for P in Ps]
    torch.cuda.synchronize()
    cuts = [_chunks(rng, len(P)) for P in Ps]
    for i in range(max(len(c) for c in cuts)):
        for m in range(2):
            if i < len(cuts[m]):
                a, b = cuts[m][i]
                sts[m].update_deferred(Pds[m][a:b], out=outs[m][a:b], stream=hs[(i + m) % 2])
                if i == len(cuts[m]) // 2:
                    sts[m].flush(stream=hs[(i + m + 1) % 2])
    tags = [sts[m].finish(stream=hs[m]) for m in range(2)]
    torch.cuda.synchronize()
    for m in range(2):
        assert np.array_equal(np.concatenate([host(outs[m]), host(tags[m])]), ones[m]), m
        sts[m].close()
