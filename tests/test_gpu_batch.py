"""Batched path (persistent kernel in a HIP graph) vs the oracle and the plain path."""
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


def _make(lz, sizes, pws, seed):
    import torch

    rng = np.random.default_rng(seed)
    plains = [rng.integers(0, 256, int(n), dtype=np.uint8) for n in sizes]
    in_off, in_tot = lz.packed_offsets(sizes, 0)
    out_off, out_tot = lz.packed_offsets(sizes, 24)
    flat = np.concatenate(plains) if in_tot else np.zeros(1, np.uint8)
    d_in = to_dev(flat if len(flat) else np.zeros(1, np.uint8))
    d_out = torch.zeros(max(out_tot, 1), dtype=torch.uint8, device="cuda")
    return plains, in_off, out_off, d_in, d_out


def _slices(arr, offs, lens):
    return [arr[int(o):int(o) + int(n)] for o, n in zip(offs, lens)]


@pytest.mark.parametrize("shape", [None, (1, 64, 16, 1), (2, 256, 64, 2), (4, 64, 32, 2), (1, 256, 128, 8)])
def test_batch_small_vs_oracle(lz, shape):
    """Mixed sizes (empty, sub-block, exact blocks, ragged), own passwords, vs the oracle."""
    import torch

    rng = np.random.default_rng(31)
    sizes = [0, 1, 255, 256, 257, 512, 1000, 4096, 33, 70000, 0, 12345, 256 * 64, 3 * 256 + 1] + \
            list(rng.integers(0, 9000, 30))
    pws = [bytes(rng.integers(32, 127, int(rng.integers(8, 65)), dtype=np.uint8)) for _ in sizes]
    plains, in_off, out_off, d_in, d_out = _make(lz, sizes, pws, 32)
    ctx = lz.Context(0, lz.params(n_it=30))
    sh = lz.LaunchShape(*shape) if shape else None
    say("batch shape", sh)
    b = lz.Batch(ctx, False, sizes, pws, d_in, in_off, d_out, out_off, shape=sh)
    b.launch()
    C = host(d_out)
    cts = _slices(C, out_off, [n + 24 for n in sizes])
    for i, (P, pw) in enumerate(zip(plains, pws)):
        assert np.array_equal(cts[i], oracle.encrypt(pw, P, n_it=30)), i
    # decrypt batch, with two tampered ciphertexts
    flat_c = C.copy()
    bad = [3, 9]
    for i in bad:
        flat_c[int(out_off[i]) + int(rng.integers(0, sizes[i] + 24))] ^= 0x40
    d_cin = to_dev(flat_c)
    d_pout = torch.full((max(sum(sizes), 1),), 0xAB, dtype=torch.uint8, device="cuda")
    p_off, _ = lz.packed_offsets(sizes, 0)
    st = torch.full((len(sizes),), 99, dtype=torch.int32, device="cuda")
    bd = lz.Batch(ctx, True, sizes, pws, d_cin, out_off, d_pout, p_off, d_status=st, shape=sh)
    bd.launch()
    Pout = host(d_pout)
    status = st.cpu().numpy()
    for i, P in enumerate(plains):
        got = Pout[int(p_off[i]):int(p_off[i]) + sizes[i]]
        if i in bad:
            assert status[i] == -2, i
            assert not got.any()
            assert not oracle.decrypt(pws[i], flat_c[int(out_off[i]):int(out_off[i]) + sizes[i] + 24], n_it=30)[1]
        else:
            assert status[i] == 0, i
            assert np.array_equal(got, P), i


def test_batch_graph_replays(lz):
    """Replaying the captured graph gives the same bytes every time, with eager work in between."""
    import torch

    rng = np.random.default_rng(33)
    sizes = list(rng.integers(1, 3000, 64))
    pws = [b"replay-%d" % i for i in range(len(sizes))]
    plains, in_off, out_off, d_in, d_out = _make(lz, sizes, pws, 34)
    ctx = lz.Context(0, lz.params(n_it=20))
    b = lz.Batch(ctx, False, sizes, pws, d_in, in_off, d_out, out_off)
    b.launch()
    first = host(d_out).copy()
    for r in range(4):
        d_out.fill_(0x5A)  # eager work between replays
        torch.cuda.synchronize()
        b.launch()
        assert np.array_equal(host(d_out), first), r
    cts = _slices(first, out_off, [n + 24 for n in sizes])
    for i in (0, 17, 63):
        assert np.array_equal(cts[i], oracle.encrypt(pws[i], plains[i], n_it=20))


def test_batch_equals_plain_path(lz):
    rng = np.random.default_rng(35)
    sizes = [int(x) for x in rng.integers(100, 40000, 24)]
    pws = [bytes(rng.integers(32, 127, 20, dtype=np.uint8)) for _ in sizes]
    plains, in_off, out_off, d_in, d_out = _make(lz, sizes, pws, 36)
    ctx = lz.Context(0)
    b = lz.Batch(ctx, False, sizes, pws, d_in, in_off, d_out, out_off)
    b.launch()
    C = host(d_out)
    for i in range(len(sizes)):
        one = ctx.encrypt(to_dev(plains[i]), pws[i])
        assert np.array_equal(host(one), C[int(out_off[i]):int(out_off[i]) + sizes[i] + 24]), i
    # and the oracle on two of them (full n_it)
    for i in (0, 5):
        assert np.array_equal(C[int(out_off[i]):int(out_off[i]) + sizes[i] + 24],
                              oracle.encrypt(pws[i], plains[i], nthreads=ORACLE_THREADS))


def test_batch_and_integrity_full_config(lz):
    """4096 messages, log-uniform 1 KiB..1 MiB, own 8..64-byte passwords (one persistent launch);
    then 10% of the ciphertexts with one flipped byte: the untouched 90% decrypt exactly and every
    altered one is flagged and zeroed.  Sampled messages are checked against the oracle."""
    import torch

    from paper_1201_3114_amd import workloads

    wl = workloads.batch()
    sizes = wl.sizes
    n = len(sizes)
    say("batch config", n, int(sizes.sum()))
    ctx = lz.Context(0)
    in_off = wl.offsets.astype(np.uint64)
    out_off, out_tot = lz.packed_offsets(sizes, 24)
    d_in = to_dev(wl.data)
    d_out = torch.empty(out_tot, dtype=torch.uint8, device="cuda")
    b = lz.Batch(ctx, False, sizes, wl.passwords, d_in, in_off, d_out, out_off)
    b.launch()
    torch.cuda.synchronize()
    C = host(d_out)
    rng = np.random.default_rng(7)
    small = [i for i in range(n) if sizes[i] <= 4096]
    picks = sorted(set(list(rng.choice(small, 6, replace=False)) + [int(np.argmax(sizes))]))
    B = 256
    for i in picks:
        P = wl.data[int(in_off[i]):int(in_off[i]) + int(sizes[i])]
        ct = C[int(out_off[i]):int(out_off[i]) + int(sizes[i]) + 24]
        if sizes[i] <= 4096:
            assert np.array_equal(ct, oracle.encrypt(wl.passwords[i], P, nthreads=ORACLE_THREADS)), i
        else:  # largest message: sampled blocks
            nb = (int(sizes[i]) + B - 1) // B
            for blk in sorted(set([0, nb - 1] + list(rng.integers(0, nb, 6)))):
                seg = P[blk * B:(blk + 1) * B]
                out, _ = oracle.crypt_block(wl.passwords[i], int(blk), seg)
                assert np.array_equal(ct[blk * B:blk * B + len(seg)], out), (i, blk)
    # integrity: flip one byte in 10% of the ciphertexts
    idx, offs, vals = workloads.tamper_plan(sizes + 24)
    for i, o, v in zip(idx, offs, vals):
        C[int(out_off[i]) + int(o)] ^= v
    d_cin = to_dev(C)
    d_pout = torch.empty(int(sizes.sum()), dtype=torch.uint8, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    bd = lz.Batch(ctx, True, sizes, wl.passwords, d_cin, out_off, d_pout, in_off, d_status=st)
    bd.launch()
    torch.cuda.synchronize()
    status = st.cpu().numpy()
    bad = np.zeros(n, bool)
    bad[idx] = True
    assert (status[bad] == -2).all()
    assert (status[~bad] == 0).all()
    Pout = host(d_pout)
    same = Pout == wl.data
    for i in range(n):
        s, e = int(in_off[i]), int(in_off[i]) + int(sizes[i])
        if bad[i]:
            assert not Pout[s:e].any(), i
        else:
            assert same[s:e].all(), i
    # the oracle flags sampled altered ciphertexts too
    for i in [int(j) for j in idx if sizes[j] <= 4096][:3]:
        ct = C[int(out_off[i]):int(out_off[i]) + int(sizes[i]) + 24]
        assert not oracle.decrypt(wl.passwords[i], ct, nthreads=ORACLE_THREADS)[1]


def test_autotune_picks_a_valid_shape_and_keeps_results(lz):
    """The autotuner (with a small n_it so the sweep is quick) stores a valid shape in the context; a batch
    launched with it gives the same bytes as the plain path and the oracle."""
    import torch

    rng = np.random.default_rng(31)
    ctx = lz.Context(0, lz.params(n_it=20))
    before = ctx.get_launch()
    best = ctx.autotune()
    assert ctx.get_launch() == best
    assert best.chains_per_lane in (1, 2, 4) and best.wg_size in (64, 128, 256) and best.tile in (16, 32, 64, 128)
    say("autotune", before, "->", best)
    sizes = [int(x) for x in rng.integers(0, 5000, 60)]
    pws = [bytes(rng.integers(32, 127, int(rng.integers(8, 65)), dtype=np.uint8)) for _ in sizes]
    data = rng.integers(0, 256, int(sum(sizes)), dtype=np.uint8)
    in_off, _ = lz.packed_offsets(sizes, 0)
    out_off, out_tot = lz.packed_offsets(sizes, 24)
    d_out = torch.zeros(out_tot, dtype=torch.uint8, device="cuda")
    d_in = to_dev(data) if len(data) else torch.zeros(1, dtype=torch.uint8, device="cuda")
    b = lz.Batch(ctx, False, sizes, pws, d_in, in_off, d_out, out_off)
    b.launch()
    C = host(d_out)
    b.close()
    for i in range(0, len(sizes), 7):
        P = data[int(in_off[i]):int(in_off[i]) + sizes[i]]
        want = oracle.encrypt(pws[i], P, n_it=20)
        assert np.array_equal(C[int(out_off[i]):int(out_off[i]) + sizes[i] + 24], want), i
        if sizes[i]:
            assert np.array_equal(host(ctx.encrypt(to_dev(P), pws[i])), want), i


def test_autotune_cache_per_device(lz, tmp_path):
    """lz_autotune_cached tunes once and writes one entry keyed by the device and the parameters; the
    next call (another context) takes the shape from the file; another n_it is another entry; a damaged
    entry is dropped and tuned again."""
    path = str(tmp_path / "shapes.tsv")
    ctx = lz.Context(0, lz.params(n_it=20))
    shape, hit = ctx.autotune_cached(path)
    assert not hit and ctx.get_launch() == shape
    lines = open(path).read().splitlines()
    say("cache after tuning:", lines)
    assert len(lines) == 1 and "n_it=20" in lines[0] and "gfx" in lines[0]
    key, val, ms = lines[0].split("\t")
    assert [int(v) for v in val.split()] == [shape.chains_per_lane, shape.wg_size, shape.tile, shape.waves_per_simd]
    assert float(ms) > 0
    ctx2 = lz.Context(0, lz.params(n_it=20))
    shape2, hit2 = ctx2.autotune_cached(path)
    assert hit2 and shape2 == shape and ctx2.get_launch() == shape
    ctx3 = lz.Context(0, lz.params(n_it=21))
    _, hit3 = ctx3.autotune_cached(path)
    assert not hit3 and len(open(path).read().splitlines()) == 2
    # damage the n_it=20 entry (only that line): an invalid tile
    text = "".join((l.replace(val, "1 256 100 4") if "n_it=20" in l else l) + "\n"
                   for l in open(path).read().splitlines())
    open(path, "w").write(text)
    ctx4 = lz.Context(0, lz.params(n_it=20))
    shape4, hit4 = ctx4.autotune_cached(path)
    assert not hit4 and shape4.tile in (16, 32, 64, 128)
    lines = open(path).read().splitlines()
    assert len(lines) == 2 and sum("n_it=20" in l for l in lines) == 1 and "1 256 100 4" not in open(path).read()
    for c in (ctx, ctx2, ctx3, ctx4):
        c.close()
