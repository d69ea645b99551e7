"""Integrator formats (Euler with FMA, RK4) and the sequential version (block_len >= n) on the GPU
vs the oracle, bit for bit."""
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


@pytest.mark.parametrize("integ", ["euler_fma", "rk4"])
@pytest.mark.parametrize("m", [1, 2, 4])
def test_variant_plain_vs_oracle(lz, integ, m):
    rng = np.random.default_rng(51)
    ctx = lz.Context(0, lz.params(n_it=20, integrator=integ))
    try:
        ctx.set_launch(lz.LaunchShape(m, 64, 32, 4))
    except lz.LorenzError:
        pytest.skip("shape over the LDS limit")
    for n in (0, 1, 255, 257, 130 * 256 + 17):
        P = rng.integers(0, 256, n, dtype=np.uint8)
        say(integ, m, n)
        C = ctx.encrypt(to_dev(P), b"variant %d" % n)
        want = oracle.encrypt(b"variant %d" % n, P, nthreads=ORACLE_THREADS, n_it=20, integrator=integ)
        assert np.array_equal(host(C), want), (integ, m, n)
        assert np.array_equal(host(ctx.decrypt(C, b"variant %d" % n)), P)


@pytest.mark.parametrize("integ", ["euler_fma", "rk4"])
def test_variant_full_iterations_64k(lz, integ):
    from paper_1201_3114_amd import workloads

    P, pw = workloads.plain("plain_64k")
    ctx = lz.Context(0, lz.params(integrator=integ))
    C = ctx.encrypt(to_dev(P), pw)
    assert np.array_equal(host(C), oracle.encrypt(pw, P, nthreads=ORACLE_THREADS, integrator=integ))
    bad = C.clone()
    bad[777] ^= 4
    with pytest.raises(lz.IntegrityError):
        ctx.decrypt(bad, pw)


@pytest.mark.parametrize("integ", ["euler", "euler_fma", "rk4"])
def test_variant_batch_and_serve(lz, integ):
    import torch

    rng = np.random.default_rng(52)
    sizes = [int(x) for x in rng.integers(0, 3000, 40)]
    pws = [bytes(rng.integers(32, 127, 12, dtype=np.uint8)) for _ in sizes]
    plains = [rng.integers(0, 256, n, dtype=np.uint8) for n in sizes]
    ctx = lz.Context(0, lz.params(n_it=15, integrator=integ))
    in_off, _ = lz.packed_offsets(sizes, 0)
    out_off, out_tot = lz.packed_offsets(sizes, 24)
    d_in = to_dev(np.concatenate(plains))
    d_out = torch.zeros(out_tot, dtype=torch.uint8, device="cuda")
    b = lz.Batch(ctx, False, sizes, pws, d_in, in_off, d_out, out_off)
    b.launch()
    C = host(d_out)
    for i in range(len(sizes)):
        want = oracle.encrypt(pws[i], plains[i], n_it=15, integrator=integ)
        assert np.array_equal(C[int(out_off[i]):int(out_off[i]) + sizes[i] + 24], want), i
    srv = lz.Server(ctx, hbm_budget=1 << 28, tick_bytes=16)
    dsts = [torch.zeros(n + 24, dtype=torch.uint8, device="cuda") for n in sizes]
    for i in range(len(sizes)):
        srv.submit(i, False, pws[i], d_in.data_ptr() + int(in_off[i]), sizes[i], dsts[i].data_ptr())
    done = 0
    while done < len(sizes):
        done += len(srv.poll(64, 100))
    srv.close()
    for i in range(len(sizes)):
        assert np.array_equal(host(dsts[i]), C[int(out_off[i]):int(out_off[i]) + sizes[i] + 24]), i


@pytest.mark.parametrize("block_len", [1 << 20, (1 << 32) - 1])
def test_sequential_version_plain_and_batch(lz, block_len):
    """block_len >= n: each message is one chain (the paper's sequential strong version)."""
    import torch

    rng = np.random.default_rng(53)
    ctx = lz.Context(0, lz.params(n_it=30, block_len=block_len))
    sizes = [0, 1, 200, 1000, 2500] + [int(x) for x in rng.integers(1, 2000, 20)]
    pws = [bytes(rng.integers(32, 127, 20, dtype=np.uint8)) for _ in sizes]
    plains = [rng.integers(0, 256, n, dtype=np.uint8) for n in sizes]
    for i in range(5):
        C = ctx.encrypt(to_dev(plains[i]) if sizes[i] else torch.zeros(0, dtype=torch.uint8, device="cuda"), pws[i])
        want = oracle.encrypt(pws[i], plains[i], n_it=30, block_len=block_len)
        assert np.array_equal(host(C), want), i
        # the sequential version is block 0 of the block mode
        if sizes[i] > 256:
            blocked = oracle.encrypt(pws[i], plains[i], n_it=30)
            assert np.array_equal(host(C)[:256], blocked[:256])
    in_off, _ = lz.packed_offsets(sizes, 0)
    out_off, out_tot = lz.packed_offsets(sizes, 24)
    d_in = to_dev(np.concatenate(plains))
    d_out = torch.zeros(out_tot, dtype=torch.uint8, device="cuda")
    b = lz.Batch(ctx, False, sizes, pws, d_in, in_off, d_out, out_off)
    b.launch()
    C = host(d_out)
    for i in range(len(sizes)):
        want = oracle.encrypt(pws[i], plains[i], n_it=30, block_len=block_len)
        assert np.array_equal(C[int(out_off[i]):int(out_off[i]) + sizes[i] + 24], want), i


def test_sequential_version_full_parameters(lz):
    """The benchmark's sequential-version workload (4,096 messages of 256 B..4 KiB, block_len 2^32 - 1,
    n_it 3000) run as one batch; the first eight messages and the longest one equal the oracle."""
    import torch

    from paper_1201_3114_amd import workloads

    wl = workloads.batch(count=4096, seed=workloads.SEED["sequential"], lo=256, hi=4096)
    bl = (1 << 32) - 1
    ctx = lz.Context(0, lz.params(block_len=bl))
    sizes = wl.sizes
    out_off, out_tot = lz.packed_offsets(sizes, 24)
    d_out = torch.zeros(out_tot, dtype=torch.uint8, device="cuda")
    b = lz.Batch(ctx, False, sizes, wl.passwords, to_dev(wl.data), wl.offsets, d_out, out_off)
    b.launch()
    C = host(d_out)
    b.close()
    pick = list(range(8)) + [int(np.argmax(sizes))]
    say("sequential messages", [int(sizes[i]) for i in pick])
    for i in pick:
        P = wl.data[int(wl.offsets[i]):int(wl.offsets[i]) + int(sizes[i])]
        want = oracle.encrypt(wl.passwords[i], P, block_len=bl)
        assert np.array_equal(C[int(out_off[i]):int(out_off[i]) + int(sizes[i]) + 24], want), i
