"""Served path (continuous batching): every result equals the plain path, alone and in a mix."""
import time

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


def _drain(srv, count, timeout_s=120):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < count:
        assert time.time() < t_end, "server did not complete in time"
        for c in srv.poll(4096, 100):
            got[c[0]] = c
    return got


def _requests(lz, ctx, rng, count, max_size, n_it):
    """Mixed encrypt/decrypt requests with device buffers; decrypt inputs made by the plain path."""
    import torch

    reqs = []
    for i in range(count):
        n = int(rng.integers(0, max_size))
        pw = bytes(rng.integers(32, 127, int(rng.integers(16, 65)), dtype=np.uint8))
        P = to_dev(rng.integers(0, 256, n, dtype=np.uint8)) if n else torch.zeros(1, dtype=torch.uint8, device="cuda")
        dec = bool(rng.integers(0, 2))
        if dec:
            C = ctx.encrypt(P[:n] if n else P[:0], pw)
            src, dst = C, torch.zeros(max(n, 1), dtype=torch.uint8, device="cuda")
        else:
            src, dst = P, torch.zeros(n + 24, dtype=torch.uint8, device="cuda")
        reqs.append(dict(id=i, n=n, pw=pw, P=P, dec=dec, src=src, dst=dst))
    torch.cuda.synchronize()
    return reqs


def _expected(ctx, r):
    if r["dec"]:
        return host(r["P"][:r["n"]])
    return host(ctx.encrypt(r["P"][:r["n"]] if r["n"] else r["P"][:0], r["pw"]))


def test_serve_mix_equals_plain(lz):
    rng = np.random.default_rng(41)
    ctx = lz.Context(0, lz.params(n_it=40))
    reqs = _requests(lz, ctx, rng, 120, 20000, 40)
    srv = lz.Server(ctx, hbm_budget=1 << 30, tick_bytes=16)
    t0 = lz.now_ns()
    for r in reqs:  # staggered arrivals: later requests join while earlier ones run
        srv.submit(r["id"], r["dec"], r["pw"], r["src"].data_ptr(), r["n"], r["dst"].data_ptr(),
                   t0 + 200_000 * r["id"])
    got = _drain(srv, len(reqs))
    st = srv.stats()
    srv.close()
    say("serve stats", st)
    assert st["completed"] == len(reqs) and st["ticks"] > 1
    for r in reqs:
        assert got[r["id"]][1] == 0, r["id"]
        n_out = r["n"] if r["dec"] else r["n"] + 24
        assert np.array_equal(host(r["dst"])[:n_out], _expected(ctx, r)), r["id"]


def test_serve_cancel(lz):
    """Cancelled requests (not yet arrived, waiting, running, already finished, and an unknown id): a
    cancelled request reports LZ_E_CANCELLED and leaves its output untouched unless it finished first;
    every other request's output equals the plain path; afterwards a request needing all 4096 chain slots
    is admitted (so no cancelled request kept a slot), then a second wave completes."""
    import torch

    rng = np.random.default_rng(45)
    ctx = lz.Context(0, lz.params())  # a 256-byte chain is about 20 ms of serial work
    reqs = _requests(lz, ctx, rng, 150, 30000, 3000)
    for r in reqs:
        r["dst"].fill_(0xA5)
    srv = lz.Server(ctx, hbm_budget=1 << 28, max_chains=4096, tick_bytes=8)
    t0 = lz.now_ns()
    for r in reqs:  # the last 30 arrive 40..70 ms later
        late = r["id"] >= 120
        srv.submit(r["id"], r["dec"], r["pw"], r["src"].data_ptr(), r["n"], r["dst"].data_ptr(),
                   t0 + (40_000_000 + 1_000_000 * (r["id"] - 120) if late else 50_000 * r["id"]))
    cancel_late = {r["id"] for r in reqs if r["id"] >= 120 and r["id"] % 3 == 0}
    for i in cancel_late:
        srv.cancel(i)
    time.sleep(0.008)  # the first 120 have arrived; most of those admitted are running
    cancel_mid = {r["id"] for r in reqs if r["id"] < 120 and r["id"] % 5 == 2}
    for i in sorted(cancel_mid, reverse=True):
        srv.cancel(i)
    srv.cancel(99_999)
    got = _drain(srv, len(reqs))
    cancelled = cancel_late | cancel_mid
    n_cancelled = 0
    for r in reqs:
        status = got[r["id"]][1]
        n_out = r["n"] if r["dec"] else r["n"] + 24
        if r["id"] in cancelled and status == -6:
            n_cancelled += 1
            assert (host(r["dst"]) == 0xA5).all(), r["id"]
            continue
        assert status == 0, (r["id"], status)
        assert np.array_equal(host(r["dst"])[:n_out], _expected(ctx, r)), r["id"]
    say("cancelled", n_cancelled, "of", len(cancelled))
    for i in cancel_late:  # cancelled before they arrived: completed at once, before their arrival time
        assert got[i][1] == -6 and got[i][4] < got[i][2], (i, got[i])
    assert n_cancelled > len(cancel_late)  # some were cancelled while waiting or running
    # a request that needs every chain slot is admitted only if no cancelled request kept any
    big = dict(id=500, n=4096 * 256, pw=b"all-slots-password", dec=False)
    big["P"] = big["src"] = to_dev(rng.integers(0, 256, big["n"], dtype=np.uint8))
    big["dst"] = torch.zeros(big["n"] + 24, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    srv.submit(500, False, big["pw"], big["src"].data_ptr(), big["n"], big["dst"].data_ptr())
    assert _drain(srv, 1, 60)[500][1] == 0
    assert np.array_equal(host(big["dst"]), _expected(ctx, big))
    # then a second wave
    wave = _requests(lz, ctx, rng, 60, 30000, 3000)
    for r in wave:
        srv.submit(1000 + r["id"], r["dec"], r["pw"], r["src"].data_ptr(), r["n"], r["dst"].data_ptr())
    got2 = _drain(srv, len(wave))
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) + 1 + len(wave)
    for r in wave:
        assert got2[1000 + r["id"]][1] == 0
        n_out = r["n"] if r["dec"] else r["n"] + 24
        assert np.array_equal(host(r["dst"])[:n_out], _expected(ctx, r)), r["id"]


def test_serve_alone_equals_in_mix(lz):
    """The same request gives the same bytes alone on an idle server and inside a mix."""
    import torch

    rng = np.random.default_rng(42)
    ctx = lz.Context(0, lz.params(n_it=60))
    P = to_dev(rng.integers(0, 256, 5 * 256 + 100, dtype=np.uint8))
    pw = b"alone-or-mixed"
    outs = []
    for mixed in (False, True):
        srv = lz.Server(ctx, hbm_budget=1 << 28, tick_bytes=8)
        dst = torch.zeros(P.numel() + 24, dtype=torch.uint8, device="cuda")
        others = _requests(lz, ctx, rng, 40, 6000, 60) if mixed else []
        for r in others[:20]:
            srv.submit(1000 + r["id"], r["dec"], r["pw"], r["src"].data_ptr(), r["n"], r["dst"].data_ptr())
        srv.submit(7, False, pw, P.data_ptr(), P.numel(), dst.data_ptr())
        for r in others[20:]:
            srv.submit(1000 + r["id"], r["dec"], r["pw"], r["src"].data_ptr(), r["n"], r["dst"].data_ptr())
        _drain(srv, 1 + len(others))
        srv.close()
        outs.append(host(dst).copy())
        for r in others:
            n_out = r["n"] if r["dec"] else r["n"] + 24
            assert np.array_equal(host(r["dst"])[:n_out], _expected(ctx, r))
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], host(ctx.encrypt(P, pw)))
    assert np.array_equal(outs[0], oracle.encrypt(pw, host(P), n_it=60))


def test_serve_integrity_budget_and_host_buffers(lz):
    """Tampered ciphertext -> LZ_E_INTEGRITY and zeroed output; a request larger than the budget
    completes with LZ_E_NOMEM; host (pageable) buffers work as sources and destinations; a budget
    that holds only a few requests at a time still completes everything in order."""
    rng = np.random.default_rng(43)
    ctx = lz.Context(0, lz.params(n_it=30))
    pw = b"served integrity"
    P = rng.integers(0, 256, 3000, dtype=np.uint8)
    C = host(ctx.encrypt(to_dev(P), pw))
    C_bad = C.copy()
    C_bad[1234] ^= 1
    out_ok = np.full(3000, 0xEE, np.uint8)
    out_bad = np.full(3000, 0xEE, np.uint8)
    big = np.zeros(4 << 20, np.uint8)
    big_out = np.zeros((4 << 20) + 24, np.uint8)
    srv = lz.Server(ctx, hbm_budget=3 << 20, max_chains=4096, tick_bytes=32)
    srv.submit(1, True, pw, C.ctypes.data, 3000, out_ok.ctypes.data)
    srv.submit(2, True, pw, C_bad.ctypes.data, 3000, out_bad.ctypes.data)
    srv.submit(3, False, pw, big.ctypes.data, len(big), big_out.ctypes.data)
    many = [rng.integers(0, 256, 100_000, dtype=np.uint8) for _ in range(12)]
    many_out = [np.zeros(100_024, np.uint8) for _ in many]
    for i, (m, o) in enumerate(zip(many, many_out)):
        srv.submit(10 + i, False, pw, m.ctypes.data, len(m), o.ctypes.data)
    got = _drain(srv, 3 + len(many))
    st = srv.stats()
    srv.close()
    assert got[1][1] == 0 and np.array_equal(out_ok, P)
    assert got[2][1] == -2 and not out_bad.any()
    assert got[3][1] == -3
    assert st["peak_hbm"] <= 3 << 20
    for i, (m, o) in enumerate(zip(many, many_out)):
        assert got[10 + i][1] == 0
        assert np.array_equal(o, oracle.encrypt(pw, m, nthreads=8, n_it=30)), i


def test_serve_submit_many_replay(lz):
    """Bulk submission with future arrival times replays a trace; every result equals the plain path."""
    rng = np.random.default_rng(44)
    ctx = lz.Context(0, lz.params(n_it=25))
    reqs = _requests(lz, ctx, rng, 300, 9000, 25)
    srv = lz.Server(ctx, hbm_budget=1 << 30, tick_bytes=32)
    base = lz.now_ns() + 200_000_000
    arr = [base + 50_000 * r["id"] for r in reqs]
    srv.submit_many([r["id"] for r in reqs], [r["dec"] for r in reqs], [r["pw"] for r in reqs],
                    [r["src"].data_ptr() for r in reqs], [r["n"] for r in reqs], [r["dst"].data_ptr() for r in reqs],
                    arr)
    got = _drain(srv, len(reqs))
    srv.close()
    for r in reqs:
        rid, status, a, adm, dn = got[r["id"]]
        assert status == 0
        assert a == arr[r["id"]] and adm >= a and dn >= adm
        n_out = r["n"] if r["dec"] else r["n"] + 24
        assert np.array_equal(host(r["dst"])[:n_out], _expected(ctx, r)), r["id"]


def test_serve_workload_prefix_vs_batched_and_oracle(lz):
    """The first 2,000 requests of the 200,000-request serving workload (lognormal sizes, mixed
    directions, 16..64-byte passwords, Poisson arrivals at 12,000 requests/s) at full parameters
    (n_it 3000): every result equals the batched path (bit-identical to the plain path) and a seeded
    1% sample, at most 1 MiB in all, equals the oracle."""
    import torch

    from paper_1201_3114_amd import workloads

    count = 2000
    tr = workloads.serve_trace(count=count, qps=12000.0)
    sizes = tr.sizes.astype(np.int64)
    rng = np.random.default_rng(workloads.SEED["serve_data"])
    P_all = rng.integers(0, 256, int(sizes.sum()), dtype=np.uint8)
    in_off = np.zeros(count, np.int64)
    in_off[1:] = np.cumsum(sizes[:-1])
    ctx = lz.Context(0)
    d_P = to_dev(P_all)
    c_off, c_tot = lz.packed_offsets(sizes, 24)
    c_off = c_off.astype(np.int64)
    d_C = torch.empty(int(c_tot), dtype=torch.uint8, device="cuda")
    b = lz.Batch(ctx, False, sizes, tr.passwords, d_P, in_off, d_C, c_off)
    b.launch()
    torch.cuda.synchronize()
    b.close()
    C_all = host(d_C)
    out_len = np.where(tr.decrypt == 1, sizes, sizes + 24)
    o_off = np.zeros(count, np.int64)
    o_off[1:] = np.cumsum(out_len[:-1])
    d_out = torch.zeros(int(out_len.sum()), dtype=torch.uint8, device="cuda")
    src = [d_C[int(c_off[i]):].data_ptr() if tr.decrypt[i] else d_P[int(in_off[i]):].data_ptr() for i in range(count)]
    dst = [d_out[int(o_off[i]):].data_ptr() for i in range(count)]
    ns = [int(v) for v in sizes]  # plaintext lengths in both directions
    srv = lz.Server(ctx, hbm_budget=8 << 30, tick_bytes=16)
    base = lz.now_ns() + 100_000_000
    arr = [base + int(t * 1e9) for t in tr.arrival_s]
    say("serving", count, "requests,", int(sizes.sum()), "bytes")
    srv.submit_many(list(range(count)), [bool(d) for d in tr.decrypt], tr.passwords, src, ns, dst, arr)
    got = _drain(srv, count, timeout_s=240)
    srv.close()
    out = host(d_out)
    for i in range(count):
        assert got[i][1] == 0, i
        a, n = int(o_off[i]), int(out_len[i])
        want = (P_all[in_off[i]:in_off[i] + sizes[i]] if tr.decrypt[i]
                else C_all[c_off[i]:c_off[i] + sizes[i] + 24])
        assert np.array_equal(out[a:a + n], want), i
    pick, total = [], 0
    for i in np.random.default_rng(workloads.SEED["serve_sample"]).permutation(count):
        if len(pick) == count // 100:
            break
        if total + sizes[i] <= 1 << 20:
            pick.append(int(i))
            total += int(sizes[i])
    say("oracle sample", len(pick), "requests,", total, "bytes")
    assert len(pick) >= 10
    for i in pick:
        a, n, pw = int(o_off[i]), int(sizes[i]), tr.passwords[i]
        P = P_all[in_off[i]:in_off[i] + n]
        if tr.decrypt[i]:
            back, ok = oracle.decrypt(pw, C_all[c_off[i]:c_off[i] + n + 24], nthreads=8)
            assert ok and np.array_equal(back, P) and np.array_equal(out[a:a + n], back), i
        else:
            assert np.array_equal(out[a:a + n + 24], oracle.encrypt(pw, P, nthreads=8)), i


def test_server_and_stream_argument_errors(lz):
    """Bad configurations and arguments are rejected on the host with LZ_E_INVAL, before any work."""
    import torch

    ctx = lz.Context(0, lz.params(n_it=5))
    with pytest.raises(lz.LorenzError):
        lz.Server(ctx, hbm_budget=1 << 16)                    # smaller than the fixed part
    with pytest.raises(lz.LorenzError):
        lz.Server(ctx, hbm_budget=1 << 30, tick_bytes=(1 << 20) + 1)
    with pytest.raises(lz.LorenzError):
        lz.Server(ctx, hbm_budget=1 << 30, run_waves=9)                     # more than 8 waves per SIMD
    import ctypes

    from paper_1201_3114_amd import binding as B

    bad = B.ServerConfig(1 << 30, 0, 16, 0, 2)                              # no such policy
    h = ctypes.c_void_p()
    assert B.lib.lz_server_create(ctx.handle, ctypes.byref(bad), ctypes.byref(h)) == B.LZ_E_INVAL
    assert b"policy" in B.lib.lz_last_error() and not h.value
    srv = lz.Server(ctx, hbm_budget=1 << 28, max_chains=1024, tick_bytes=16)
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(lz.LorenzError):
        srv.submit(1, False, b"", buf.data_ptr(), 10, buf.data_ptr())           # empty password
    with pytest.raises(lz.LorenzError):
        srv.submit(2, False, b"x" * 65, buf.data_ptr(), 10, buf.data_ptr())     # password over 64 bytes
    with pytest.raises(lz.LorenzError):
        srv.submit(3, False, b"pw", 0, 10, buf.data_ptr())                      # NULL source
    with pytest.raises(lz.LorenzError):
        srv.submit(4, True, b"pw", buf.data_ptr(), (1 << 32) + 1, buf.data_ptr())  # over 2^32 bytes
    srv.submit(5, False, b"pw", buf.data_ptr(), 10, buf.data_ptr() + 32)      # a valid one still completes
    got = _drain(srv, 1)
    assert got[5][1] == 0
    srv.close()
    with pytest.raises(lz.LorenzError):
        lz.Stream(ctx, False, b"")
    st = lz.Stream(ctx, False, b"pw")
    st.update(buf[:10], out=torch.empty(10, dtype=torch.uint8, device="cuda"))
    st.finish()
    with pytest.raises(lz.LorenzError):
        st.finish()                                                            # finished twice
    st.close()


@pytest.mark.parametrize("max_chains,budget,tick", [(64, 1 << 22, 1), (256, 6 << 20, 7), (1024, 1 << 24, 100)])
def test_serve_slot_reuse_stress(lz, max_chains, budget, tick):
    """Few chain slots and a small arena force constant reuse of slots, request records and memory while
    ticks overlap (two in flight); every result must still equal the plain path."""
    rng = np.random.default_rng(45 + max_chains)
    ctx = lz.Context(0, lz.params(n_it=12))
    reqs = _requests(lz, ctx, rng, 400, 6000, 12)
    srv = lz.Server(ctx, hbm_budget=budget, max_chains=max_chains, tick_bytes=tick)
    base = lz.now_ns() + 50_000_000
    arr = [base + int(x) for x in np.cumsum(rng.exponential(20_000, len(reqs)))]
    srv.submit_many([r["id"] for r in reqs], [r["dec"] for r in reqs], [r["pw"] for r in reqs],
                    [r["src"].data_ptr() for r in reqs], [r["n"] for r in reqs], [r["dst"].data_ptr() for r in reqs],
                    arr)
    got = _drain(srv, len(reqs), timeout_s=240)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["peak_hbm"] <= budget
    for r in reqs:
        assert got[r["id"]][1] == 0, r["id"]
        n_out = r["n"] if r["dec"] else r["n"] + 24
        assert np.array_equal(host(r["dst"])[:n_out], _expected(ctx, r)), (r["id"], r["n"], r["dec"])


# (policy, run_waves, chains of each request in units of one wave per SIMD, ticks, requests that finish last)
TICK_CASES = [
    # one wave per SIMD at most: A, C and D share the first 16 ticks, B (over the cap) runs alone after them
    ("adaptive", 1, [0.5, 1.0625, 0.25, 3], 32, {1}),
    # backlog 1.8 waves (at most 3): one wave per SIMD, the same schedule
    ("adaptive", 4, [0.5, 1.0625, 0.25, 3], 32, {1}),
    # every admitted chain in every tick
    ("all_chains", 4, [0.5, 1.0625, 0.25, 3], 16, set()),
    # backlog 2.7 waves: one wave per SIMD, the requests one after another
    ("adaptive", 4, [0.9, 0.9, 0.9], 48, {1, 2}),
    # backlog 3.6 waves: two waves per SIMD for A and B; then 1.8 waves: one wave, C, then D
    ("adaptive", 4, [0.9, 0.9, 0.9, 0.9], 48, {2, 3}),
    # backlog 6.3 waves: four waves per SIMD for A..D; then 2.7 waves: one wave, E, F, G in turn
    ("adaptive", 4, [0.9] * 7, 64, {4, 5, 6}),
]


@pytest.mark.parametrize("policy,run_waves,units,ticks,last", TICK_CASES)
def test_serve_tick_cap_and_backfill(lz, policy, run_waves, units, ticks, last):
    """More chains than one tick may run: a tick holds 1 wave per SIMD while the backlog is at most 3
    waves, 2 up to 6 waves, then up to run_waves; requests join it in admission order, whole or not at
    all, later ones fill the room an earlier one leaves, and a request larger than the cap still runs.
    An integer entry of `units` is a chain count, a fraction is that part of one wave on every SIMD."""
    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    wave = 4 * 64 * cus
    ctx = lz.Context(0, lz.params(n_it=3))
    rng = np.random.default_rng(460 + run_waves + len(units) + len(policy))
    B = 256
    reqs = []
    for i, u in enumerate(units):
        nb = u if isinstance(u, int) else int(u * wave)
        n = nb * B - int(rng.integers(0, B))
        pw = bytes(rng.integers(32, 127, 20, dtype=np.uint8))
        P = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")
        dec = i % 2 == 1
        if dec:
            src, dst = ctx.encrypt(P, pw), torch.zeros(n, dtype=torch.uint8, device="cuda")
        else:
            src, dst = P, torch.zeros(n + 24, dtype=torch.uint8, device="cuda")
        reqs.append(dict(id=i, n=n, pw=pw, P=P, dec=dec, src=src, dst=dst))
    torch.cuda.synchronize()
    srv = lz.Server(ctx, hbm_budget=4 << 30, tick_bytes=16, run_waves=run_waves, policy=policy)
    at = lz.now_ns() + 20_000_000
    srv.submit_many([r["id"] for r in reqs], [r["dec"] for r in reqs], [r["pw"] for r in reqs],
                    [r["src"].data_ptr() for r in reqs], [r["n"] for r in reqs], [r["dst"].data_ptr() for r in reqs],
                    [at] * len(reqs))
    got = _drain(srv, len(reqs), timeout_s=120)
    st = srv.stats()
    srv.close()
    say(f"{policy}, run_waves {run_waves}, units {units}: ticks {st['ticks']}, done ns", {i: got[i][4] - at for i in got})
    for r in reqs:
        assert got[r["id"]][1] == 0, r["id"]
        n_out = r["n"] if r["dec"] else r["n"] + 24
        assert torch.equal(r["dst"][:n_out], torch.from_numpy(_expected(ctx, r)).cuda()), r["id"]
    assert st["ticks"] == ticks
    done = {i: got[i][4] for i in got}
    if last:
        assert max(done[i] for i in done if i not in last) < min(done[i] for i in last)
