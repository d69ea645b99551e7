"""Benchmark of the Lorenz chaotic cipher on one MI355X.

One step = encrypt + decrypt of a 64 MiB message of uniform random bytes with a
32-byte printable password (parallel version, default parameters, binary64),
inputs resident in HBM.  value = 2 * 64 MiB * steps / timed seconds (GB = 1e9 B).

Beside it, on the same line:
  roofline     the plain kernel's algorithmic binary64 operations per launch over
               its average launch time (HIP events on the launch stream) against
               the FP64 VALU issue peak of the chip;
  cpu_baseline the CPU oracle on a bounded prefix of the same message;
  batched      4096 messages (log-uniform 1 KiB..1 MiB, own passwords) in one
               graph-captured persistent launch, vs the plain path per message,
               and the integrity check of 10% altered ciphertexts;
  served       a Poisson trace of mixed encrypt/decrypt requests at fixed offered
               loads (0.3, 0.5, 0.7, 0.9 of capacity) through the continuous-
               batching server: p50/p99 latency and GB/s under the adaptive tick
               (waves per SIMD from the backlog) and with every admitted chain in
               each tick, and vs the plain path one request at a time on a prefix.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MiB = 1 << 20
GB = 1e9
# MI355X: 256 CUs x 4 SIMDs x 16 binary64 lanes x 2.4 GHz = one binary64 VALU op per lane per clock
FP64_VALU_OPS_PEAK = 256 * 4 * 16 * 2.4e9  # 39.32e12 op/s (78.6 TFLOP/s counts an FMA as two)
FP64_FMA_COUNTED_PEAK = 78.6e12
HBM_PEAK = 8e12


# binary64 operations per step of each integrator format (one VALU instruction each)
STEP_OPS = {"euler": 14, "euler_fma": 9, "rk4": 68}


def fp64_ops_per_byte(n_it: int, integrator: str = "euler") -> int:
    """Algorithmic binary64 operations per message byte: n_it integrator steps (14 operations
    for Euler), the Theta division and add, six alpha * 10^13 products of R_nu, three a' adds."""
    return STEP_OPS[integrator] * n_it + 2 + 6 + 3


def kernel_stamp() -> str:
    """First 16 hex digits of sha256 over the kernel source and the build script (its compiler
    flags shape the kernels' code)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("csrc/kernels.hip", "build.py"):
        with open(os.path.join(ROOT, "paper_1201_3114_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(launch):
    """HBM bytes per plain-kernel launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None when the kernel's code or the launch
    shape differ from those the counters were taken with."""
    path = os.path.join(ROOT, "profiles", "plain_kernel_64MiB.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(("kernel_source_stamp:", "traffic_bytes_per_launch:", "launch_shape:")))
    if fields.get("kernel_source_stamp", "").strip() != kernel_stamp():
        return None
    shape = " ".join(str(launch[k]) for k in ("chains_per_lane", "wg_size", "tile"))
    if fields.get("launch_shape", "").strip() != shape:
        return None
    try:
        return int(fields["traffic_bytes_per_launch"].strip())
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(x, q):
    return float(np.percentile(np.asarray(x, dtype=np.float64), q)) if len(x) else float("nan")


# ---------------------------------------------------------------------------------------------
def bench_plain(lz, torch, steps, warmup):
    from paper_1201_3114_amd import workloads

    P, pw = workloads.plain("plain_64m")
    n = len(P)
    ctx = lz.Context(0)
    dP = torch.from_numpy(P).cuda()
    C = torch.empty(n + 24, dtype=torch.uint8, device="cuda")
    Q = torch.empty(n, dtype=torch.uint8, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.encrypt(dP, pw, out=C)
        ctx.decrypt(C, pw, out=Q, status=st)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        ctx.encrypt(dP, pw, out=C)
        ev[k][1].record(stream)
        ctx.decrypt(C, pw, out=Q, status=st)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    enc_ms = [ev[k][0].elapsed_time(ev[k][1]) for k in range(steps)]
    dec_ms = [ev[k][1].elapsed_time(ev[k][2]) for k in range(steps)]
    ok = bool(torch.equal(Q, dP)) and int(st.item()) == 0
    # outside the timed steps: latency of the 64 KiB workload (256 blocks: four waves, one block's serial time)
    P64, pw64 = workloads.plain("plain_64k")
    d64 = torch.from_numpy(P64).cuda()
    C64 = ctx.encrypt(d64, pw64)
    Q64 = torch.empty_like(d64)
    ctx.decrypt(C64, pw64, out=Q64, status=st)
    e3 = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    e3[0].record(stream)
    ctx.encrypt(d64, pw64, out=C64)
    e3[1].record(stream)
    ctx.decrypt(C64, pw64, out=Q64, status=st)
    e3[2].record(stream)
    torch.cuda.synchronize()
    lat64 = (e3[0].elapsed_time(e3[1]), e3[1].elapsed_time(e3[2]))
    ok = ok and bool(torch.equal(Q64, d64)) and int(st.item()) == 0
    # outside the timed steps: the same round trip from and to pinned host memory, PCIe copies included
    hP = torch.from_numpy(P).pin_memory()
    hC = torch.empty(n + 24, dtype=torch.uint8).pin_memory()
    hQ = torch.empty(n, dtype=torch.uint8).pin_memory()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    e[0].record(stream)
    dP.copy_(hP, non_blocking=True)
    ctx.encrypt(dP, pw, out=C)
    hC.copy_(C, non_blocking=True)
    C.copy_(hC, non_blocking=True)
    ctx.decrypt(C, pw, out=Q, status=st)
    hQ.copy_(Q, non_blocking=True)
    e[1].record(stream)
    torch.cuda.synchronize()
    pcie_ms = e[0].elapsed_time(e[1])
    ok = ok and bool(torch.equal(hQ, hP))
    shape = ctx.get_launch()
    n_it = ctx.params.n_it
    ctx.close()
    return dict(n=n, wall_s=wall, enc_ms=enc_ms, dec_ms=dec_ms, roundtrip_ok=ok, shape=shape, n_it=n_it,
                pcie_ms=pcie_ms, lat64=lat64)


def bench_cpu_baseline(target_s: float = 12.0):
    """The oracle as it stands on a prefix of the 64 MiB message, encrypt then decrypt."""
    import oracle
    from paper_1201_3114_amd import workloads

    P, pw = workloads.plain("plain_64m")
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    threads = max(1, min(16, cores))
    cal = P[: 4 * 256]
    t = time.perf_counter()
    oracle.encrypt(pw, cal, nthreads=1)
    per_byte = (time.perf_counter() - t) / len(cal)
    blocks = max(threads, int(target_s / 2 / (per_byte * 256) * threads) // threads * threads)
    S = min(len(P), blocks * 256)
    sample = P[:S]
    t = time.perf_counter()
    C = oracle.encrypt(pw, sample, nthreads=threads)
    te = time.perf_counter() - t
    t = time.perf_counter()
    Q, ok = oracle.decrypt(pw, C, nthreads=threads)
    td = time.perf_counter() - t
    assert ok and np.array_equal(Q, sample)
    # one thread, on 16 blocks, for the per-core rate
    one = P[:16 * 256]
    t = time.perf_counter()
    oracle.encrypt(pw, one, nthreads=1)
    t1 = time.perf_counter() - t
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=2 * S / (te + td) / GB, unit="GB/s", cores=threads, kind="oracle",
                sample=f"first {S} bytes ({S // 256} blocks) of the 64 MiB message, encrypt then decrypt, "
                       f"{threads} pthreads; enc {te:.2f} s, dec {td:.2f} s",
                one_thread_GBps=len(one) / t1 / GB, host_cores=cores, cpu_model=model)


# ---------------------------------------------------------------------------------------------
def bench_variants(lz, torch, steps=2):
    """Integrator formats on the 64 MiB workload: the explicit-FMA Euler (9 roundings per step)
    and classical RK4 (68), each a distinct ciphertext format."""
    from paper_1201_3114_amd import workloads

    P, pw = workloads.plain("plain_64m")
    n = len(P)
    dP = torch.from_numpy(P).cuda()
    C = torch.empty(n + 24, dtype=torch.uint8, device="cuda")
    Q = torch.empty(n, dtype=torch.uint8, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    res = {}
    for integ in ("euler_fma", "rk4"):
        ctx = lz.Context(0, lz.params(integrator=integ))
        ctx.encrypt(dP, pw, out=C)
        ctx.decrypt(C, pw, out=Q, status=st)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        e[0].record(stream)
        for _ in range(steps):
            ctx.encrypt(dP, pw, out=C)
            ctx.decrypt(C, pw, out=Q, status=st)
        e[1].record(stream)
        torch.cuda.synchronize()
        ms = e[0].elapsed_time(e[1])
        launch_s = ms / 1e3 / (2 * steps)
        ops = n * fp64_ops_per_byte(ctx.params.n_it, integ)
        res[integ] = dict(enc_dec_GBps=2 * n * steps / (ms / 1e3) / GB, avg_launch_ms=launch_s * 1e3,
                          ops_per_byte=fp64_ops_per_byte(ctx.params.n_it, integ),
                          achieved_Tops=ops / launch_s / 1e12, frac_of_issue_peak=ops / launch_s / FP64_VALU_OPS_PEAK,
                          roundtrip_exact=bool(torch.equal(Q, dP)) and int(st.item()) == 0)
        ctx.close()
    return res


def bench_sequential(lz, torch, count=4096):
    """The sequential strong version (one chain per message: block_len >= n), batched one
    message per lane, against the block mode on the same messages."""
    from paper_1201_3114_amd import workloads

    wl = workloads.batch(count=count, seed=workloads.SEED["sequential"], lo=256, hi=4096)
    sizes = wl.sizes
    total = int(sizes.sum())
    in_off = wl.offsets.astype(np.uint64)
    out_off, out_tot = lz.packed_offsets(sizes, 24)
    d_in = torch.from_numpy(wl.data).cuda()
    d_out = torch.empty(out_tot, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    res = dict(messages=count, bytes=total, sizes="log-uniform 256 B..4 KiB, own 8..64-byte passwords")
    for name, bl in (("sequential", (1 << 32) - 1), ("block_256", 256)):
        ctx = lz.Context(0, lz.params(block_len=bl))
        b = lz.Batch(ctx, False, sizes, wl.passwords, d_in, in_off, d_out, out_off)
        b.launch()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        e[0].record(stream)
        b.launch()
        e[1].record(stream)
        torch.cuda.synchronize()
        ms = e[0].elapsed_time(e[1])
        res[name] = dict(encrypt_GBps=total / ms / 1e6, ms=ms, chains=int(count if bl > 4096 else
                                                                           sum((int(x) + 255) // 256 for x in sizes)))
        b.close()
        ctx.close()
    return res


# ---------------------------------------------------------------------------------------------
def bench_streaming(lz, torch):
    """The 64 MiB workload fed through a stream in chunks (one byte more than a power of two, so every
    update has a partial head and tail block), against the one-shot encrypt, both bit-exact."""
    from paper_1201_3114_amd import workloads

    P, pw = workloads.plain("plain_64m")
    n = len(P)
    dP = torch.from_numpy(P).cuda()
    ctx = lz.Context(0)
    stream = torch.cuda.current_stream()
    one = ctx.encrypt(dP, pw)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    e[0].record(stream)
    ctx.encrypt(dP, pw, out=one)
    e[1].record(stream)
    torch.cuda.synchronize()
    res = {"one_shot": dict(ms=e[0].elapsed_time(e[1]), encrypt_GBps=n / e[0].elapsed_time(e[1]) / 1e6)}
    out = torch.empty(n + 24, dtype=torch.uint8, device="cuda")
    for chunk in ((16 << 20) + 1, (4 << 20) + 1, (1 << 20) + 1):
        out.zero_()
        torch.cuda.synchronize()
        e[0].record(stream)
        st = lz.Stream(ctx, False, pw)
        for a in range(0, n, chunk):
            b = min(a + chunk, n)
            st.update(dP[a:b], out=out[a:b])
        out[n:] = st.finish()
        e[1].record(stream)
        torch.cuda.synchronize()
        st.close()
        ms = e[0].elapsed_time(e[1])
        res[f"chunks_of_{chunk}"] = dict(updates=(n + chunk - 1) // chunk, ms=ms, encrypt_GBps=n / ms / 1e6,
                                         equals_one_shot=bool(torch.equal(out, one)))
    # deferred updates: small chunks staged and run together (runs of one wave per SIMD), flushed at the end
    for chunk in ((1 << 20) + 1, (64 << 10) + 1):
        out.zero_()
        st = lz.Stream(ctx, False, pw)
        st.update_deferred(dP[:1], out=out[:1])  # allocates the staging buffer outside the timed region
        st.close()
        torch.cuda.synchronize()
        e[0].record(stream)
        st = lz.Stream(ctx, False, pw)
        for a in range(0, n, chunk):
            b = min(a + chunk, n)
            st.update_deferred(dP[a:b], out=out[a:b])
        out[n:] = st.finish()
        e[1].record(stream)
        torch.cuda.synchronize()
        st.close()
        ms = e[0].elapsed_time(e[1])
        res[f"deferred_chunks_of_{chunk}"] = dict(updates=(n + chunk - 1) // chunk, ms=ms, encrypt_GBps=n / ms / 1e6,
                                                  equals_one_shot=bool(torch.equal(out, one)))
    # a 256 MiB message (uniform bytes from torch's device generator) in chunks of 64 MiB + 1 byte
    g = torch.Generator(device="cuda")
    g.manual_seed(workloads.SEED["plain_64m"])
    big = torch.randint(0, 256, (256 << 20,), dtype=torch.uint8, device="cuda", generator=g)
    nb = big.numel()
    one = ctx.encrypt(big, pw)
    torch.cuda.synchronize()
    e[0].record(stream)
    ctx.encrypt(big, pw, out=one)
    e[1].record(stream)
    torch.cuda.synchronize()
    ms1 = e[0].elapsed_time(e[1])
    out = torch.empty(nb + 24, dtype=torch.uint8, device="cuda")
    chunk = (64 << 20) + 1
    e[0].record(stream)
    st = lz.Stream(ctx, False, pw)
    for a in range(0, nb, chunk):
        b = min(a + chunk, nb)
        st.update(big[a:b], out=out[a:b])
    out[nb:] = st.finish()
    e[1].record(stream)
    torch.cuda.synchronize()
    st.close()
    ms = e[0].elapsed_time(e[1])
    res["256MiB_one_shot"] = dict(ms=ms1, encrypt_GBps=nb / ms1 / 1e6)
    res[f"256MiB_chunks_of_{chunk}"] = dict(updates=(nb + chunk - 1) // chunk, ms=ms, encrypt_GBps=nb / ms / 1e6,
                                           equals_one_shot=bool(torch.equal(out, one)))
    ctx.close()
    return res


# ---------------------------------------------------------------------------------------------
def bench_diag(lz, torch, reps=5):
    """Section 4 analyses on ciphertext-like (uniform random) bytes: histogram of 1 GiB (HBM-bound),
    the autocorrelation up to lag 256 of 16 MiB, the 2-D power spectrum and autocorrelation matrix
    of a 1024 x 1024 byte image (two / four FFT passes), and the power spectrum of a 1000 x 1000
    image (mixed-radix FFT passes) and of a 1009 x 1009 image (two direct DFT passes on the binary64
    matrix cores)."""
    from paper_1201_3114_amd import workloads

    ctx = lz.Context(0)
    g = torch.Generator(device="cuda")
    g.manual_seed(workloads.SEED["diagnostics"])
    x = torch.randint(0, 256, (64 * MiB,), dtype=torch.uint8, device="cuda", generator=g)
    img = x[:1 << 20].view(1024, 1024)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record(stream)
        for _ in range(reps):
            fn()
        e[1].record(stream)
        torch.cuda.synchronize()
        return e[0].elapsed_time(e[1]) / reps

    res = {}
    # the histogram on 1 GiB (the 64 MiB input repeated), so per-call host overhead does not dominate
    big = x.repeat(16)
    ms = timed(lambda: lz.histogram(ctx, big))
    res["histogram_1GiB"] = dict(ms=ms, GBps=big.numel() / ms / 1e6, frac_of_hbm=big.numel() / ms * 1e3 / HBM_PEAK)
    # skewed inputs put equal bytes in many lanes of a wave: English-like text (a 28-symbol alphabet
    # with spaces and frequent letters repeated) and one constant byte
    alpha = torch.tensor(list(b"       eeeetttaaoinshrdlu.,\n"), dtype=torch.uint8, device="cuda")
    big = alpha[(big.to(torch.int32) * len(alpha)) >> 8]
    ms = timed(lambda: lz.histogram(ctx, big))
    res["histogram_1GiB_text"] = dict(ms=ms, GBps=big.numel() / ms / 1e6)
    big.fill_(32)
    ms = timed(lambda: lz.histogram(ctx, big))
    res["histogram_1GiB_constant"] = dict(ms=ms, GBps=big.numel() / ms / 1e6)
    del big
    h = lz.histogram(ctx, x)
    res["entropy_bits"] = lz.entropy(ctx, h)
    n16, L = 16 * MiB, 256
    ms = timed(lambda: lz.autocorrelation(ctx, x[:n16], L))
    res["autocorrelation_16MiB_lag256"] = dict(ms=ms, int_MAC_per_s=n16 * (L + 1) / ms * 1e3)
    # lags up to 256: 32-byte rows, nine tiles of 32 x 32 x 32 int8 products, one launch
    ms = timed(lambda: lz.lag_sums(ctx, x[:n16], L))
    res["lag_sums_16MiB_lag256"] = dict(ms=ms, int_MAC_per_s=n16 * (L + 1) / ms * 1e3,
                                        hbm_GBps=n16 / ms / 1e6)
    L = 16384  # the largest lag count: five windows of at most 4096 lags on the int8 matrix cores
    ms = timed(lambda: lz.lag_sums(ctx, x[:n16], L))
    res["lag_sums_16MiB_lag16384"] = dict(ms=ms, int_MAC_per_s=n16 * (L + 1) / ms * 1e3)
    ms = timed(lambda: lz.autocorrelation(ctx, x[:n16], L))
    res["autocorrelation_16MiB_lag16384"] = dict(ms=ms, int_MAC_per_s=n16 * (L + 1) / ms * 1e3)
    # power-of-two sides: two FFT passes; algorithmic bytes: the image (1 B per value) in, the half
    # spectrum (h/2 + 1 of each column's h indices, 16 B complex) out and in again, 8 B |Z|^2 out
    def spectrum_bytes(h, w):
        return h * w + 2 * 16 * w * (h // 2 + 1) + 8 * h * w

    N = 1024
    ms = timed(lambda: lz.power_spectrum_2d(ctx, img))
    res["power_spectrum_1024x1024"] = dict(ms=ms, route="fft", hbm_GBps=spectrum_bytes(N, N) / ms / 1e6)
    ms = timed(lambda: lz.autocorrelation_2d(ctx, img))
    res["autocorrelation_2d_1024x1024"] = dict(ms=ms, route="fft")
    a = lz.autocorrelation_2d(ctx, img)
    res["max_abs_offzero_acf2"] = float(a.flatten()[1:].abs().max())
    # sides with no prime factor above 5: mixed-radix FFT passes (1000 = 2^3 5^3)
    N = 1000
    img_m = x[:N * N].view(N, N)
    ms = timed(lambda: lz.power_spectrum_2d(ctx, img_m))
    res["power_spectrum_1000x1000"] = dict(ms=ms, route="mixed-radix fft",
                                           hbm_GBps=spectrum_bytes(N, N) / ms / 1e6)
    # other sides (1009 is prime): the direct DFT, dense matrix products on the binary64 matrix cores:
    # the first pass real data times complex twiddles (2 FMA = 4 flops per term) for h/2 + 1 outputs
    # of each column, the second complex times complex (8 flops per term) for those h/2 + 1 columns
    N = 1009
    img_d = x[:N * N].view(N, N)
    hh = N // 2 + 1
    flops = 4 * N * hh * N + 8 * N * N * hh
    ms = timed(lambda: lz.power_spectrum_2d(ctx, img_d))
    res["power_spectrum_1009x1009"] = dict(ms=ms, route="direct", TFLOPs=flops / ms / 1e9,
                                           frac_of_fp64_matrix_peak=flops / ms * 1e3 / FP64_FMA_COUNTED_PEAK)
    ctx.close()
    return res


# ---------------------------------------------------------------------------------------------
def bench_batch(lz, torch, steps, plain_sample=256):
    from paper_1201_3114_amd import workloads

    wl = workloads.batch()
    sizes = wl.sizes
    total = int(sizes.sum())
    ctx = lz.Context(0)
    tuned, tune = None, dict(source="none")
    try:
        t = time.perf_counter()
        tuned, hit = ctx.autotune_cached(budget_ms=8000)
        tune = dict(source="cache" if hit else "tuned", seconds=time.perf_counter() - t, shape=vars(tuned))
        log(f"autotune: {tuned} ({tune['source']}) in {tune['seconds']:.1f} s")
    except lz.LorenzError as e:
        log("autotune failed:", e)
    in_off = wl.offsets.astype(np.uint64)
    out_off, out_tot = lz.packed_offsets(sizes, 24)
    d_in = torch.from_numpy(wl.data).cuda()
    d_out = torch.empty(out_tot, dtype=torch.uint8, device="cuda")
    d_back = torch.empty(total, dtype=torch.uint8, device="cuda")
    st = torch.empty(len(sizes), dtype=torch.int32, device="cuda")
    t = time.perf_counter()
    be = lz.Batch(ctx, False, sizes, wl.passwords, d_in, in_off, d_out, out_off)
    setup_s = time.perf_counter() - t
    be.launch()
    torch.cuda.synchronize()
    bd = lz.Batch(ctx, True, sizes, wl.passwords, d_out, out_off, d_back, in_off, d_status=st)
    stream = torch.cuda.current_stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    enc, dec = [], []
    for _ in range(steps):
        e[0].record(stream)
        be.launch()
        e[1].record(stream)
        bd.launch()
        e[2].record(stream)
        torch.cuda.synchronize()
        enc.append(e[0].elapsed_time(e[1]))
        dec.append(e[1].elapsed_time(e[2]))
    ok = bool(torch.equal(d_back, d_in)) and bool((st == 0).all())
    # plain path, one call per message, on a prefix of the batch
    k = min(plain_sample, len(sizes))
    pb = int(sizes[:k].sum())
    outs = [torch.empty(int(s) + 24, dtype=torch.uint8, device="cuda") for s in sizes[:k]]
    views = [d_in[int(in_off[i]):int(in_off[i]) + int(sizes[i])] for i in range(k)]
    torch.cuda.synchronize()
    e[0].record(stream)
    for i in range(k):
        ctx.encrypt(views[i], wl.passwords[i], out=outs[i])
    e[1].record(stream)
    torch.cuda.synchronize()
    plain_ms = e[0].elapsed_time(e[1])
    same = all(torch.equal(outs[i], d_out[int(out_off[i]):int(out_off[i]) + int(sizes[i]) + 24]) for i in range(k))
    # integrity: 10% of the ciphertexts get one altered byte
    idx, offs, vals = workloads.tamper_plan(sizes + 24)
    pos = torch.from_numpy((out_off[idx] + offs.astype(np.uint64)).astype(np.int64)).cuda()
    d_out[pos] ^= torch.from_numpy(vals).cuda()
    torch.cuda.synchronize()
    e[0].record(stream)
    bd.launch()
    e[1].record(stream)
    torch.cuda.synchronize()
    integ_ms = e[0].elapsed_time(e[1])
    status = st.cpu().numpy()
    bad = np.zeros(len(sizes), bool)
    bad[idx] = True
    flagged_ok = bool((status[bad] == -2).all() and (status[~bad] == 0).all())
    back = d_back.cpu().numpy()
    good_exact = True
    for i in np.nonzero(~bad)[0]:
        s0, s1 = int(in_off[i]), int(in_off[i]) + int(sizes[i])
        if not np.array_equal(back[s0:s1], wl.data[s0:s1]):
            good_exact = False
            break
    zeroed = all(not back[int(in_off[i]):int(in_off[i]) + int(sizes[i])].any() for i in idx)
    shape = ctx.get_launch()
    be.close()
    bd.close()
    ctx.close()
    enc_ms, dec_ms = float(np.median(enc)), float(np.median(dec))
    return dict(
        messages=len(sizes), bytes=total, launch=dict(chains_per_lane=shape.chains_per_lane, wg_size=shape.wg_size,
                                                      tile=shape.tile, waves_per_simd=shape.waves_per_simd),
        autotune=tune, encrypt_GBps=total / enc_ms / 1e6, decrypt_GBps=total / dec_ms / 1e6,
        enc_dec_GBps=2 * total / (enc_ms + dec_ms) / 1e6, enc_ms=enc_ms, dec_ms=dec_ms, setup_s=setup_s,
        roundtrip_exact=ok,
        plain_per_message=dict(messages=k, bytes=pb, encrypt_GBps=pb / plain_ms / 1e6, ms=plain_ms,
                               same_bytes_as_batched=same),
        speedup_vs_plain_per_message=(total / enc_ms) / (pb / plain_ms),
        integrity=dict(altered=int(len(idx)), flagged_exactly=flagged_ok, untouched_exact=good_exact,
                       altered_zeroed=zeroed, decrypt_ms=integ_ms))


# ---------------------------------------------------------------------------------------------
def bench_serve(lz, torch, count, plain_prefix, budget, tick_bytes=16, run_waves=0, curve_requests=40_000):
    """Continuous batching on the fixed-QPS trace: the headline run at 0.7 of capacity, the
    latency curve at every fixed load, the same runs with every admitted chain in each tick
    (the all-chains policy), saturation, and the plain path one request at a time."""
    from paper_1201_3114_amd import workloads

    q_ref = workloads.SERVE_QPS[0.7]
    tr = workloads.serve_trace(count=count, qps=q_ref)
    sizes = tr.sizes
    dec = tr.decrypt.astype(bool)
    tot = int(sizes.sum())
    ctx = lz.Context(0)
    # request plaintexts on the device (torch's generator, seeded), packed 256-byte aligned
    g = torch.Generator(device="cuda")
    g.manual_seed(workloads.SEED["serve"])
    p_off, p_tot = lz.packed_offsets(sizes, 0, 256)
    dP = torch.randint(0, 256, (p_tot,), dtype=torch.uint8, device="cuda", generator=g)
    # ciphertexts of every request made by the batched path (bit-identical to the plain path):
    # the inputs of the decrypt requests and the expected outputs of the encrypt requests
    c_off, c_tot = lz.packed_offsets(sizes, 24, 256)
    dC = torch.zeros(c_tot, dtype=torch.uint8, device="cuda")
    t = time.perf_counter()
    b = lz.Batch(ctx, False, sizes, tr.passwords, dP, p_off, dC, c_off)
    b.launch()
    torch.cuda.synchronize()
    b.close()
    prep_s = time.perf_counter() - t
    dOut = torch.zeros(c_tot, dtype=torch.uint8, device="cuda")  # every output at its request's c_off
    src_all = np.where(dec, dC.data_ptr() + c_off, dP.data_ptr() + p_off).astype(np.uint64)
    dst_all = (dOut.data_ptr() + c_off).astype(np.uint64)

    def run_server(ids, load=0.7, all_at_once=False, policy="adaptive"):
        srv = lz.Server(ctx, hbm_budget=budget, tick_bytes=tick_bytes, run_waves=run_waves, policy=policy)
        lead_ns = int(1.0e9) + 10_000 * len(ids)
        base = lz.now_ns() + lead_ns
        # the trace's arrivals are drawn at the 0.7 rate; another fixed load rescales them
        scale = q_ref / workloads.SERVE_QPS[load]
        arr_s = (tr.arrival_s[ids] - tr.arrival_s[ids[0]]) * scale
        arr = (base + np.round(arr_s * 1e9)).astype(np.uint64)
        if all_at_once:
            arr[:] = base
        t_sub = time.perf_counter()
        srv.submit_many(ids, dec[ids], [tr.passwords[i] for i in ids], src_all[ids], sizes[ids], dst_all[ids], arr)
        submit_s = time.perf_counter() - t_sub
        submitted_in_time = lz.now_ns() < base
        lat, status = [], []
        first_arr, last_done = None, 0
        while len(lat) < len(ids):
            for (rid, stc, a, adm, dn) in srv.poll(8192, 200):
                lat.append((dn - a) / 1e6)
                status.append(stc)
                first_arr = a if first_arr is None else min(first_arr, a)
                last_done = max(last_done, dn)
        stats = srv.stats()
        srv.close()
        span = (last_done - first_arr) / 1e9
        nbytes = int(sizes[ids].sum())
        r = dict(requests=len(ids), bytes=nbytes, GBps=nbytes / span / GB, makespan_s=span,
                 p50_ms=percentile(lat, 50), p99_ms=percentile(lat, 99), max_ms=float(np.max(lat)),
                 all_ok=all(s == 0 for s in status), ticks=stats["ticks"], device_busy_ms=stats["busy_ms"],
                 device_busy_frac=stats["busy_ms"] / 1e3 / span, peak_hbm_GB=stats["peak_hbm"] / GB,
                 tick_bytes=tick_bytes, policy=policy, submit_s=submit_s,
                 submitted_before_first_arrival=submitted_in_time)
        if not all_at_once:
            r.update(load=load, qps=workloads.SERVE_QPS[load], offered_GBps=nbytes / float(arr_s[-1]) / GB)
        return r

    # expected bytes of every response: the batched ciphertexts for encrypt requests and the
    # original plaintexts (then 24 untouched zero bytes) for decrypt requests
    E = dC.clone()
    for i in np.nonzero(dec)[0]:
        o, po, n = int(c_off[i]), int(p_off[i]), int(sizes[i])
        E[o:o + n] = dP[po:po + n]
        E[o + n:o + n + 24] = 0

    def exact(ids):
        torch.cuda.synchronize()
        last = int(c_off[ids[-1]]) + int(sizes[ids[-1]]) + 24
        ok = bool(torch.equal(E[:last], dOut[:last]))
        dOut.zero_()
        return ok

    ids = np.arange(count)
    log(f"serve: {count} requests, {tot / GB:.2f} GB, qps {q_ref:.0f} (0.7 of capacity)")
    served = run_server(ids)
    served["bit_exact_vs_plain"] = exact(ids)
    # latency against offered load, on the first curve_requests requests of the trace
    cids = ids[:min(count, curve_requests)]
    curve, curve_all = [], []
    for load in sorted(workloads.SERVE_QPS):
        log(f"serve: load {load}, {len(cids)} requests")
        curve.append(run_server(cids, load=load))
        curve[-1]["bit_exact_vs_plain"] = exact(cids)
        curve_all.append(run_server(cids, load=load, policy="all_chains"))
        curve_all[-1]["bit_exact_vs_plain"] = exact(cids)
    # saturation: the first quarter of the requests all offered at once (the engine's peak rate)
    sat_ids = ids[:max(1, count // 4)]
    log(f"serve: saturated, {len(sat_ids)} requests")
    saturated = run_server(sat_ids, all_at_once=True)
    saturated["bit_exact_vs_plain"] = exact(sat_ids)
    saturated_all = run_server(sat_ids, all_at_once=True, policy="all_chains")
    saturated_all["bit_exact_vs_plain"] = exact(sat_ids)
    del E
    # plain path, one request at a time in arrival order, on a prefix of the trace
    k = min(plain_prefix, count)
    pre = np.arange(k)
    lat = []
    stream = torch.cuda.current_stream()
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    outs_ok = True
    t_start = lz.now_ns()
    a0 = tr.arrival_s[0]
    for i in pre:
        arr = t_start + int((tr.arrival_s[i] - a0) * 1e9)
        while lz.now_ns() < arr:
            pass
        n = int(sizes[i])
        o = int(c_off[i])
        if dec[i]:
            out = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
            ctx.decrypt(dC[o:o + n + 24], tr.passwords[i], out=out[:n] if n else None, status=st, stream=stream)
        else:
            out = torch.empty(n + 24, dtype=torch.uint8, device="cuda")
            ctx.encrypt(dP[int(p_off[i]):int(p_off[i]) + n], tr.passwords[i], out=out, stream=stream)
        stream.synchronize()
        lat.append((lz.now_ns() - arr) / 1e6)
        if dec[i]:
            outs_ok &= bool(torch.equal(out[:n], dP[int(p_off[i]):int(p_off[i]) + n]))
        else:
            outs_ok &= bool(torch.equal(out, dC[o:o + n + 24]))
    span = (lz.now_ns() - t_start) / 1e9
    pbytes = int(sizes[pre].sum())
    plain = dict(requests=k, bytes=pbytes, GBps=pbytes / span / GB, p50_ms=percentile(lat, 50),
                 p99_ms=percentile(lat, 99), bit_exact=outs_ok)
    served_prefix = run_server(pre)
    ctx.close()
    keep = ("load", "qps", "requests", "GBps", "offered_GBps", "p50_ms", "p99_ms", "max_ms", "ticks",
            "device_busy_frac", "all_ok", "bit_exact_vs_plain")
    return dict(config=dict(qps=workloads.SERVE_QPS, capacity_GBps=workloads.SERVE_CAPACITY_GBPS,
                            mean_request_bytes=tot / count, hbm_budget_GB=budget / GB, tick_bytes=tick_bytes,
                            run_waves=run_waves or 4),
                requests=count, bytes=tot, prep_s=prep_s, continuous=served,
                latency_curve=[{k_: c[k_] for k_ in keep} for c in curve],
                latency_curve_all_chains=[{k_: c[k_] for k_ in keep} for c in curve_all],
                saturated=saturated, saturated_all_chains=saturated_all,
                plain_per_request_prefix=plain, continuous_same_prefix=served_prefix,
                p99_speedup_vs_plain_on_prefix=plain["p99_ms"] / served_prefix["p99_ms"])


# ---------------------------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--only", choices=["all", "plain", "batch", "serve", "variants", "stream", "diag", "copycal"], default="all")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200_000)
    ap.add_argument("--serve-run-waves", type=int, default=0, help="most waves per SIMD of a serving tick (0 = 4)")
    ap.add_argument("--serve-curve-requests", type=int, default=40_000)
    ap.add_argument("--serve-plain-prefix", type=int, default=200)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-tick-bytes", type=int, default=16)
    ap.add_argument("--batch-steps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; every block is independent, so more GPUs "
                                   "would shard the blocks, with a 24-byte tag XOR as the only collective; "
                                   "--gpus must be 1"}))
        sys.exit(2)

    import torch

    import paper_1201_3114_amd as lz

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)

    if args.only == "copycal":
        # a plain device copy of known size: the scale for the HBM byte counters of the profiler
        nbytes = 512 * MiB
        src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 3}))
        return

    out = {"metric": "encrypt+decrypt GB/s at 64 MiB; batched/served GB/s + p50/p99 vs plain", "unit": "GB/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded uniform random bytes, printable passwords)",
           "paper_context": {"parallel_version_MBps": {"GeForce 8800 GT": 2.5, "GTX 285": 4.3},
                             "note": "the paper's own figures (Section 5), another computation on other hardware: "
                                     "context only, not a baseline for this metric"}}
    plain = None
    if args.only in ("all", "plain", "serve"):
        log("plain 64 MiB ...")
        plain = bench_plain(lz, torch, args.steps, args.warmup)
        t_enc, t_dec = sum(plain["enc_ms"]), sum(plain["dec_ms"])
        n = plain["n"]
        ms_step = (t_enc + t_dec) / args.steps
        value = 2 * n * args.steps / ((t_enc + t_dec) / 1e3) / GB
        launches = 2 * args.steps
        avg_launch_s = (t_enc + t_dec) / launches / 1e3
        ops = n * fp64_ops_per_byte(plain["n_it"])
        achieved = ops / avg_launch_s
        sh = plain["shape"]
        out.update(value=value, ms_per_step=ms_step,
                   config={"workload": "plain 64 MiB: one 67108864-byte message, 32-byte password, block 256, "
                                       "n_it 3000, dt 0.01, encrypt then decrypt",
                           "message_bytes": n, "password_bytes": 32, "block_len": 256, "n_it": plain["n_it"],
                           "launch": {"chains_per_lane": sh.chains_per_lane, "wg_size": sh.wg_size,
                                      "tile": sh.tile}},
                   encrypt_GBps=n / (t_enc / args.steps / 1e3) / GB, decrypt_GBps=n / (t_dec / args.steps / 1e3) / GB,
                   wall_s=plain["wall_s"], roundtrip_exact=plain["roundtrip_ok"],
                   host_buffers_GBps=2 * n / (plain["pcie_ms"] / 1e3) / GB,
                   latency_64KiB_ms={"encrypt": plain["lat64"][0], "decrypt": plain["lat64"][1]},
                   roofline={"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VALU_OPS_PEAK / 1e12,
                             "unit": "TFLOP/s", "frac": achieved / FP64_VALU_OPS_PEAK, "traffic": profiled_traffic(vars(sh)),
                             "traffic_unit": "bytes per launch (copy-calibrated FETCH_SIZE + WRITE_SIZE)",
                             "algorithmic_bytes_per_launch": 2 * n + 24,
                             "kernel": "plain_kernel (binary64 VALU, one op per lane per clock)",
                             "ops_per_launch": ops, "avg_launch_ms": avg_launch_s * 1e3,
                             "frac_of_fma_counted_78.6": achieved / FP64_FMA_COUNTED_PEAK,
                             "hbm_GBps": 2 * n / avg_launch_s / GB})
    if args.only in ("all", "plain") and not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = bench_cpu_baseline()
    if args.only in ("all", "batch"):
        log("batched ...")
        out["batched"] = bench_batch(lz, torch, args.batch_steps)
    if args.only in ("all", "variants"):
        log("integrator formats and sequential version ...")
        out["integrator_formats"] = bench_variants(lz, torch)
        out["sequential_version"] = bench_sequential(lz, torch)
    if args.only in ("all", "stream"):
        log("streaming ...")
        out["streaming"] = bench_streaming(lz, torch)
    if args.only in ("all", "diag"):
        log("diagnostics ...")
        out["diagnostics"] = bench_diag(lz, torch)
    if args.only in ("all", "serve"):
        log("served ...")
        sv = bench_serve(lz, torch, args.serve_requests, args.serve_plain_prefix, int(args.serve_budget_gb * GB),
                         args.serve_tick_bytes, args.serve_run_waves, args.serve_curve_requests)
        if "batched" in out:
            sv["saturated_frac_of_batched"] = sv["saturated"]["GBps"] / out["batched"]["enc_dec_GBps"]
        out["served"] = sv
    print(json.dumps(out))


if __name__ == "__main__":
    main()
