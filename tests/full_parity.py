"""Full-size parity check, run by hand on a machine with an MI355X (not collected by pytest: about ten
minutes, almost all of it the CPU oracle): every byte and the tag of the 64 MiB plain workload, and every one of the 4,096
messages of the batch workload (638 MB), against the oracle.

    python tests/full_parity.py
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import oracle  # noqa: E402
import paper_1201_3114_amd as lz  # noqa: E402
from paper_1201_3114_amd import workloads  # noqa: E402


def main() -> int:
    threads = min(16, len(os.sched_getaffinity(0)))
    print("oracle threads", threads, flush=True)
    ctx = lz.Context(0)
    P, pw = workloads.plain("plain_64m")
    C = ctx.encrypt(torch.from_numpy(P).cuda(), pw).cpu().numpy()
    t = time.time()
    ok1 = bool(np.array_equal(C, oracle.encrypt(pw, P, nthreads=threads)))
    print(f"64 MiB message: bit-exact {ok1} (oracle {time.time() - t:.0f} s)", flush=True)
    wl = workloads.batch()
    out_off, out_tot = lz.packed_offsets(wl.sizes, 24)
    d_out = torch.zeros(out_tot, dtype=torch.uint8, device="cuda")
    b = lz.Batch(ctx, False, wl.sizes, wl.passwords, torch.from_numpy(wl.data).cuda(), wl.offsets, d_out, out_off)
    b.launch()
    torch.cuda.synchronize()
    b.close()
    G = d_out.cpu().numpy()
    t, bad = time.time(), 0
    for i, n in enumerate(wl.sizes):
        o, n = int(out_off[i]), int(n)
        Pi = wl.data[int(wl.offsets[i]):int(wl.offsets[i]) + n]
        bad += not np.array_equal(G[o:o + n + 24], oracle.encrypt(wl.passwords[i], Pi, nthreads=threads))
        if i % 512 == 511:
            print(f"batch: {i + 1} messages, {bad} mismatches ({time.time() - t:.0f} s)", flush=True)
    print(f"batch of {len(wl.sizes)} messages: {bad} mismatches", flush=True)
    return 0 if ok1 and bad == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
