"""Workload runner for profiling with rocprofv3.

    python -m paper_1811_01490_amd.workloads --workload fft_k8 --reps 20

runs one measured workload `reps` times on device 0, after one 64 MiB device
copy (``__amd_rocclr_copyBuffer``) whose byte counters calibrate FETCH_SIZE and
WRITE_SIZE (see profiling.py), and after a warm-up of about 0.3 s so that the
clock is up.  Inputs are the seeded synthetic inputs of bench.py.

Workloads:
  fft_k8       forward transform over p = (2^63+2^34)^8+1, N = 16^5 = 2^20,
               digit-major, default plan
  fft_k16      forward transform over p = (2^62+2^36)^16+1, N = 32^4 = 2^20
  polymul_k8   product of two degree < 2^19 polynomials over the k = 8 prime
  polymul_k16  the same over the k = 16 prime
  batched      the 256 products of the batched workload (k = 8, transform
               sizes drawn from 16^2..16^5) as one gfp_polymul_batched call
"""

from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

P8 = (8, 2 ** 63 + 2 ** 34)
P16 = (16, 2 ** 62 + 2 ** 36)
WORKLOADS = ("fft_k8", "fft_k16", "polymul_k8", "polymul_k16", "batched")


def build(name: str, torch, dev):
    """A callable that runs the workload once (enqueue only)."""
    import gfp_inputs as gi
    from paper_1811_01490_amd import Field, to_device

    if name in ("fft_k8", "fft_k16"):
        k, r = P8 if name == "fft_k8" else P16
        f = Field(k, r)
        n = 1 << 20
        x = to_device(gi.uniform_digits(k, r, n, gi.BASE_SEED + 1, 0), dev)
        y = torch.empty_like(x)
        ws = torch.empty(f.fft_workspace_size(n) // 8, dtype=torch.int64, device=dev)
        return lambda: f.fft_forward(x, y=y, workspace=ws)
    if name in ("polymul_k8", "polymul_k16"):
        k, r = P8 if name == "polymul_k8" else P16
        f = Field(k, r)
        la = 1 << 19
        a = to_device(gi.uniform_digits(k, r, la, gi.BASE_SEED + 1, 1), dev)
        b = to_device(gi.uniform_digits(k, r, la, gi.BASE_SEED + 1, 2), dev)
        c = torch.empty((k, 2 * la - 1), dtype=torch.int64, device=dev)
        ws = torch.empty(f.polymul_workspace_size(la, la) // 8, dtype=torch.int64, device=dev)
        return lambda: f.polymul(a, b, c=c, workspace=ws)
    if name == "batched":
        k, r = P8
        f = Field(k, r)
        seed = gi.BASE_SEED + 3
        g = gi.rng(seed, 1000)
        sizes = [16 ** int(e) for e in g.integers(2, 6, size=256)]
        reqs = []
        for i, n in enumerate(sizes):
            a = to_device(gi.uniform_digits(k, r, n // 2, seed, 2 + 2 * i), dev)
            b = to_device(gi.uniform_digits(k, r, n // 2, seed, 3 + 2 * i), dev)
            c = torch.empty((k, n - 1), dtype=torch.int64, device=dev)
            reqs.append((a, b, c))
        descs = f.batch_descs(reqs)
        ws = torch.empty(f.polymul_batched_workspace_size(descs) // 8 + 1, dtype=torch.int64, device=dev)
        stream = torch.cuda.Stream(device=dev)
        keep = (f, reqs, descs, ws, stream)

        def run():
            keep[0].polymul_batched(keep[2], workspace=keep[3], graph=True, stream=keep[4])
        return run
    raise ValueError("unknown workload %r" % name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=WORKLOADS, required=True)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--warmup-s", type=float, default=0.3)
    args = ap.parse_args()
    import torch

    if not torch.cuda.is_available():
        raise SystemExit("needs a GPU")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    # calibration copy: 64 MiB read, 64 MiB written
    src = torch.empty(8 << 20, dtype=torch.int64, device=dev).fill_(7)
    dst = torch.empty_like(src)
    dst.copy_(src)
    run = build(args.workload, torch, dev)
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < args.warmup_s:
        run()
        torch.cuda.synchronize()
    for _ in range(args.reps):
        run()
    torch.cuda.synchronize()
    print("workload %s: %d runs done" % (args.workload, args.reps), flush=True)


if __name__ == "__main__":
    main()
