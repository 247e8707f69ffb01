#!/usr/bin/env python3
"""Benchmark: forward FFT over Z/pZ, p = (2^63 + 2^34)^8 + 1 (k = 8), of
N = 16^5 = 1,048,576 coefficients on one MI355X.

Prints one JSON line.  value = N / (time of one forward transform), inputs
resident in HBM before the timed region.  The timed region is `steps`
back-to-back calls of gfp_fft_forward bracketed by synchronisations, timed
with HIP events on the stream the library launches on.

Extra objects:
  roofline      the dominant kernel (the slowest radix-16 pass), timed alone
                with HIP events; ALU-bound, so achieved = algorithmic integer
                operations per launch / mean launch time against the chip's
                32-bit VALU peak (256 CU x 64 lanes x 2.4 GHz).
  hbm           the whole transform against the HBM roofline: algorithmic
                bytes (read + write the vector once) / transform time.
  cpu_baseline  the CPU oracle (multithreaded C++ radix-2 transform with
                schoolbook multiprecision arithmetic) timed on this host on
                the full workloads, median of 3.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Z/pZ FFT coeffs/s (k=8,N=16^5); batched-vs-plain polymul speedup; p99 latency"
K_DIG, R = 8, 2 ** 63 + 2 ** 34
R16 = 2 ** 62 + 2 ** 36  # the k = 16 prime of the served workload
LOG2N = 20
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # 32-bit integer lane-ops per second (Tops/s)
HBM_PEAK_GBS = 8000.0
PROFILE_LABEL = "fft_forward_k8_n1048576"  # the profiles/ summary of this workload


def pass_counts(N: int, K: int, s: int, k: int):
    """Per-pass algorithmic work of the radix-K schedule at stage s:
    general twiddle products (twiddle not a power of r), butterflies, and
    the integer operations they need at minimum: 4 k^2 32x32-bit limb
    products per general product (schoolbook on k 64-bit digits) and 4 k
    32-bit add/sub-with-carry per radix-2 butterfly (one k-digit addition and
    one subtraction)."""
    import numpy as np

    ns = K ** s
    a = np.arange(ns, dtype=np.int64)
    general = 0
    for t in range(1, K):
        general += int(np.count_nonzero((a * t) % ns))
    general *= (N // K) // ns
    lgk = K.bit_length() - 1
    butterflies = (N // K) * (K // 2) * lgk
    ops = general * 4 * k * k + butterflies * 4 * k
    return general, butterflies, ops


def traffic_from_profiles(kernel_key: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 --pmc
    summary (profiles/pmc_traffic.json), if it was taken on the current
    kernel sources; else None."""
    from paper_1811_01490_amd.profiling import source_hash

    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != source_hash():
        return None
    ent = d.get("workloads", {}).get(PROFILE_LABEL, {}).get("kernels", {}).get(kernel_key)
    return ent.get("bytes_per_launch") if ent else None


def cpu_baseline(reps: int = 3):
    """The CPU oracle timed on this host: the multithreaded C++ radix-2
    transform of oracle/cpu_ntt.cpp (schoolbook multiprecision Montgomery
    arithmetic mod p, std::thread over the host's CPUs, twiddle powers and
    digit conversions included in every call), median of `reps` runs, on the
    full workloads: transform size 4096 product of two degree < 2048 factors
    (k = 8); forward and inverse transforms of 2^20 coefficients and the
    product of two degree < 2^19 factors (k = 8); the same product over the
    k = 16 prime.  Also the Python definitional oracle (schoolbook product,
    one thread) on the degree < 2048 product, for context.  value = the k = 8
    forward transform rate, the headline workload."""
    import statistics

    import gfp_inputs as gi
    from oracle import cpu_ntt
    from oracle import transform as T
    from oracle.field import GFPField

    threads = cpu_ntt.default_threads()
    cpu_ntt.build()

    def med(fn):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts), ts

    out = {}
    F8, F16 = GFPField(K_DIG, R), GFPField(16, R16)
    N = 2 ** LOG2N
    # headline: k = 8 forward and inverse transforms of 2^20 coefficients
    x = gi.uniform_digits(K_DIG, R, N, gi.BASE_SEED + 1, 0)
    w = F8.paper_root_of_unity(N)
    wi = pow(w, F8.p - 2, F8.p)
    t_fwd, ts_fwd = med(lambda: cpu_ntt.transform(K_DIG, R, x, w, threads=threads))
    t_inv, _ = med(lambda: cpu_ntt.transform(K_DIG, R, x, wi, inverse=True, threads=threads))
    out["k8_forward_2^20_s"] = round(t_fwd, 4)
    out["k8_forward_2^20_runs_s"] = [round(v, 4) for v in ts_fwd]
    out["k8_inverse_2^20_s"] = round(t_inv, 4)
    # products of two degree < 2^19 factors (transform size 2^20), k = 8 and 16
    for name, F, seed in (("k8", F8, gi.BASE_SEED + 1), ("k16", F16, gi.BASE_SEED + 2)):
        a = gi.uniform_digits(F.k, F.r, N // 2, seed, 0)
        b = gi.uniform_digits(F.k, F.r, N // 2, seed, 1)
        wf = F.paper_root_of_unity(N)
        wfi = pow(wf, F.p - 2, F.p)
        t, _ = med(lambda: cpu_ntt.polymul(F.k, F.r, a, b, N, wf, wfi, threads=threads))
        out["%s_polymul_2^19x2^19_s" % name] = round(t, 4)
    # transform size 4096 product, k = 8
    a = gi.uniform_digits(K_DIG, R, 2048, gi.BASE_SEED + 0, 0)
    b = gi.uniform_digits(K_DIG, R, 2048, gi.BASE_SEED + 0, 1)
    w12 = F8.paper_root_of_unity(4096)
    t, _ = med(lambda: cpu_ntt.polymul(K_DIG, R, a, b, 4096, w12, pow(w12, F8.p - 2, F8.p), threads=threads))
    out["k8_polymul_2048x2048_s"] = round(t, 5)
    # Python definitional oracle (schoolbook, one thread), same product
    def ints(v):
        obj = v.astype(object)
        acc = obj[K_DIG - 1].copy()
        for d in range(K_DIG - 2, -1, -1):
            acc = acc * R + obj[d]
        return [int(t_) for t_ in acc]
    ai, bi = ints(a), ints(b)
    t0 = time.perf_counter()
    T.polymul(ai, bi, F8.p)
    out["python_schoolbook_2048x2048_s"] = round(time.perf_counter() - t0, 3)
    return {
        "value": round(N / t_fwd, 1),
        "unit": "coeffs/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "C++ oracle (oracle/cpu_ntt.cpp: radix-2 transform, schoolbook Montgomery arithmetic mod p, "
                  "%d threads) on the full workloads, median of %d runs each; value = the k = 8 forward "
                  "transform of 2^20 coefficients (%.3f s)" % (threads, reps, t_fwd),
        "workloads": out,
        "cpu_model": _cpu_model(),
        "host_cpus": os.cpu_count(),
    }


def batched_leg(torch, f, dev, reps: int):
    """Batched workload: 256 products over the k = 8 prime, transform sizes N_i drawn
    uniformly from {16^2, 16^3, 16^4, 16^5} (log-uniform in N), la = lb = N_i / 2,
    uniform coefficients.  The stage grouping of every (size, batch class)
    either path uses is autotuned first (gfp_tune).  Times 256 separate
    gfp_polymul calls against one gfp_polymul_batched call replayed from its
    hipGraph and against the persistent batched launch (one cooperative
    launch over a device work list), on one stream, and checks that all give
    the same 256 products."""
    import numpy as np

    import gfp_inputs as gi
    from paper_1811_01490_amd import to_device

    seed = gi.BASE_SEED + 3
    g = gi.rng(seed, 1000)
    sizes = [16 ** int(e) for e in g.integers(2, 6, size=256)]
    reqs = []
    for i, n in enumerate(sizes):
        a = to_device(gi.uniform_digits(K_DIG, R, n // 2, seed, 2 + 2 * i), dev)
        b = to_device(gi.uniform_digits(K_DIG, R, n // 2, seed, 3 + 2 * i), dev)
        reqs.append((a, b))
    # autotune the stage grouping of every (size, batch class) both paths use:
    # gfp_polymul runs 2 forward and 1 inverse transform per product, the
    # batched path 2C and C per chunk of C requests (element-major)
    from paper_1811_01490_amd.gfp import LAYOUT_ELEMENT_MAJOR

    tuned = {}
    for n in sorted(set(sizes)):
        per = f.polymul_workspace_size(n // 2, n // 2)
        chunk = min(sizes.count(n), max(1, (4 << 30) // per))
        for nvec in sorted({1, 2, chunk, 2 * chunk}):
            plan, us = f.tune(n, nvec=nvec, layout=LAYOUT_ELEMENT_MAJOR)
            tuned["%d/%d" % (n, nvec)] = {"plan": plan, "us": round(us, 1)}
    c_plain = [torch.empty((K_DIG, a.shape[1] + b.shape[1] - 1), dtype=torch.int64, device=dev) for a, b in reqs]
    c_batch = [torch.empty_like(c) for c in c_plain]
    ws1 = torch.empty(f.polymul_workspace_size(2 ** 19, 2 ** 19) // 8, dtype=torch.int64, device=dev)
    descs = f.batch_descs([(a, b, c) for (a, b), c in zip(reqs, c_batch)])
    wsb = torch.empty(f.polymul_batched_workspace_size(descs) // 8 + 1, dtype=torch.int64, device=dev)
    stream = torch.cuda.Stream(device=dev)  # graph capture needs a non-null stream

    def plain():
        for (a, b), c in zip(reqs, c_plain):
            f.polymul(a, b, c=c, workspace=ws1, stream=stream)

    def batched():
        f.polymul_batched(descs, workspace=wsb, graph=True, stream=stream)

    c_pers = [torch.empty_like(c) for c in c_plain]
    descs_p = f.batch_descs([(a, b, c) for (a, b), c in zip(reqs, c_pers)])

    def persistent():
        f.polymul_batched(descs_p, workspace=wsb, persistent=True, stream=stream)

    def timed(fn):
        torch.cuda.synchronize()
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_plain = timed(plain)
    t_batch = timed(batched)
    t_pers = timed(persistent)
    same = all(torch.equal(x, y) for x, y in zip(c_plain, c_batch))
    same_p = all(torch.equal(x, y) for x, y in zip(c_plain, c_pers))
    coefs = sum(a.shape[1] + b.shape[1] - 1 for a, b in reqs)
    hist = {str(n): sizes.count(n) for n in sorted(set(sizes))}
    return {
        "workload": "256 products, p = (2^63+2^34)^8+1, transform sizes log-uniform on {16^2..16^5}, la = lb = N/2, "
                    "seed 1811014903",
        "size_histogram": hist,
        "output_coeffs": coefs,
        "plain_ms": round(t_plain, 3),
        "batched_graph_ms": round(t_batch, 3),
        "speedup": round(t_plain / t_batch, 3),
        "batched_coeffs_per_s": round(coefs / (t_batch * 1e-3), 1),
        "plain_coeffs_per_s": round(coefs / (t_plain * 1e-3), 1),
        "identical_outputs": bool(same),
        "persistent_ms": round(t_pers, 3),
        "persistent_identical_outputs": bool(same_p),
        "tuned_plans": tuned,
    }


def served_leg(torch, dev, n_req: int, loads, workspace_gib: int, slots: int, express_log2n: int):
    """Served workload: a stream of n_req product requests, each over the k = 8 or the
    k = 16 prime (fair coin), la = lb = floor(2^U), U uniform on [8, 19],
    Poisson arrivals.  The arrival rate is `load` times the saturated request
    rate of the plain path (all requests back to back, one gfp_polymul each,
    one stream).  Each stream is served twice: by the request loop (continuous
    batching over `slots` streams) and by a one-request-per-launch FIFO loop
    (one slot, batches of one), reporting p50/p99 latency (done - scheduled
    arrival) and throughput.  The request loop runs with its batches replayed
    as hipGraphs (the default) and, for comparison, launched eagerly.  Every
    served result is compared with the plain run's result of the same request
    through a 64-bit digest."""
    import numpy as np

    import gfp_inputs as gi
    from paper_1811_01490_amd import Field, Server, to_device

    seed = gi.BASE_SEED + 4
    pool_n = 1 << 21
    fields = {8: Field(K_DIG, R), 16: Field(16, R16)}
    pools = {k: to_device(gi.uniform_digits(k, fields[k].r, pool_n, seed, i), dev) for i, k in enumerate((8, 16))}
    g = gi.rng(seed, 1000)
    ks = np.where(g.integers(0, 2, size=n_req) == 0, 8, 16)
    ls = np.floor(2.0 ** g.uniform(8, 19, size=n_req)).astype(np.int64)
    offs = g.integers(0, pool_n - ls[:, None] + 1, size=(n_req, 2))
    # outputs: one arena per field, request i owns columns [start, start + 2L - 1)
    starts, tot = np.zeros(n_req, dtype=np.int64), {8: 0, 16: 0}
    for i in range(n_req):
        starts[i] = tot[int(ks[i])]
        tot[int(ks[i])] += 2 * int(ls[i]) - 1
    arena = {k: torch.empty((k, max(tot[k], 1)), dtype=torch.int64, device=dev) for k in (8, 16)}
    weights = torch.randint(-2 ** 62, 2 ** 62, (16, 2 ** 20), generator=torch.Generator().manual_seed(seed),
                            dtype=torch.int64).to(dev)

    def views(i):
        k, L = int(ks[i]), int(ls[i])
        a = pools[k][:, int(offs[i, 0]):int(offs[i, 0]) + L]
        b = pools[k][:, int(offs[i, 1]):int(offs[i, 1]) + L]
        c = arena[k][:, int(starts[i]):int(starts[i]) + 2 * L - 1]
        return fields[k], a, b, c

    reqs = [Server.request(*views(i)) for i in range(n_req)]

    def digests():
        out = []
        for i in range(n_req):
            c = views(i)[3]
            out.append((c * weights[:c.shape[0], :c.shape[1]]).sum())
        return torch.stack(out).cpu().numpy()

    # plain path, saturated: every request alone, back to back on one stream
    stream = torch.cuda.Stream(device=dev)
    ws = torch.empty(fields[16].polymul_workspace_size(2 ** 19, 2 ** 19) // 8, dtype=torch.int64, device=dev)
    for i in range(min(n_req, 64)):  # warm-up: twiddle tables of every size, code paths
        f, a, b, c = views(i)
        f.polymul(a, b, c=c, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(n_req):
        f, a, b, c = views(i)
        f.polymul(a, b, c=c, workspace=ws, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_plain = e0.elapsed_time(e1) * 1e-3
    ref = digests()
    del ws
    print("served: plain saturated run %.3f s" % t_plain, file=sys.stderr, flush=True)
    coefs = int((2 * ls - 1).sum())
    mu = n_req / t_plain

    def serve(srv, lam, stream_id):
        gaps = gi.rng(seed, 1001 + stream_id).exponential(1.0 / lam, size=n_req)
        arrive = np.cumsum(gaps) - gaps[0]
        for k in arena:
            arena[k].fill_(-1)
        torch.cuda.synchronize()
        tickets = [0] * n_req
        t0 = time.monotonic_ns() + 2_000_000
        sched = (t0 + arrive * 1e9).astype(np.int64)
        for i in range(n_req):
            while time.monotonic_ns() < sched[i]:
                pass
            tickets[i] = srv.submit_request(reqs[i])
        srv.drain()
        res = [srv.poll(t) for t in tickets]
        st = srv.stats()
        done = np.array([r["t_done_ns"] for r in res], dtype=np.int64)
        sub = np.array([r["t_submit_ns"] for r in res], dtype=np.int64)
        lat = (done - sched) * 1e-6
        lag = (sub - sched) * 1e-6
        ok = all(r["status"] == 0 for r in res)
        same = bool(ok and np.array_equal(digests(), ref))
        span = (done.max() - sched[0]) * 1e-9
        return {
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3),
            "max_submit_lag_ms": round(float(lag.max()), 3),
            "makespan_s": round(float(span), 3),
            "coeffs_per_s": round(coefs / span, 1),
            "requests_per_s": round(n_req / span, 1),
            "batches": st["batches"],
            "max_batch_size": st["max_batch_size"],
            "overlapped_batches": st["overlapped_batches"],
            "graph_launches": st["graph_launches"],
            "graph_captures": st["graph_captures"],
            "identical_to_alone": same,
        }

    runs = {}
    for j, load in enumerate(loads):
        lam = load * mu
        with Server(workspace_bytes=workspace_gib << 30, slots=slots, max_batch=256, max_pending=n_req,
                    express_log2n=express_log2n) as srv:
            cb = serve(srv, lam, j)
        print("served: load %.2f continuous batching, graphs p99 %.3f ms" % (load, cb["p99_ms"]), file=sys.stderr,
              flush=True)
        with Server(workspace_bytes=workspace_gib << 30, slots=slots, max_batch=256, max_pending=n_req,
                    express_log2n=express_log2n, graphs=False) as srv:
            cbe = serve(srv, lam, j)
        print("served: load %.2f continuous batching, eager p99 %.3f ms" % (load, cbe["p99_ms"]), file=sys.stderr,
              flush=True)
        with Server(workspace_bytes=2 << 30, slots=1, max_batch=1, max_pending=n_req, graphs=False) as srv:
            fifo = serve(srv, lam, j)
        print("served: load %.2f plain FIFO p99 %.3f ms" % (load, fifo["p99_ms"]), file=sys.stderr, flush=True)
        runs[str(load)] = {"arrival_rate_per_s": round(lam, 1), "continuous_batching": cb,
                           "continuous_batching_eager": cbe, "plain_fifo": fifo,
                           "p99_speedup": round(fifo["p99_ms"] / cb["p99_ms"], 3)}
    for f in fields.values():
        f.close()
    return {
        "workload": "%d product requests, p = (2^63+2^34)^8+1 or (2^62+2^36)^16+1 by a fair coin, la = lb = "
                    "floor(2^U), U uniform on [8, 19], Poisson arrivals, seed 1811014904" % n_req,
        "output_coeffs": coefs,
        "plain_saturated_s": round(t_plain, 3),
        "plain_saturated_requests_per_s": round(mu, 1),
        "plain_saturated_coeffs_per_s": round(coefs / t_plain, 1),
        "slots": slots,
        "express_log2n": express_log2n,
        "workspace_gib": workspace_gib,
        "loads": runs,
    }


def bigint_leg(torch, dev, words: int, reps: int):
    """Integer product of two random `words`-word integers through the k = 8
    polynomial product (63-bit coefficients), operands and result resident
    in HBM; time per product with HIP events."""
    import numpy as np

    import gfp_inputs as gi
    from paper_1811_01490_amd import Field

    f = Field(K_DIG, R)
    g = gi.rng(gi.BASE_SEED + 5, 0)
    a = torch.from_numpy(g.integers(0, 2 ** 64, size=words, dtype=np.uint64).view(np.int64)).to(dev)
    b = torch.from_numpy(g.integers(0, 2 ** 64, size=words, dtype=np.uint64).view(np.int64)).to(dev)
    c = torch.empty(2 * words, dtype=torch.int64, device=dev)
    ws = torch.empty(f.bigint_mul_workspace_size(words, words) // 8 + 1, dtype=torch.int64, device=dev)
    for _ in range(3):
        f.bigint_mul(a, b, c=c, workspace=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        f.bigint_mul(a, b, c=c, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # the library's coefficient width: the product's coefficients must stay below p
    bits = min(448, (K_DIG * 63 - 2 - (64 * words - 1).bit_length()) // 2)
    la = (64 * words + bits - 1) // bits
    n = f.polymul_size(la, la)
    f.close()
    return {"workload": "product of two uniform random %d-bit integers (seed 1811014905), %d-bit coefficients over "
                        "p = (2^63+2^34)^8+1" % (64 * words, bits),
            "words": words, "coefficient_bits": bits, "transform_size": n, "ms": round(ms, 4),
            "input_bits_per_s": round(2 * 64 * words / (ms * 1e-3), 1)}


# The paper's element multiplication timings (Table multiplication, FFT-based
# and GMP columns, serial CPU, machine unstated, printed in units of 10^-6 s)
# for the Table 1 primes.
PAPER_MUL = {8: (1303.38, 224.03), 16: (2602.56, 471.45), 32: (5500.56, 1282.36), 64: (10656.10, 3032.44)}
ELEMENT_PRIMES = [(8, 2 ** 63 + 2 ** 34, "2^63+2^34"), (16, 2 ** 62 + 2 ** 36, "2^62+2^36"),
                  (32, 2 ** 62 + 2 ** 56, "2^62+2^56"), (64, 2 ** 63 - 2 ** 40, "2^63-2^40")]


def element_leg(torch, dev, n: int, reps: int):
    """Element products z = x y on n uniform random elements of each Table 1
    prime, by the two multipliers (the schoolbook columns the transforms use,
    and the FFT-based product of section 3.3), operands resident in HBM; time
    per launch with HIP events, results compared."""
    import gfp_inputs as gi
    from paper_1811_01490_amd import Field, to_device
    from paper_1811_01490_amd.gfp import OP_MUL, OP_MUL_NTT

    rows = []
    for k, r, label in ELEMENT_PRIMES:
        f = Field(k, r)
        x = to_device(gi.uniform_digits(k, r, n, gi.BASE_SEED + 7, 0), dev)
        y = to_device(gi.uniform_digits(k, r, n, gi.BASE_SEED + 7, 1), dev)
        z = {op: torch.empty_like(x) for op in (OP_MUL, OP_MUL_NTT)}
        row = {"k": k, "r": label, "elements": n}
        for op, name in ((OP_MUL, "schoolbook"), (OP_MUL_NTT, "fft_based")):
            for _ in range(3):
                f.elementwise(op, x, y, z=z[op])
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                f.elementwise(op, x, y, z=z[op])
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / reps * 1e3
            row[name + "_us"] = round(us, 2)
            row[name + "_products_per_s"] = round(n / (us * 1e-6), 1)
        row["identical"] = bool(torch.equal(z[OP_MUL], z[OP_MUL_NTT]))
        row["fft_based_over_schoolbook"] = round(row["fft_based_us"] / row["schoolbook_us"], 2)
        row["paper_fft_based"], row["paper_gmp"] = PAPER_MUL[k]
        rows.append(row)
        f.close()
    return {"workload": "element products over the Table 1 primes, uniform random operands (seed 1811014907)",
            "paper_units": "as printed in the paper's Table multiplication (10^-6 s scale, serial CPU)", "rows": rows}


def twiddle_multiplier_leg(torch, dev, reps: int = 10):
    """The two twiddle multipliers inside the transforms of the k = 32 and
    k = 64 primes of Table 1: every plan of one pass per launch, each pass
    with the schoolbook column product ('1') or the FFT-based product of
    section 3.3 ('n', twiddle transforms tabulated); forward transforms at
    N = 2^20 (k = 64) and 2^17 (k = 32: a radix-2 pass, then two radix-64
    passes with twiddles), outputs compared with the schoolbook plan.  Each
    plan is warmed up for 50 ms before it is timed."""
    import gfp_inputs as gi
    from paper_1811_01490_amd import Field, to_device

    rows = []
    for k, r, label, n in ((64, 2 ** 63 - 2 ** 40, "2^63-2^40", 1 << 20), (32, 2 ** 62 + 2 ** 56, "2^62+2^56", 1 << 17)):
        f = Field(k, r)
        lk = (2 * k).bit_length() - 1
        e = (n.bit_length() - 1) // lk
        x = to_device(gi.uniform_digits(k, r, n, gi.BASE_SEED + 8, 0), dev)
        y = torch.empty_like(x)
        ws = torch.empty(f.fft_workspace_size(n) // 8, dtype=torch.int64, device=dev)
        plans = [""]
        for _ in range(e):
            plans = [p + c for p in plans for c in "1n"]
        ref = None
        for plan in plans:
            f.set_plan(n, plan)
            f.fft_forward(x, y=y, workspace=ws)  # builds the twiddle transforms on the first 'n' plan
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < 0.05:
                f.fft_forward(x, y=y, workspace=ws)
                torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                f.fft_forward(x, y=y, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            same = True
            if ref is None:
                ref = y.clone()
            else:
                same = bool(torch.equal(y, ref))
            rows.append({"k": k, "r": label, "N": n, "plan": plan, "forward_us": round(e0.elapsed_time(e1) / reps * 1e3, 1),
                         "identical_to_schoolbook": same})
        f.close()
    return {"workload": "forward transforms, uniform random coefficients (seed 1811014908), plans '1' (schoolbook "
                        "twiddle product) and 'n' (FFT-based twiddle product) per pass", "rows": rows}


# The paper's FFT timings (Table fftoverprimefield, FFT-based column, serial
# CPU, machine unstated, units inferred as ms) for its test primes (Table
# testprimes).
PAPER_FFT_MS = [(8, 2 ** 59 + 2 ** 16, 256, 0.211), (8, 2 ** 59 + 2 ** 16, 4096, 5.961),
                (16, 2 ** 58 + 2 ** 10, 1024, 1.819), (16, 2 ** 58 + 2 ** 10, 32768, 109.681),
                (32, 2 ** 56 + 2 ** 21, 4096, 15.775), (32, 2 ** 56 + 2 ** 21, 262144, 1995.939)]


def paper_context_leg(torch, dev):
    """Forward transforms on the paper's own FFT workloads (same primes and
    sizes), for context only: the paper's numbers are serial CPU code on
    unstated hardware."""
    import gfp_inputs as gi
    from paper_1811_01490_amd import Field, to_device

    rows = []
    for k, r, n, paper_ms in PAPER_FFT_MS:
        f = Field(k, r)
        x = to_device(gi.uniform_digits(k, r, n, gi.BASE_SEED + 6, 0), dev)
        y = torch.empty_like(x)
        ws = torch.empty(f.fft_workspace_size(n) // 8, dtype=torch.int64, device=dev)
        for _ in range(200):
            f.fft_forward(x, y=y, workspace=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(200):
            f.fft_forward(x, y=y, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / 200 * 1e3
        rows.append({"k": k, "r": "2^%d+2^%d" % (r.bit_length() - 1, (r & -r).bit_length() - 1), "N": n,
                     "gpu_us": round(us, 2), "paper_cpu_ms": paper_ms, "ratio": round(paper_ms * 1e3 / us, 1)})
        f.close()
    return rows


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=300,
                    help="untimed steps first; the first call also builds the twiddle tables on the host, and the "
                         "GPU clock needs tens of ms of work to come back up after that idle time")
    ap.add_argument("--warmup-s", type=float, default=0.5,
                    help="keep warming up until this many seconds of transforms have run")
    ap.add_argument("--pass-reps", type=int, default=50)
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-reps", type=int, default=3)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-bigint", action="store_true")
    ap.add_argument("--no-paper-context", action="store_true")
    ap.add_argument("--no-element", action="store_true")
    ap.add_argument("--element-log2", type=int, default=20)
    ap.add_argument("--bigint-words", type=int, default=2 ** 18)
    ap.add_argument("--served-requests", type=int, default=10000)
    ap.add_argument("--served-loads", default="0.5,0.7,0.9",
                    help="comma-separated fractions of the plain saturated rate")
    ap.add_argument("--served-workspace-gib", type=int, default=16)
    ap.add_argument("--served-slots", type=int, default=3)
    ap.add_argument("--served-express-log2n", type=int, default=16,
                    help="the last slot serves only transform sizes up to 2^this (0: no express slot)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (one transform does not span GPUs). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gfp_inputs as gi
    from paper_1811_01490_amd import Field, to_device

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    N = 2 ** LOG2N
    K = 2 * K_DIG
    f = Field(K_DIG, R)
    x = to_device(gi.uniform_digits(K_DIG, R, N, gi.BASE_SEED + 1, 0), dev)
    y = torch.empty_like(x)
    ws = torch.empty(f.fft_workspace_size(N) // 8, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    # calibration copy of known size (64 MiB read + 64 MiB written), outside the
    # timed region: rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of this kernel
    # scales the counters of the FFT kernels to bytes
    y.copy_(x)
    torch.cuda.synchronize()
    # warm-up: the requested steps, then more until the GPU has been busy for
    # at least --warmup-s seconds (the first call builds the twiddle tables,
    # the GPU mostly idle meanwhile, and the clock needs tens of ms of work to
    # come back up), so that a short --warmup still times the steady state
    f.fft_forward(x, y=y, workspace=ws)
    torch.cuda.synchronize()
    warm_steps, tw0 = 1, time.perf_counter()
    while warm_steps < args.warmup or time.perf_counter() - tw0 < args.warmup_s:
        for _ in range(20):
            f.fft_forward(x, y=y, workspace=ws)
        warm_steps += 20
        torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        f.fft_forward(x, y=y, workspace=ws)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall0
    ms = ev0.elapsed_time(ev1) / args.steps

    # dominant kernel: each launch of the transform's plan alone, on the same
    # stream, in the layouts the transform uses (digit-major in, element-major
    # between launches, digit-major out)
    e = LOG2N // (K.bit_length() - 1)
    plan = f.plan(N)
    em = [ws[: K_DIG * N], ws[K_DIG * N:]]
    launches, s0 = [], 0
    for c in plan:
        launches.append((s0, c))
        s0 += 1 if c == "1" else 2
    per_launch = []
    for i, (s0, c) in enumerate(launches):
        src = x if i == 0 else em[i % 2]
        dst = y if i == len(launches) - 1 else em[(i + 1) % 2]
        kw = dict(in_element_major=i > 0, out_element_major=i < len(launches) - 1, code=c)
        f.fft_pass(s0, src, dst, N, **kw)  # warm
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.pass_reps):
            f.fft_pass(s0, src, dst, N, **kw)
        b.record(stream)
        torch.cuda.synchronize()
        per_launch.append(a.elapsed_time(b) / args.pass_reps)
    dom = int(np.argmax(per_launch))
    s_dom, c_dom = launches[dom]
    gen = bfl = ops = 0
    for s in range(s_dom, s_dom + (1 if c_dom == "1" else 2)):
        g_, b_, o_ = pass_counts(N, K, s, K_DIG)
        gen, bfl, ops = gen + g_, bfl + b_, ops + o_
    dom_us = per_launch[dom] * 1e3
    achieved = ops / (dom_us * 1e-6) / 1e12
    last = dom == len(launches) - 1
    tail = ",last>" if last else ",mid>"
    if c_dom == "w":
        key = "k_pass2u<8,63,34,fwd" + tail
    elif c_dom == "2":
        key = "k_pass2<8,63,34,fwd" + tail
    else:  # one pass: uniform twiddles on the middle stages, see gfp_kernels.hpp
        key = "k_pass<8,63,34,fwd,last>" if last else ("k_pass<8,63,34,fwd,mid,unif>" if s_dom > 0
                                                       else "k_pass<8,63,34,fwd,mid>")
    traffic = traffic_from_profiles(key)
    alg_bytes = 2 * N * K_DIG * 8
    out = {
        "metric": METRIC,
        "value": round(N / (ms * 1e-3), 1),
        "unit": "coeffs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_steps_run": warm_steps,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "forward FFT over Z/pZ, p = (2^63+2^34)^8+1 (k=8, radix-16 base case), N = 16^5 = 1048576, "
                        "uniform random coefficients (seed 1811014901), out-of-place, caller workspace",
            "passes": e,
            "plan": plan,
        },
        "roofline": {
            "bound": "alu",
            "kernel": key,
            "launch": dom,
            "passes_in_launch": [s_dom, s_dom + (0 if c_dom == "1" else 1)],
            "achieved": round(achieved, 3),
            "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "Tops/s",
            "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": traffic,
            "alg_ops_per_launch": ops,
            "general_products_per_launch": gen,
            "butterflies_per_launch": bfl,
            "mean_launch_us": round(dom_us, 2),
            "launch_us": [round(v * 1e3, 2) for v in per_launch],
        },
        "hbm": {
            "alg_bytes_per_transform": alg_bytes,
            "achieved_GBs": round(alg_bytes / (ms * 1e-3) / 1e9, 1),
            "peak_GBs": HBM_PEAK_GBS,
            "frac": round(alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
        "timed_wall_s": round(t_wall, 4),
    }
    if not args.no_batched:
        out["batched"] = batched_leg(torch, f, dev, args.batched_reps)
    if not args.no_served:
        out["served"] = served_leg(torch, dev, args.served_requests, [float(x) for x in args.served_loads.split(",")],
                                   args.served_workspace_gib, args.served_slots, args.served_express_log2n)
    if not args.no_bigint:
        out["bigint"] = bigint_leg(torch, dev, args.bigint_words, 20)
    if not args.no_paper_context:
        out["paper_context"] = paper_context_leg(torch, dev)
    if not args.no_element:
        out["element_products"] = element_leg(torch, dev, 1 << args.element_log2, 20)
        out["twiddle_multipliers"] = twiddle_multiplier_leg(torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_reps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
