"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_1811_01490_amd.profiling --trace DIR [--fetch DIR --write DIR]
        --label NAME --command "..." --out profiles/

reads the CSV files rocprofv3 writes with ``--output-format csv``
(``*_kernel_stats.csv`` from ``--kernel-trace --stats``, and
``*_counter_collection.csv`` from ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``,
and from ``--pmc SQ_...`` runs given with ``--sq``) and writes
``profiles/<label>.txt`` (durations, bytes and instruction counts per
kernel) and, when counters are given, updates ``profiles/pmc_traffic.json``
(bytes per launch per kernel, keyed like bench.py's roofline kernel) and
``profiles/pmc_counters.json`` (instructions per wavefront, VALU busy), per
workload label, with the hash of the kernel sources they were taken on.

Counter scaling: FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; each is
scaled by the ratio known bytes / counter value of the calibration copy
(``__amd_rocclr_copyBuffer`` of the largest grid, a 64 MiB device copy that
bench.py runs before its timed region).
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_1811_01490_amd/csrc/gfp_kernels.hpp", "paper_1811_01490_amd/csrc/gfp_device.hpp",
                  "paper_1811_01490_amd/csrc/gfp_copy.hip"]
CALIB_BYTES = 64 * 2 ** 20


def source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_key(name: str) -> str:
    """'void gfpk::k_pass<8, 63, 34, false, 0, true, false, false, false>(...)' ->
    'k_pass<8,63,34,fwd,last>' (',unif' for the uniform-twiddle variant,
    'inv', 'scale' and 'product' for the inverse, ',bnd' for a product's
    bounded first forward launch); the fused pairs likewise as 'k_pass2<...>'
    and 'k_pass2u<...>' (the wide variant)."""
    def tail(mode, bnd):
        t = ",scale" if mode == "1" else (",product" if mode == "2" else "")
        return t + (",bnd" if bnd == "true" else "")

    m = re.search(r"(k_pass2u?)<(\d+), (\d+), (\d+), (true|false), (\d), (true|false), (true|false)"
                  r"(?:, (true|false))?>", name)
    if m:
        kern, k, w, u, inv, mode, last, t2, bnd = m.groups()
        key = "%s<%s,%s,%s,%s,%s" % (kern, k, w, u, "inv" if inv == "true" else "fwd", "last" if last == "true" else "mid")
        return key + tail(mode, bnd) + ">"
    m = re.search(r"k_pass<(\d+), (\d+), (\d+), (true|false), (\d), (true|false), (true|false), (true|false)"
                  r"(?:, (true|false))?>", name)
    if m:
        k, w, u, inv, mode, last, unif, t2, bnd = m.groups()
        key = "k_pass<%s,%s,%s,%s,%s" % (k, w, u, "inv" if inv == "true" else "fwd", "last" if last == "true" else "mid")
        if unif == "true":
            key += ",unif"
        return key + tail(mode, bnd) + ">"
    m = re.search(r"(k_\w+)<([^>]*)>", name)
    if m:
        return "%s<%s>" % (m.group(1), m.group(2).replace(" ", ""))
    return name.split("(")[0].replace("void ", "")


def _one(dirname: str, pattern: str) -> str:
    files = glob.glob(os.path.join(dirname, "**", pattern), recursive=True)
    if not files:
        raise FileNotFoundError("%s not found under %s" % (pattern, dirname))
    return files[0]


def ours(name: str) -> bool:
    """Kernels of this library and the calibration copy (not torch's own
    kernels, such as the fill that initialises the calibration buffer)."""
    return "at::native" not in name


def read_stats(trace_dir: str):
    rows = list(csv.DictReader(open(_one(trace_dir, "*kernel_stats.csv"))))
    out = []
    for r in rows:
        if not ours(r["Name"]):
            continue
        out.append(dict(kernel=kernel_key(r["Name"]), calls=int(r["Calls"]), avg_us=float(r["AverageNs"]) / 1e3,
                        min_us=float(r["MinNs"]) / 1e3, max_us=float(r["MaxNs"]) / 1e3, pct=float(r["Percentage"])))
    return out


def read_counter(pmc_dir: str):
    rows = list(csv.DictReader(open(_one(pmc_dir, "*counter_collection.csv"))))
    calib = max((r for r in rows if "copyBuffer" in r["Kernel_Name"]), key=lambda r: int(r["Grid_Size"]), default=None)
    scale = CALIB_BYTES / (float(calib["Counter_Value"]) * 1024) if calib else 1.0
    per = {}
    for r in rows:
        if "copyBuffer" in r["Kernel_Name"] or not ours(r["Kernel_Name"]):
            continue
        per.setdefault(kernel_key(r["Kernel_Name"]), []).append(float(r["Counter_Value"]) * 1024 * scale)
    return scale, {k: sum(v) / len(v) for k, v in per.items()}, rows[0]["Counter_Name"] if rows else "?"


def read_sq(dirs):
    """Mean value per dispatch of every counter in the counter_collection CSVs
    under the given directories, per kernel: {kernel: {counter: value}}."""
    per = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if "copyBuffer" in r["Kernel_Name"] or not ours(r["Kernel_Name"]):
                    continue
                per.setdefault(kernel_key(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
                    float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in per.items()}


SIMDS = 256 * 4  # MI355X: 256 CUs of 4 SIMDs
CLOCK_HZ = 2.4e9  # peak engine clock
VALU_CYCLES = 4  # a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles


def sq_table(sq, stats):
    """Instruction mix and VALU issue share per kernel: VALU busy = VALU
    instructions x 4 cycles / (1024 SIMDs x 2.4 GHz x mean duration)."""
    dur = {s["kernel"]: s["avg_us"] for s in stats}
    lines = ["", "## Instruction counters per dispatch (rocprofv3 --pmc SQ_*)", "",
             "VALU busy = SQ_INSTS_VALU x %d cycles / (%d SIMDs x %.1f GHz x mean duration from the trace above)."
             % (VALU_CYCLES, SIMDS, CLOCK_HZ / 1e9), "",
             "| kernel | waves | VALU / wave | of which 64-bit | SALU / wave | LDS / wave | VMEM rd / wave | "
             "LDS bank conflicts / wave | VALU busy |", "|---|---|---|---|---|---|---|---|---|"]
    out = {}
    for k in sorted(sq):
        c = sq[k]
        w = c.get("SQ_WAVES", 0.0)
        if not w:
            continue
        valu = c.get("SQ_INSTS_VALU", 0.0)
        busy = valu * VALU_CYCLES / (SIMDS * CLOCK_HZ * dur[k] * 1e-6) if k in dur and dur[k] else None
        row = {"waves": round(w), "valu_per_wave": round(valu / w, 1),
               "valu64_per_wave": round(c.get("SQ_INSTS_VALU_INT64", 0.0) / w, 1),
               "salu_per_wave": round(c.get("SQ_INSTS_SALU", 0.0) / w, 1),
               "lds_per_wave": round(c.get("SQ_INSTS_LDS", 0.0) / w, 1),
               "vmem_rd_per_wave": round(c.get("SQ_INSTS_VMEM_RD", 0.0) / w, 1),
               "lds_bank_conflicts_per_wave": round(c.get("SQ_LDS_BANK_CONFLICT", 0.0) / w, 1),
               "valu_busy": round(busy, 3) if busy is not None else None}
        out[k] = row
        lines.append("| %s | %d | %.0f | %.0f | %.0f | %.0f | %.0f | %.0f | %s |" % (
            k, row["waves"], row["valu_per_wave"], row["valu64_per_wave"], row["salu_per_wave"],
            row["lds_per_wave"], row["vmem_rd_per_wave"], row["lds_bank_conflicts_per_wave"],
            "%.2f" % busy if busy is not None else "-"))
    if any(r["valu_busy"] is not None and r["valu_busy"] > 1.0 for r in out.values()):
        lines += ["", "A busy share above 1 means that launches of this kernel overlapped others (the size "
                  "classes of a batch run on forked streams), so the chip was not its alone for its duration."]
    return lines, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--sq", nargs="*", default=[], help="directories of --pmc SQ_* runs")
    ap.add_argument("--label", required=True)
    ap.add_argument("--command", required=True, help="the rocprofv3 command lines that produced the data")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    stats = read_stats(args.trace)
    lines = ["# %s" % args.label, "", "Commands (run from the repository root on the GPU host):", ""]
    lines += ["    " + c for c in args.command.split(";;")]
    lines += ["", "Kernel source hash: %s" % source_hash(), "",
              "## Kernel durations (rocprofv3 --kernel-trace --stats)", "",
              "| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for s in stats:
        lines.append("| %s | %d | %.2f | %.2f | %.2f | %.1f |" % (s["kernel"], s["calls"], s["avg_us"], s["min_us"],
                                                               s["max_us"], s["pct"]))
    traffic = {}
    if args.fetch and args.write:
        fs, fetch, _ = read_counter(args.fetch)
        ws, write, _ = read_counter(args.write)
        lines += ["", "## HBM traffic per launch (rocprofv3 --pmc FETCH_SIZE, --pmc WRITE_SIZE)", "",
                  "Calibration: a 64 MiB device copy reads FETCH_SIZE x%.4f and WRITE_SIZE x%.4f of its bytes; "
                  "the counters below are scaled by those factors." % (1 / fs, 1 / ws), "",
                  "| kernel | fetch MB | write MB | total MB |", "|---|---|---|---|"]
        for k in sorted(set(fetch) | set(write)):
            f, w = fetch.get(k, 0.0), write.get(k, 0.0)
            traffic[k] = {"fetch_bytes": round(f), "write_bytes": round(w), "bytes_per_launch": round(f + w)}
            lines.append("| %s | %.1f | %.1f | %.1f |" % (k, f / 1e6, w / 1e6, (f + w) / 1e6))
        jpath = os.path.join(args.out, "pmc_traffic.json")
        d = json.load(open(jpath)) if os.path.exists(jpath) else {}
        if d.get("source_hash") != source_hash():
            d = {"source_hash": source_hash(), "workloads": {}}
        d["workloads"][args.label] = {"kernels": traffic, "fetch_scale": round(fs, 6), "write_scale": round(ws, 6)}
        json.dump(d, open(jpath, "w"), indent=1, sort_keys=True)
    if args.sq:
        sq_lines, sq_rows = sq_table(read_sq(args.sq), stats)
        lines += sq_lines
        jpath = os.path.join(args.out, "pmc_counters.json")
        d = json.load(open(jpath)) if os.path.exists(jpath) else {}
        if d.get("source_hash") != source_hash():
            d = {"source_hash": source_hash(), "workloads": {}}
        d["workloads"][args.label] = {"kernels": sq_rows}
        json.dump(d, open(jpath, "w"), indent=1, sort_keys=True)
    with open(os.path.join(args.out, args.label + ".txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
