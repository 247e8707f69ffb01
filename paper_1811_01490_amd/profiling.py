"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_1811_01490_amd.profiling --trace DIR [--fetch DIR --write DIR]
        --label NAME --command "..." --out profiles/

reads the CSV files rocprofv3 writes with ``--output-format csv``
(``*_kernel_stats.csv`` from ``--kernel-trace --stats``, and
``*_counter_collection.csv`` from ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``)
and writes ``profiles/<label>.txt`` (durations and bytes per kernel) and,
when counters are given, updates ``profiles/pmc_traffic.json`` (bytes per
launch per kernel, keyed like bench.py's roofline kernel, with the hash of
the kernel sources they were taken on).

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
KERNEL_SOURCES = ["paper_1811_01490_amd/csrc/gfp_kernels.hpp", "paper_1811_01490_amd/csrc/gfp_device.hpp"]
CALIB_BYTES = 64 * 2 ** 20


def source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_key(name: str) -> str:
    """'void gfpk::k_pass<8, 63, 34, false, 0, true, false>(...)' ->
    'k_pass<8,63,34,fwd,last>' (',unif' for the uniform-twiddle variant,
    'inv' and 'scale' for the inverse); the fused pairs likewise as
    'k_pass2<...>' and 'k_pass2u<...>' (the wide variant)."""
    m = re.search(r"(k_pass2u?)<(\d+), (\d+), (\d+), (true|false), (\d), (true|false), (true|false)>", name)
    if m:
        kern, k, w, u, inv, mode, last, t2 = m.groups()
        key = "%s<%s,%s,%s,%s,%s" % (kern, k, w, u, "inv" if inv == "true" else "fwd", "last" if last == "true" else "mid")
        if mode == "1":
            key += ",scale"
        return key + ">"
    m = re.search(r"k_pass<(\d+), (\d+), (\d+), (true|false), (\d), (true|false), (true|false), (true|false)>", name)
    if m:
        k, w, u, inv, mode, last, unif, t2 = m.groups()
        key = "k_pass<%s,%s,%s,%s,%s" % (k, w, u, "inv" if inv == "true" else "fwd", "last" if last == "true" else "mid")
        if mode == "1":
            key += ",scale"
        if unif == "true":
            key += ",unif"
        return key + ">"
    m = re.search(r"(k_\w+)<([^>]*)>", name)
    if m:
        return "%s<%s>" % (m.group(1), m.group(2).replace(" ", ""))
    return name.split("(")[0].replace("void ", "")


def _one(dirname: str, pattern: str) -> str:
    files = glob.glob(os.path.join(dirname, "**", pattern), recursive=True)
    if not files:
        raise FileNotFoundError("%s not found under %s" % (pattern, dirname))
    return files[0]


def read_stats(trace_dir: str):
    rows = list(csv.DictReader(open(_one(trace_dir, "*kernel_stats.csv"))))
    out = []
    for r in rows:
        out.append(dict(kernel=kernel_key(r["Name"]), calls=int(r["Calls"]), avg_us=float(r["AverageNs"]) / 1e3,
                        min_us=float(r["MinNs"]) / 1e3, max_us=float(r["MaxNs"]) / 1e3, pct=float(r["Percentage"])))
    return out


def read_counter(pmc_dir: str):
    rows = list(csv.DictReader(open(_one(pmc_dir, "*counter_collection.csv"))))
    calib = max((r for r in rows if "copyBuffer" in r["Kernel_Name"]), key=lambda r: int(r["Grid_Size"]), default=None)
    scale = CALIB_BYTES / (float(calib["Counter_Value"]) * 1024) if calib else 1.0
    per = {}
    for r in rows:
        if "copyBuffer" in r["Kernel_Name"]:
            continue
        per.setdefault(kernel_key(r["Kernel_Name"]), []).append(float(r["Counter_Value"]) * 1024 * scale)
    return scale, {k: sum(v) / len(v) for k, v in per.items()}, rows[0]["Counter_Name"] if rows else "?"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
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
            d = {"source_hash": source_hash(), "kernels": {}}
        d["kernels"].update(traffic)
        d["fetch_scale"] = round(fs, 6)
        d["write_scale"] = round(ws, 6)
        json.dump(d, open(jpath, "w"), indent=1, sort_keys=True)
    with open(os.path.join(args.out, args.label + ".txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
