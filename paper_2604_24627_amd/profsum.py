"""Summaries of rocprofv3 output for this library's kernels.

kernel_stats(csv)        -> {kernel: (calls, avg_ns)}   from --kernel-trace --stats
counters(csv)            -> {kernel: [value per dispatch]} from --pmc <counter>
Kernel names are reduced to the bare function name (k_...).
"""
from __future__ import annotations

import csv
import re
import statistics
import sys


def short(name: str) -> str:
    m = re.search(r"(k_[a-z0-9_]+)", name)
    if m:
        return m.group(1)
    return name.split("(")[0][-60:]


def kernel_stats(path):
    out = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            k = short(row["Name"])
            calls, avg = int(row["Calls"]), float(row["AverageNs"])
            if k in out:
                c0, a0 = out[k]
                out[k] = (c0 + calls, (a0 * c0 + avg * calls) / (c0 + calls))
            else:
                out[k] = (calls, avg)
    return out


def counters(path, counter):
    out = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            out.setdefault(short(row["Kernel_Name"]), []).append(float(row["Counter_Value"]))
    return out


def main(argv):
    stats = kernel_stats(argv[1])
    fetch = counters(argv[2], "FETCH_SIZE") if len(argv) > 2 else {}
    write = counters(argv[3], "WRITE_SIZE") if len(argv) > 3 else {}
    copy_bytes = float(argv[4]) if len(argv) > 4 else None
    scale_f = scale_w = 1.0
    if copy_bytes and "k_stream_copy" in fetch:
        scale_f = copy_bytes / (statistics.median(fetch["k_stream_copy"]) * 1024.0)
        scale_w = copy_bytes / (statistics.median(write["k_stream_copy"]) * 1024.0)
    print(f"{'kernel':24s} {'calls':>6s} {'avg_us':>10s} {'fetch_MB':>10s} {'write_MB':>10s}")
    for k, (c, a) in sorted(stats.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        fm = statistics.median(fetch[k]) * 1024 * scale_f / 1e6 if k in fetch else float("nan")
        wm = statistics.median(write[k]) * 1024 * scale_w / 1e6 if k in write else float("nan")
        print(f"{k:24s} {c:6d} {a / 1e3:10.2f} {fm:10.2f} {wm:10.2f}")
    print(f"counter scale (copy-calibrated): fetch x{scale_f:.4f} write x{scale_w:.4f}")


if __name__ == "__main__":
    main(sys.argv)
