"""Summaries of rocprofv3 output for this library's kernels.

kernel_stats(csv)        -> {kernel: (calls, avg_ns)}   from --kernel-trace --stats
counters(csv)            -> {kernel: [value per dispatch]} from --pmc <counter>
source_digest()          -> SHA-256 of the sources the stepping kernels are
                            compiled from (axpic.hip, its device headers and
                            include/axpic.h),
                            which names the kernels a set of counters was taken
                            from; traffic lines cover only kernels of that unit
read_traffic(path)       -> the per-dispatch HBM bytes recorded in a summary,
                            or None when the kernels have changed since
Kernel names are reduced to the bare function name (k_...).

Usage: python profsum.py <kernel_stats.csv> [<fetch.csv>
<write.csv> <copy_bytes>] -- prints the table;
python profsum.py --trace <kernel_trace.csv> <kernel> <n> -- per-kernel calls and
mean duration from the n-th dispatch of <kernel> on (one leg of a run);
python profsum.py --sq <counter_collection.csv> -- per-kernel
medians over dispatches of SQ_WAVES and of the other SQ counters per wavefront; the FETCH_SIZE / WRITE_SIZE
medians (KiB per dispatch) are scaled so that k_stream_copy of copy_bytes reads
and writes copy_bytes, and a "traffic" line per kernel is printed with the
source digest for read_traffic: the mean of its last LAST_DISPATCHES dispatches,
which in a trace of bench.py's plain leg are the steps in which bench.py times the
dominant kernel alone (the axion kernels' populations grow over the run, so a
median dispatch would not match the launches the roofline divides).
"""
from __future__ import annotations

import csv
import hashlib
import os
import re
import statistics

LAST_DISPATCHES = 3
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_2604_24627_amd", "csrc")

# the stepping kernels' sources, and the ABI header whose structs they compile against
STEP_SOURCES = ("axpic.hip", "axpic_device.hpp", "axpic_timing.hpp",
                os.path.join("..", "..", "include", "axpic.h"))


def source_digest(root: str = CSRC) -> str:
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        h.update(name.encode())
        with open(os.path.join(root, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def step_kernels(root: str = CSRC) -> set:
    """Names of the __global__ kernels defined in the stepping unit."""
    with open(os.path.join(root, STEP_SOURCES[0])) as f:
        text = f.read()
    return set(re.findall(r"\b(k_[A-Za-z0-9_]+)\s*\(", text))


def read_traffic(path: str, kernel: str):
    """(fetch_bytes, write_bytes) per dispatch of `kernel` from a summary written
    by main(), if its source digest matches the current sources."""
    if not os.path.exists(path):
        return None
    digest, found = None, None
    with open(path) as f:
        for line in f:
            t = line.split()
            if len(t) == 2 and t[0] == "source_sha256":
                digest = t[1]
            if len(t) == 4 and t[0] == "traffic" and t[1] == kernel:
                found = (float(t[2]), float(t[3]))
    if digest != source_digest() or found is None:
        return None
    return found


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


def sq_table(path):
    """Per kernel: median SQ_WAVES and the median per-wavefront value of every other
    counter in the file (one dispatch = one sample)."""
    per = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            key = (short(row["Kernel_Name"]), row["Dispatch_Id"])
            per.setdefault(key, {})[row["Counter_Name"]] = float(row["Counter_Value"])
    names = sorted({c for d in per.values() for c in d if c != "SQ_WAVES"})
    rows = {}
    for (k, _), d in per.items():
        if "SQ_WAVES" not in d or d["SQ_WAVES"] <= 0 or not k.startswith("k_"):
            continue
        rows.setdefault(k, []).append([d["SQ_WAVES"]] + [d.get(c, float("nan")) / d["SQ_WAVES"]
                                                          for c in names])
    print(f"{'kernel':20s} {'waves':>8s} " + " ".join(f"{c[3:]:>18s}" for c in names))
    for k in sorted(rows, key=lambda k: -statistics.median(r[0] for r in rows[k])):
        med = [statistics.median(col) for col in zip(*rows[k])]
        print(f"{k:20s} {med[0]:8.0f} " + " ".join(f"{v:18.1f}" for v in med[1:]))


def trace_table(path, since, nth):
    """Per kernel of a --kernel-trace CSV: calls and mean duration over the dispatches
    from the nth dispatch of kernel `since` on (in start order), e.g. one leg of a run."""
    with open(path) as f:
        rows = sorted(((short(r["Kernel_Name"]), int(r["Start_Timestamp"]),
                        int(r["End_Timestamp"])) for r in csv.DictReader(f)),
                      key=lambda r: r[1])
    seen, first = 0, None
    for i, (k, _, _) in enumerate(rows):
        if k == since:
            seen += 1
            if seen == nth:
                first = i
                break
    if first is None:
        raise SystemExit(f"no dispatch {nth} of {since}")
    acc = {}
    for k, a, b in rows[first:]:
        c, t = acc.get(k, (0, 0))
        acc[k] = (c + 1, t + (b - a))
    span = (rows[-1][2] - rows[first][1]) / 1e6
    print(f"window: {len(rows) - first} dispatches over {span:.1f} ms")
    print(f"{'kernel':24s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s}")
    for k, (c, t) in sorted(acc.items(), key=lambda kv: -kv[1][1]):
        print(f"{k:24s} {c:6d} {t / c / 1e3:10.2f} {t / 1e6:10.3f}")


def main(argv):
    if len(argv) > 2 and argv[1] == "--sq":
        sq_table(argv[2])
        return
    if len(argv) > 4 and argv[1] == "--trace":
        trace_table(argv[2], argv[3], int(argv[4]))
        return
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
    if fetch and write:
        print("per-dispatch HBM bytes (kernel fetch write):")
        own = step_kernels()
        for k in sorted(k for k in set(fetch) & set(write) if k in own):
            fb = statistics.mean(fetch[k][-LAST_DISPATCHES:]) * 1024 * scale_f
            wb = statistics.mean(write[k][-LAST_DISPATCHES:]) * 1024 * scale_w
            print(f"traffic {k} {fb:.6g} {wb:.6g}")
        print(f"source_sha256 {source_digest()}")


if __name__ == "__main__":
    main(sys.argv)
