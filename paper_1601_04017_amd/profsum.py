"""Summarises rocprofv3 CSV output of the benchmark into short text files.

    python -m paper_1601_04017_amd.profsum --trace DIR/bench_kernel_stats.csv \
        --fetch DIR/bench_counter_collection.csv --write DIR/bench_counter_collection.csv \
        --cal-fetch DIR/rl_counter_collection.csv --cal-write DIR/rl_counter_collection.csv \
        --cmd "..." --out profiles/NAME

Writes NAME.md (kernel durations, HBM bytes per dispatch) and NAME.traffic.json
(the dominant kernel's measured HBM bytes per launch, with the hash of the
kernel source the counters were taken with).

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what the same
counters read for the plain streaming copy of libroofline.so, whose true byte
count is known: factor = true bytes / counted bytes.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import OrderedDict

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRCS = [os.path.join(PKG, "csrc", f) for f in ("lpht_kernels.hip", "lpht_migrate.h", "lpht_device.h", "lpht_internal.h")]
SHRINK_SRCS = [os.path.join(PKG, "csrc", f)
               for f in ("lpht_shrink.hip", "lpht_shrink.h", "lpht_device.h", "lpht_internal.h")]
STR_SRCS = [os.path.join(PKG, "csrc", f) for f in ("lpht_str.hip", "lpht_str.h", "lpht_device.h", "lpht_internal.h")]
ASYNC_SRCS = [os.path.join(PKG, "csrc", f)
              for f in ("lpht_async.hip", "lpht_async.h", "lpht_migrate.h", "lpht_device.h", "lpht_internal.h")]
PART_SRCS = [os.path.join(PKG, "csrc", f) for f in ("lpht_part.hip", "lpht_part.h", "lpht_device.h", "lpht_internal.h")]


def kernel_source_sha(srcs=None) -> str:
    """Hash of the sources the table kernels (or the given files) are built from."""
    h = hashlib.sha256()
    for f in srcs or KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("lpht::", "").replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    name = name.split("(")[0] if "(" in name else name
    return name if len(name) <= 48 else name[:45] + "..."


def read_stats(path):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        out.append({"name": _short(r["Name"]), "calls": int(r["Calls"]),
                    "avg_us": float(r["AverageNs"]) / 1e3, "total_ms": float(r["TotalDurationNs"]) / 1e6,
                    "pct": float(r["Percentage"])})
    return out


def read_counters(path, counter):
    agg = OrderedDict()
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        agg.setdefault(_short(r["Kernel_Name"]), []).append(
            (int(r["Grid_Size"]), float(r["Counter_Value"])))
    return agg


def calibration(path, counter, true_bytes):
    vals = read_counters(path, counter).get("k_copy")
    if not vals:
        raise SystemExit(f"no k_copy dispatch with {counter} in {path}")
    kib = sum(v for _, v in vals) / len(vals)
    return true_bytes / (kib * 1024.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", help="FETCH_SIZE pass (omit, with the other counter files, for a "
                                    "durations-only summary)")
    ap.add_argument("--write")
    ap.add_argument("--cal-fetch")
    ap.add_argument("--cal-write")
    ap.add_argument("--rows", type=int, default=14, help="kernels listed in the durations table")
    ap.add_argument("--copy-bytes", type=float, default=float(1 << 31),
                    help="bytes read (= bytes written) by one calibration copy")
    ap.add_argument("--cmd", required=True, help="the commands that produced the CSV files")
    ap.add_argument("--dominant", default="k_bulk<1, 1, 0, 1>",
                    help="kernel whose bytes per launch go into the benchmark's roofline")
    ap.add_argument("--min-frac", type=float, default=0.05,
                    help="ignore dispatches whose count is below this fraction of the kernel's "
                         "largest (small spot-check launches)")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()

    stats = read_stats(a.trace)
    lines = [f"# rocprofv3 summary: {os.path.basename(a.out)}", "", "Commands:", "", "```"]
    lines += a.cmd.split(";;")
    lines += ["```", "", f"Kernel source sha256[:16]: `{kernel_source_sha()}` "
              f"(shrink kernels: `{kernel_source_sha(SHRINK_SRCS)}`, "
              f"string-key kernels: `{kernel_source_sha(STR_SRCS)}`, "
              f"in-kernel growth: `{kernel_source_sha(ASYNC_SRCS)}`, "
              f"partitioned insert-or-add: `{kernel_source_sha(PART_SRCS)}`)", "",
              "## Kernel durations (--kernel-trace --stats)", "",
              "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for s in stats[:a.rows]:
        lines.append(f"| `{s['name']}` | {s['calls']} | {s['avg_us']:.1f} | {s['total_ms']:.2f} | {s['pct']:.1f} |")
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    if not a.fetch:
        with open(a.out + ".md", "w") as f:
            f.write("\n".join(lines) + "\n")
        print(open(a.out + ".md").read())
        return
    ff = calibration(a.cal_fetch, "FETCH_SIZE", a.copy_bytes)
    fw = calibration(a.cal_write, "WRITE_SIZE", a.copy_bytes)
    fetch = read_counters(a.fetch, "FETCH_SIZE")
    write = read_counters(a.write, "WRITE_SIZE")
    lines += ["", f"## HBM bytes per dispatch (FETCH_SIZE x {ff:.3f}, WRITE_SIZE x {fw:.3f})", "",
              "Calibration: a streaming copy of libroofline.so moving a known byte count.", "",
              "| kernel | dispatches | read MB/dispatch | write MB/dispatch |", "|---|---|---|---|"]
    traffic = {}
    for name, vals in fetch.items():
        big = [v for _, v in vals if v >= a.min_frac * max(x for _, x in vals)]
        wvals = write.get(name, [])
        wv = [v for _, v in wvals if wvals and v >= a.min_frac * max(x for _, x in wvals)]
        if not big or not wv:
            continue
        rd = sum(big) / len(big) * 1024 * ff
        wr = sum(wv) / len(wv) * 1024 * fw
        traffic[name] = {"read_bytes": rd, "write_bytes": wr, "dispatches": len(big)}
        lines.append(f"| `{name}` | {len(big)} | {rd / 1e6:.1f} | {wr / 1e6:.1f} |")
    lines.append("")
    with open(a.out + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")
    dom = traffic.get(a.dominant)
    with open(a.out + ".traffic.json", "w") as f:
        json.dump({"kernel": a.dominant, "kernel_source_sha": kernel_source_sha(),
                   "fetch_factor": ff, "write_factor": fw,
                   "bytes_per_launch": None if dom is None else dom["read_bytes"] + dom["write_bytes"],
                   "read_bytes_per_launch": None if dom is None else dom["read_bytes"],
                   "write_bytes_per_launch": None if dom is None else dom["write_bytes"],
                   "per_kernel": traffic}, f, indent=1)
    print(open(a.out + ".md").read())


if __name__ == "__main__":
    main()
