"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_1909_09825_amd.profiling trace  <kernel_trace.csv> --command "..." --out F.md
    python -m paper_1909_09825_amd.profiling traffic <fetch counter_collection.csv> <write ...csv>
            --copy-bytes B --steps S --command "..." --out profiles/traffic_counters.json

`trace` writes a per-kernel table (dispatches, mean duration, and for the
radix-pass kernel the mean over the dispatches that move data, i.e. the ones
longer than a twentieth of the longest).  `traffic` turns FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) into HBM bytes per launch, each scaled by what
the same counter reads for the plain device copy of `copy_bytes` bytes that
bench.py runs with --copy-bytes, and records a hash of the kernel sources so
that bench.py reports the figure only while the kernels are unchanged.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
KERNEL_SOURCES = {
    "k_onesweep": ["paper_1909_09825_amd/csrc/fgt_sort.hip", "paper_1909_09825_amd/csrc/fgt_internal.h"],
    "k_final_fast": ["paper_1909_09825_amd/csrc/fgt_scan.hip", "paper_1909_09825_amd/csrc/fgt_device.h",
                     "paper_1909_09825_amd/csrc/fgt_internal.h"],
    "k_reduce": ["paper_1909_09825_amd/csrc/fgt_scan.hip", "paper_1909_09825_amd/csrc/fgt_device.h",
                 "paper_1909_09825_amd/csrc/fgt_internal.h"],
}
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def source_hash(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """'void fgt::(anonymous namespace)::k_onesweep<double>(int, ...)' -> 'k_onesweep<double>'."""
    m = re.search(r"::(\w+(?:<[^()]*>)?)\(", name)
    return m.group(1) if m else name.strip()


def base_name(name: str) -> str:
    return short_name(name).split("<")[0]


def load_trace(path):
    durs = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            durs[short_name(r["Kernel_Name"])].append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return durs


def trace_summary(path, command: str) -> str:
    durs = load_trace(path)
    lines = ["# rocprofv3 kernel trace", "", f"Command: `{command}`", "",
             "| kernel | dispatches | mean us | mean us (data-moving dispatches) | total ms |",
             "|---|---|---|---|---|"]
    for k, v in sorted(durs.items(), key=lambda kv: -sum(kv[1])):
        big = [d for d in v if d > 0.05 * max(v)]
        lines.append(f"| `{k}` | {len(v)} | {sum(v) / len(v):.1f} | "
                     f"{sum(big) / len(big):.1f} ({len(big)}) | {sum(v) / 1e3:.3f} |")
    return "\n".join(lines) + "\n"


def load_counter(path, counter):
    vals = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                vals[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return vals


def traffic(fetch_csv, write_csv, copy_bytes: int, command: str):
    fetch = load_counter(fetch_csv, "FETCH_SIZE")
    write = load_counter(write_csv, "WRITE_SIZE")
    f_scale = copy_bytes / (1024.0 * sum(fetch[COPY_KERNEL]))
    w_scale = copy_bytes / (1024.0 * sum(write[COPY_KERNEL]))
    out = {"_about": ("HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per "
                      "dispatch), scaled by the same counters on a plain copy of copy_bytes bytes; "
                      "for the radix-pass kernel the mean is over the data-moving dispatches"),
           "command": command, "copy_bytes": copy_bytes,
           "fetch_scale": f_scale, "write_scale": w_scale}
    for k in fetch:
        b = base_name(k)
        if b not in KERNEL_SOURCES:
            continue
        fv, wv = fetch[k], write.get(k, [])
        big_f = [v for v in fv if v > 0.05 * max(fv)]
        big_w = [v for v in wv if v > 0.05 * max(wv)] if wv else [0.0]
        fb = sum(big_f) / len(big_f) * 1024.0 * f_scale
        wb = sum(big_w) / len(big_w) * 1024.0 * w_scale
        out[b] = {"kernel": k, "fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                  "sources": KERNEL_SOURCES[b], "source_sha": source_hash(KERNEL_SOURCES[b])}
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--command", required=True)
    t.add_argument("--out", required=True)
    c = sub.add_parser("traffic")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "trace":
        with open(a.out, "w") as f:
            f.write(trace_summary(a.csv, a.command))
    else:
        with open(a.out, "w") as f:
            json.dump(traffic(a.fetch_csv, a.write_csv, a.copy_bytes, a.command), f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
