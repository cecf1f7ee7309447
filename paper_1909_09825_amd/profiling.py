"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_1909_09825_amd.profiling trace  <kernel_trace.csv> --command "..." --out F.md
    python -m paper_1909_09825_amd.profiling traffic <fetch counter_collection.csv> <write ...csv>
            --copy-bytes B --command "..." --out profiles/traffic_counters.json
    python -m paper_1909_09825_amd.profiling valu <counter_collection.csv> --command "..."
            --out profiles/valu_counters.json --md profiles/F.md
    python -m paper_1909_09825_amd.profiling stalls <counter_collection.csv> --command "..."
            --out profiles/F.md
    python -m paper_1909_09825_amd.profiling mix <counter_collection.csv> --command "..."
            --out profiles/F.md --json profiles/valu_mix_counters.json

`trace` writes a per-kernel table (dispatches, mean duration, and for the
radix-pass kernel the mean over the dispatches that move data, i.e. the ones
longer than a twentieth of the longest).  rocprofv3 reports a counter in
several rows per dispatch (one per hardware instance); they are summed per
dispatch.  `traffic` turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch) into
HBM bytes per launch, each scaled by what the same counter reads for the plain
device copy of `copy_bytes` bytes that bench.py runs with --copy-bytes; `valu`
records the SQ instruction counters per launch of each kernel's largest
dispatches (the full-size workload) and the fraction of the chip's VALU issue
slots they fill during the counter run.  Both record a hash of the kernel
sources so that bench.py uses a figure only while the kernels are unchanged.
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
_SCAN = ["paper_1909_09825_amd/csrc/fgt_scan.hip", "paper_1909_09825_amd/csrc/fgt_device.h",
         "paper_1909_09825_amd/csrc/fgt_internal.h"]
_SORT = ["paper_1909_09825_amd/csrc/fgt_sort.hip", "paper_1909_09825_amd/csrc/fgt_internal.h"]
_ADJ = ["paper_1909_09825_amd/csrc/fgt_adjoint.hip", "paper_1909_09825_amd/csrc/fgt_device.h",
        "paper_1909_09825_amd/csrc/fgt_internal.h"]
_BATCH = ["paper_1909_09825_amd/csrc/fgt_batch.hip", "paper_1909_09825_amd/csrc/fgt_device.h",
          "paper_1909_09825_amd/csrc/fgt_internal.h"]
KERNEL_SOURCES = {
    "k_onesweep": _SORT, "k_range": _SORT, "k_histogram": _SORT,
    "k_wreduce": _SCAN, "k_wfinal_fast": _SCAN, "k_gather": _SCAN,
    "k_adj_reduce": _ADJ, "k_adj_final_fast": _ADJ,
    "k_bscan": _BATCH, "k_bucket_sort": _BATCH, "k_seg_scatter": _BATCH,
}
COPY_KERNEL = "__amd_rocclr_copyBuffer"
# VALU issue slots per second: 256 CUs x 4 SIMDs at 2.4 GHz, 4 cycles per wave64 instruction.
VALU_SLOTS_PER_S = 256 * 4 * 2.4e9 / 4


def code_text(src: str) -> str:
    """C++ source without comments and with whitespace collapsed, so that a
    comment edit does not count as a change of the kernel."""
    out = []
    i, n = 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":                       # string or character literal, kept whole
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
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


def main_grid(base: str, grids):
    """The dispatches that stand for a kernel: its largest grid (the full-size
    single transform), or for the batched kernels the grid launched most often
    (the autotuner times other configurations a few times each)."""
    if base.startswith(("k_bscan", "k_bucket", "k_seg")):
        cnt = collections.Counter(grids)
        return max(cnt, key=lambda g: (cnt[g], g))
    return max(grids)


def load_counter(path, counter):
    """{kernel: [(value summed over the dispatch's rows, grid size, duration us)]}."""
    per = collections.defaultdict(float)
    meta = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            key = (short_name(r["Kernel_Name"]), r["Dispatch_Id"])
            per[key] += float(r["Counter_Value"])
            meta[key] = (int(r["Grid_Size"]),
                         (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    vals = collections.defaultdict(list)
    for key, v in per.items():
        vals[key[0]].append((v, *meta[key]))
    return vals


def traffic(fetch_csv, write_csv, copy_bytes: int, command: str):
    fetch = load_counter(fetch_csv, "FETCH_SIZE")
    write = load_counter(write_csv, "WRITE_SIZE")
    f_scale = copy_bytes / (1024.0 * max(v for v, _, _ in fetch[COPY_KERNEL]))
    w_scale = copy_bytes / (1024.0 * max(v for v, _, _ in write[COPY_KERNEL]))
    out = {"_about": ("HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB, summed "
                      "over each dispatch's rows), scaled by the same counters on a plain copy of "
                      "copy_bytes bytes; the mean is over each kernel's dispatches of the largest "
                      "grid that move data (more than a twentieth of the largest)"),
           "command": command, "copy_bytes": copy_bytes,
           "fetch_scale": f_scale, "write_scale": w_scale}
    for k in fetch:
        b = base_name(k)
        if b not in KERNEL_SOURCES:
            continue
        grid = main_grid(b, [g for _, g, _ in fetch[k]])
        fv = [v for v, g, _ in fetch[k] if g == grid]
        wv = [v for v, g, _ in write.get(k, []) if g == grid] or [0.0]
        big_f = [v for v in fv if v > 0.05 * max(fv)] or [0.0]
        big_w = [v for v in wv if v > 0.05 * max(wv)] or [0.0]
        fb = sum(big_f) / len(big_f) * 1024.0 * f_scale
        wb = sum(big_w) / len(big_w) * 1024.0 * w_scale
        name = b if b not in out else k
        out[name] = {"kernel": k, "grid": grid, "fetch_bytes": fb, "write_bytes": wb,
                     "bytes_per_launch": fb + wb, "sources": KERNEL_SOURCES[b],
                     "source_sha": source_hash(KERNEL_SOURCES[b])}
    return out


SQ = ["SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS",
      "SQ_LDS_BANK_CONFLICT", "SQ_WAVES", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES"]


def valu(csv_path, command: str):
    """Per kernel (its main grid, see main_grid; data-moving dispatches): SQ counters per launch."""
    data = {c: load_counter(csv_path, c) for c in SQ}
    out = {"_about": ("SQ instruction counters per launch (wave instructions, summed over each "
                      "dispatch's rows) for each kernel's dispatches of its main grid (the largest; "
                      "for batched kernels the one launched most often) that do work; valu_frac_pmc = SQ_INSTS_VALU x 4 cycles over the chip's VALU issue "
                      "slots (1024 SIMDs at 2.4 GHz) during the counter run's own dispatch time"),
           "command": command}
    for k, rows in data["SQ_INSTS_VALU"].items():
        b = base_name(k)
        if b not in KERNEL_SOURCES:
            continue
        grid = main_grid(b, [g for _, g, _ in rows])
        vals = [(v, d) for v, g, d in rows if g == grid]
        vmax = max(v for v, _ in vals)
        keep = [(v, d) for v, d in vals if v > 0.05 * vmax] or vals
        rec = {"kernel": k, "grid": grid, "dispatches": len(keep),
               "valu_insts_per_launch": sum(v for v, _ in keep) / len(keep),
               "us_per_launch_pmc": sum(d for _, d in keep) / len(keep)}
        for c in SQ[1:]:
            cv = [v for v, g, _ in data[c].get(k, []) if g == grid]
            cv = sorted(cv)[-len(keep):] if cv else [0.0]
            rec[c.lower() + "_per_launch"] = sum(cv) / len(cv)
        rec["valu_frac_pmc"] = rec["valu_insts_per_launch"] / (
            rec["us_per_launch_pmc"] * 1e-6 * VALU_SLOTS_PER_S)
        rec["sources"] = KERNEL_SOURCES[b]
        rec["source_sha"] = source_hash(KERNEL_SOURCES[b])
        out[k if b in out or b in ("k_bscan",) else b] = rec
    return out


def valu_md(rec: dict) -> str:
    lines = ["# rocprofv3 SQ counters (VALU, LDS)", "", f"Command: `{rec['command']}`", "",
             rec["_about"] + ".", "",
             "| kernel | grid | launches | us/launch (counter run) | VALU insts | VALU issue frac "
             "| LDS insts | LDS bank conflicts | SALU insts | waves |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for name, r in rec.items():
        if name.startswith("_") or name == "command":
            continue
        lines.append(f"| `{r['kernel']}` | {r['grid']} | {r['dispatches']} | "
                     f"{r['us_per_launch_pmc']:.1f} | {r['valu_insts_per_launch']:.4g} | "
                     f"{r['valu_frac_pmc']:.3f} | {r['sq_insts_lds_per_launch']:.4g} | "
                     f"{r['sq_lds_bank_conflict_per_launch']:.4g} | "
                     f"{r['sq_insts_salu_per_launch']:.4g} | {r['sq_waves_per_launch']:.0f} |")
    return "\n".join(lines) + "\n"


STALL = ["SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
         "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_INSTS_VALU"]


def stalls(csv_path, command: str) -> str:
    """Where each kernel's waves spend their time: SQ wave-cycle counters per launch as
    fractions of SQ_WAVE_CYCLES (all of them count in the same cycle units)."""
    data = {c: load_counter(csv_path, c) for c in STALL}
    lines = ["# rocprofv3 SQ wait and activity counters", "", f"Command: `{command}`", "",
             "Per kernel (its main grid, data-moving dispatches), each counter summed over the "
             "dispatch's rows and taken as a fraction of SQ_WAVE_CYCLES (the cycles its waves are "
             "resident): waiting on anything (SQ_WAIT_ANY: memory or barrier dependencies), "
             "waiting to issue (SQ_WAIT_INST_ANY), waiting to issue an LDS instruction "
             "(SQ_WAIT_INST_LDS), issuing VALU (SQ_ACTIVE_INST_VALU) and LDS (SQ_ACTIVE_INST_LDS) "
             "instructions; the fractions are per resident wave.", "",
             "| kernel | grid | launches | us/launch (counter run) | wait any | wait issue "
             "| wait LDS issue | VALU active | LDS active |",
             "|---|---|---|---|---|---|---|---|---|"]
    for k, rows in sorted(data["SQ_WAVE_CYCLES"].items()):
        b = base_name(k)
        if b not in KERNEL_SOURCES:
            continue
        grid = main_grid(b, [g for _, g, _ in rows])
        vals = [(v, d) for v, g, d in rows if g == grid]
        vmax = max(v for v, _ in vals)
        keep = [(v, d) for v, d in vals if v > 0.05 * vmax] or vals
        wc = sum(v for v, _ in keep) / len(keep)

        def frac(c):
            cv = [v for v, g, _ in data[c].get(k, []) if g == grid]
            cv = sorted(cv)[-len(keep):] if cv else [0.0]
            return (sum(cv) / len(cv)) / wc if wc > 0 else 0.0
        us = sum(d for _, d in keep) / len(keep)
        lines.append(f"| `{k}` | {grid} | {len(keep)} | {us:.1f} | {frac('SQ_WAIT_ANY'):.3f} | "
                     f"{frac('SQ_WAIT_INST_ANY'):.3f} | {frac('SQ_WAIT_INST_LDS'):.3f} | "
                     f"{frac('SQ_ACTIVE_INST_VALU'):.3f} | {frac('SQ_ACTIVE_INST_LDS'):.3f} |")
    return "\n".join(lines) + "\n"


MIX = ["SQ_INSTS_VALU", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
       "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU_INT32",
       "SQ_INSTS_VALU_INT64"]
FP64_PEAK_FLOPS = 78.6e12   # MI355X FP64 vector, an FMA counted as two operations


def mix(csv_path, command: str):
    """FP64 operation rate and instruction mix per kernel (wave instructions x 64 lanes):
    the markdown table and a record per kernel (FP64 operations per launch, sources hash)."""
    data = {c: load_counter(csv_path, c) for c in MIX}
    rec = {"_about": ("FP64 operations per launch (64 lanes x (add + mul + 2 fma) wave "
                      "instructions) from SQ_INSTS_VALU_{ADD,MUL,FMA}_F64 on each kernel's main grid"),
           "command": command}
    lines = ["# rocprofv3 VALU instruction mix and FP64 rate", "", f"Command: `{command}`", "",
             "Per kernel (its main grid, data-moving dispatches): wave-level VALU instructions per "
             "launch, the FP64 add, multiply and FMA instructions among them, transcendental and "
             "integer instructions; FP64 FLOP/s = 64 lanes x (add + mul + 2 fma) over the counter "
             "run's own dispatch time, against the 78.6 TFLOP/s FP64 vector peak; f64 share = "
             "FP64 arithmetic instructions / all VALU instructions.", "",
             "| kernel | grid | us/launch (counter run) | VALU insts | FP64 add | FP64 mul | FP64 fma "
             "| trans F64 | trans F32 | int32 | int64 | FP64 TFLOP/s | of peak | f64 share |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for k, rows in sorted(data["SQ_INSTS_VALU"].items()):
        b = base_name(k)
        if b not in KERNEL_SOURCES:
            continue
        grid = main_grid(b, [g for _, g, _ in rows])
        vals = [(v, d) for v, g, d in rows if g == grid]
        vmax = max(v for v, _ in vals)
        keep = [(v, d) for v, d in vals if v > 0.05 * vmax] or vals
        valu = sum(v for v, _ in keep) / len(keep)
        us = sum(d for _, d in keep) / len(keep)

        def per(c):
            cv = [v for v, g, _ in data[c].get(k, []) if g == grid]
            cv = sorted(cv)[-len(keep):] if cv else [0.0]
            return sum(cv) / len(cv)
        add, mul, fma = per("SQ_INSTS_VALU_ADD_F64"), per("SQ_INSTS_VALU_MUL_F64"), \
            per("SQ_INSTS_VALU_FMA_F64")
        flops = 64.0 * (add + mul + 2.0 * fma) / (us * 1e-6) if us > 0 else 0.0
        # The base name stands for the instantiation with the most VALU work (the
        # common one); the others keep their full names.
        r = {"kernel": k, "grid": grid, "fp64_ops_per_launch": 64.0 * (add + mul + 2.0 * fma),
             "valu_insts_per_launch": valu, "us_per_launch_pmc": us,
             "sources": KERNEL_SOURCES[b], "source_sha": source_hash(KERNEL_SOURCES[b])}
        if b not in rec or rec[b]["valu_insts_per_launch"] < valu:
            if b in rec:
                rec[rec[b]["kernel"]] = rec[b]
            rec[b] = r
        else:
            rec[k] = r
        lines.append(f"| `{k}` | {grid} | {us:.1f} | {valu:.4g} | {add:.3g} | {mul:.3g} | {fma:.3g} | "
                     f"{per('SQ_INSTS_VALU_TRANS_F64'):.3g} | {per('SQ_INSTS_VALU_TRANS_F32'):.3g} | "
                     f"{per('SQ_INSTS_VALU_INT32'):.3g} | {per('SQ_INSTS_VALU_INT64'):.3g} | "
                     f"{flops / 1e12:.2f} | {flops / FP64_PEAK_FLOPS:.3f} | "
                     f"{(add + mul + fma) / valu if valu else 0.0:.2f} |")
    return "\n".join(lines) + "\n", rec


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
    v = sub.add_parser("valu")
    v.add_argument("csv")
    v.add_argument("--command", required=True)
    v.add_argument("--out", required=True)
    v.add_argument("--md", required=True)
    x = sub.add_parser("mix")
    x.add_argument("csv")
    x.add_argument("--command", required=True)
    x.add_argument("--out", required=True)
    x.add_argument("--json", required=True)
    w = sub.add_parser("stalls")
    w.add_argument("csv")
    w.add_argument("--command", required=True)
    w.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "mix":
        text, rec = mix(a.csv, a.command)
        with open(a.out, "w") as f:
            f.write(text)
        with open(a.json, "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
    elif a.cmd == "stalls":
        with open(a.out, "w") as f:
            f.write(stalls(a.csv, a.command))
    elif a.cmd == "trace":
        with open(a.out, "w") as f:
            f.write(trace_summary(a.csv, a.command))
    elif a.cmd == "traffic":
        with open(a.out, "w") as f:
            json.dump(traffic(a.fetch_csv, a.write_csv, a.copy_bytes, a.command), f, indent=1)
            f.write("\n")
    else:
        rec = valu(a.csv, a.command)
        with open(a.out, "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
        with open(a.md, "w") as f:
            f.write(valu_md(rec))


if __name__ == "__main__":
    main()
