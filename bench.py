#!/usr/bin/env python3
"""Benchmark of the 1-D fast Gauss transform on one MI355X.

One step = one fgt_eval over the whole hot path (key build, radix sort,
tile-scan reduce, carries, fused forward/backward sweeps, mode reduction and
scatter) for M = N = 2^24 points uniform on [0,1), alpha ~ N(0,1),
delta = 1e-4, 6 digits (4 modes), FP64, with inputs resident in HBM.

Prints ONE JSON line.  `value` is (M+N) * modes / s.  `fwd_bwd` times, on the
same inputs, the forward followed by the adjoint (fgt_backward on the sorted
workspace: dL/dalpha, dL/dx, dL/dy and dL/ddelta for L = g . u, g ~ N(0,1)).
`batched` times fgt_batch_eval on 4096 transforms (N_b, M_b log-uniform in
[256, 65536], delta_b log-uniform in [1e-6, 1e-2], 16 columns, 6 digits),
eagerly and as a replayed HIP graph, next to a loop of fgt_eval calls (one per
transform and column) timed on 32 of the transforms and scaled to 4096.
`plan_reuse` times fgt_eval_sorted (new strengths on the sorted points, the
sort skipped).  `identical_points` times fgt_eval_self in the setting of the
paper's Table 1 (targets = sources, N = 10^7 uniform on [0,1), delta = 1,
n_e = 3..6), with Chebyshev points in order and the sort skipped beside it.
`small` gives the latency
of one transform at M = N = 1000 (delta 1e-3, 6 digits), eager and as a
replayed HIP graph; `clustered` the 2^24-source Gaussian-mixture case with
2^22 uniform targets (delta 1e-5, FP64 and FP32 at 6 digits); `differentiation`
forward against forward + adjoint at M = N = 2^22 (delta 1e-4, FP64 at 9 digits,
FP32 at 4 digits).  Every time is the wall clock over the timed calls
(synchronised on both sides) next to the median of per-call HIP events.
`roofline` describes the kernel with the largest share of the step, timed with
HIP events that the library records on its own stream during K further steps
run right after the timed ones (those events cost a few microseconds each, so
the steps that carry them are not the ones `value` is taken from);
`cpu_baseline` is the CPU oracle's SOE recurrence timed on a bounded sample of
the same inputs, on one thread and on all of the host's cores, with and
without its sort.

    python bench.py [--steps K] [--warmup W] [--delta D] [--digits G] [--log2n L]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X FP64 vector
# VALU issue slots: 256 CUs x 4 SIMDs at 2.4 GHz; a wave64 VALU instruction
# occupies a 16-lane SIMD for 4 cycles (FP64 FMA at the 78.6 TFLOP/s peak).
VALU_SLOTS_PER_S = 256 * 4 * 2.4e9 / 4
METRIC = "(M+N)·modes/s and transforms/s at 6 digits, fwd vs fwd+bwd, % HBM roofline"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_counters.json")
MIX_FILE = os.path.join(ROOT, "profiles", "valu_mix_counters.json")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--delta", type=float, default=1e-4)
    ap.add_argument("--digits", type=int, default=6)
    ap.add_argument("--log2n", type=int, default=24, help="M = N = 2^log2n")
    ap.add_argument("--fp32", action="store_true", help="time the FP32 path instead")
    ap.add_argument("--cpu-sample-log2n", type=int, default=22,
                    help="CPU oracle timed on the first 2^k targets and sources")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grad", action="store_true", help="skip the fwd+bwd timing")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched timing")
    ap.add_argument("--no-identical", action="store_true",
                    help="skip the identical-points (Table 1 setting) timing")
    ap.add_argument("--no-small", action="store_true", help="skip the M = N = 1000 latency")
    ap.add_argument("--no-clustered", action="store_true", help="skip the clustered workload")
    ap.add_argument("--no-diff", action="store_true", help="skip the 2^22 differentiation rows")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one plain device copy of this many bytes (counter calibration)")
    return ap.parse_args()


def _counter_record(path, kernel):
    """A committed per-kernel counter record, if the kernel's sources are unchanged."""
    from paper_1909_09825_amd.profiling import source_hash
    try:
        with open(path) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != source_hash(rec["sources"]):
        return None
    return rec


def traffic_for(kernel: str):
    """HBM bytes per launch from committed counter runs, if the kernel source is unchanged."""
    rec = _counter_record(TRAFFIC_FILE, kernel)
    return int(rec["bytes_per_launch"]) if rec else None


def valu_frac(kernel: str, ms_launch: float):
    """Fraction of the chip's VALU issue slots used: committed SQ_INSTS_VALU per
    launch (wave instructions, 4 cycles each) over the launch's measured time."""
    rec = _counter_record(VALU_FILE, kernel)
    if not rec or ms_launch <= 0:
        return None
    return round(float(rec["valu_insts_per_launch"]) / (ms_launch * 1e-3 * VALU_SLOTS_PER_S), 4)


def fp64_frac(kernel: str, ms_launch: float):
    """FP64 operations per launch from the committed instruction-mix counters (an FMA
    counted as two) over the launch's measured time, as a fraction of the FP64 vector peak."""
    rec = _counter_record(MIX_FILE, kernel)
    if not rec or ms_launch <= 0:
        return None
    return round(float(rec["fp64_ops_per_launch"]) / (ms_launch * 1e-3)
                 / (FP64_VALU_PEAK_TFLOPS * 1e12), 4)


def timed(fn, steps, warmup, torch):
    """Warm up, then run `steps` calls: wall clock over all of them (synchronised
    on both sides) and the median of per-call HIP events on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return wall, statistics.median(a.elapsed_time(b) for a, b in evs)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(x, y, a, delta, digits, n_modes, k):
    """The CPU oracle's SOE recurrence (sort + per-mode sweeps) on the first 2^k
    targets and sources: one thread and all of the host's cores (OpenMP over the
    2 n_e sweeps), each with and without the sort (the paper's t_total and t_linear)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle
    from conftest import load_oracle_tables
    t = load_oracle_tables()[n_modes]
    n = 1 << k
    xs, ys, as_ = x[:n].copy(), y[:n].copy(), a[:n].copy()
    work = (2 * n) * n_modes
    legs = {}
    all_threads = oracle.max_threads()
    for name, threads in (("one_core", 1), ("all_cores", all_threads)):
        t0 = time.perf_counter()
        oracle.soe_recurrence(xs, ys, as_, delta, t["tau0"], t["omega"], threads=threads)
        dt = time.perf_counter() - t0
        ts = oracle.last_sort_seconds()
        legs[name] = {"threads": threads, "s_total": round(dt, 3), "s_sort": round(ts, 3),
                      "with_sort": work / dt, "without_sort": work / max(dt - ts, 1e-9)}
    return {
        "value": legs["all_cores"]["with_sort"], "unit": "point-modes/s",
        "cores": all_threads, "kind": "oracle",
        "sample": (f"first 2^{k} targets and 2^{k} sources of the same inputs, {digits} digits "
                   f"({n_modes} modes): O2 SOE recurrence in C (qsort, then one sweep per mode and "
                   f"direction, OpenMP over the {2 * n_modes} sweeps), "
                   f"{legs['all_cores']['s_total']:.2f} s wall on {all_threads} threads"),
        "host": {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
                 "omp_threads": all_threads, "cpu": cpu_model()},
        "one_core": legs["one_core"],
        "all_cores": legs["all_cores"],
    }


def bench_identical(args, fgt, W, torch, np, dev):
    N = 10_000_000
    x, a = W.identical_uniform(N)
    X = torch.from_numpy(x).to(dev)
    A = torch.from_numpy(a).to(dev)
    Xc = torch.from_numpy(W.chebyshev(N)).to(dev)
    U = torch.empty(N, dtype=torch.float64, device=dev)
    rows = []
    for digits in (5, 6, 8, 10):
        p = fgt.plan(1.0, digits)
        ws = fgt.workspace(p, 0, N, dev)
        res = {"n_e": p.n_modes, "digits": digits}
        for name, pts, pre in (("uniform", X, False), ("chebyshev_presorted", Xc, True)):
            for _ in range(args.warmup):
                fgt.eval_self(pts, A, p, presorted=pre, out=U, ws=ws)
            torch.cuda.synchronize()
            if fgt.last_device_status(ws) != fgt.FGT_OK:
                raise RuntimeError("device status after identical-points warmup")
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fgt.eval_self(pts, A, p, presorted=pre, out=U, ws=ws)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            res[name] = {"ms": round(ms, 4), "points_per_s": N / (ms * 1e-3)}
        rows.append(res)
    return {
        "workload": "targets = sources, N = 10^7 uniform on [0,1) (or Chebyshev in order), "
                    "alpha ~ N(0,1), delta = 1, FP64",
        "rows": rows,
        "paper_context": ("Figure 7 (single core of an i7-4600U laptop): 2.6e6 to 1.7e6 points/s "
                          "for n_e = 3..6 without precomputation, 1.6e7 to 9e6 points/s with the "
                          "points pre-sorted and the exponentials precomputed"),
    }


def bench_batched(args, fgt, W, torch, np, dev):
    bt = W.batched()
    B, R = len(bt.delta), bt.alpha.shape[1]
    bp = fgt.batch_plan(bt.delta, bt.digits, bt.x_off, bt.y_off, R)
    X = torch.from_numpy(bt.x).to(dev)
    Y = torch.from_numpy(bt.y).to(dev)
    A = torch.from_numpy(bt.alpha).to(dev)
    U = torch.empty((bp.M, R), dtype=torch.float64, device=dev)
    ws = fgt.batch_workspace(bp, dev)
    t0 = time.perf_counter()
    config = bp.tune(X, Y, A, ws=ws)
    tune_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        fgt.eval_batch(X, Y, A, bp, out=U, ws=ws)
    torch.cuda.synchronize()
    if fgt.last_device_status(ws) != fgt.FGT_OK:
        raise RuntimeError("device status after batched warmup")
    ms_eager, ms_med = timed(lambda: fgt.eval_batch(X, Y, A, bp, out=U, ws=ws), args.steps, 0,
                             torch)
    # the same launch sequence captured once and replayed
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fgt.eval_batch(X, Y, A, bp, out=U, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fgt.eval_batch(X, Y, A, bp, out=U, ws=ws)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / args.steps
    # loop of single-transform calls on 32 transforms, all columns
    picks = np.random.default_rng(4).choice(B, 32, replace=False)
    calls = []
    for b in picks:
        xs, xe, ys, ye = (int(bt.x_off[b]), int(bt.x_off[b + 1]), int(bt.y_off[b]),
                          int(bt.y_off[b + 1]))
        p = fgt.plan(float(bt.delta[b]), bt.digits)
        wsb = fgt.workspace(p, xe - xs, ye - ys, dev)
        cols = [A[ys:ye, r].contiguous() for r in range(R)]
        calls.append((p, X[xs:xe], Y[ys:ye], cols, U[xs:xe, 0].clone(), wsb))
    for p, xb, yb, cols, ub, wsb in calls:
        fgt.eval(xb, yb, cols[0], p, out=ub, ws=wsb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, xb, yb, cols, ub, wsb in calls:
        for c in cols:
            fgt.eval(xb, yb, c, p, out=ub, ws=wsb)
    torch.cuda.synchronize()
    ms_loop32 = (time.perf_counter() - t0) * 1e3
    pts32 = sum(int(c[1].shape[0] + c[2].shape[0]) for c in calls)
    ms_loop = ms_loop32 * bp.total_points / pts32
    ms = min(ms_eager, ms_graph)
    # Roofline of the whole batch: every coordinate read once, alpha and u
    # (R columns) read and written once; VALU from the per-point-mode count of
    # one complex exponential (~50 lane-operations) and R columns of two
    # complex FMA sweeps plus the accumulation (~10 each).
    P = bp.total_points
    alg_bytes = 8 * P + 8 * R * (bp.N + bp.M)
    valu_ops = P * bp.n_modes * (50 + R * 10)
    cpu = batched_cpu_baseline(bt, bp.n_modes) if not args.no_cpu_baseline else None
    return {
        "workload": (f"{B} transforms, N_b and M_b log-uniform in [256, 65536], delta_b "
                     f"log-uniform in [1e-6, 1e-2], points uniform on [0,1), alpha [N][{R}] ~ N(0,1), "
                     f"{bt.digits} digits ({bp.n_modes} modes), FP64"),
        "total_points": P,
        "ms_per_batch_eager": round(ms_eager, 4),
        "ms_per_batch_graph": round(ms_graph, 4),
        "ms_median_event": round(ms_med, 4),
        "transforms_per_s": B / (ms * 1e-3),
        "column_transforms_per_s": B * R / (ms * 1e-3),
        "value": P * bp.n_modes * R / (ms * 1e-3),
        "unit": "point-mode-columns/s",
        "roofline": {"alg_bytes": int(alg_bytes), "hbm_frac": round(alg_bytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                     "valu_ops_model": int(valu_ops),
                     "valu_frac_model": round(valu_ops / (ms * 1e-3) / (FP64_VALU_PEAK_TFLOPS * 1e12 / 2), 4)},
        "loop_of_fgt_eval_ms": round(ms_loop, 2),
        "loop_sample": (f"fgt_eval once per column on 32 sampled transforms ({pts32} points), "
                        f"{ms_loop32:.1f} ms, scaled by total points"),
        "speedup_vs_loop": round(ms_loop / ms, 1),
        "tuned_config": {"points_per_lane": config[0], "bucket_points": config[1],
                         "tuning_s": round(tune_s, 2)},
        "cpu_baseline": cpu,
    }


def batched_cpu_baseline(bt, n_modes, n_pick=24):
    """The oracle's SOE recurrence, column by column, on a sample of the batch's
    transforms (all host threads, OpenMP over each call's sweeps)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import numpy as np
    import oracle
    from conftest import load_oracle_tables
    t = load_oracle_tables()[n_modes]
    picks = np.random.default_rng(7).choice(len(bt.delta), n_pick, replace=False)
    R = bt.alpha.shape[1]
    pts = 0
    t0 = time.perf_counter()
    for b in picks:
        xs, xe, ys, ye = (int(bt.x_off[b]), int(bt.x_off[b + 1]), int(bt.y_off[b]),
                          int(bt.y_off[b + 1]))
        for r in range(R):
            oracle.soe_recurrence(bt.x[xs:xe], bt.y[ys:ye], bt.alpha[ys:ye, r],
                                  float(bt.delta[b]), t["tau0"], t["omega"])
        pts += (xe - xs) + (ye - ys)
    dt = time.perf_counter() - t0
    return {"value": pts * n_modes * R / dt, "unit": "point-mode-columns/s",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{n_pick} sampled transforms x {R} columns ({pts} points), {dt:.2f} s wall"}


def bench_small(args, fgt, W, torch, np, dev):
    """M = N = 1000 (delta 1e-3, 6 digits): latency per transform."""
    pr = W.small_plain()
    p = fgt.plan(pr.delta, pr.digits)
    X, Y, A = (torch.from_numpy(v).to(dev) for v in (pr.x, pr.y, pr.alpha))
    ws = fgt.workspace(p, pr.M, pr.N, dev)
    u = torch.empty(pr.M, dtype=torch.float64, device=dev)
    steps = max(args.steps, 200)
    wall, med = timed(lambda: fgt.eval(X, Y, A, p, out=u, ws=ws), steps, 10, torch)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fgt.eval(X, Y, A, p, out=u, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fgt.eval(X, Y, A, p, out=u, ws=ws)
    gwall, gmed = timed(graph.replay, steps, 10, torch)
    if fgt.last_device_status(ws) != fgt.FGT_OK:
        raise RuntimeError("device status after the small workload")
    return {"workload": "M = N = 1000 uniform on [0,1), alpha ~ N(0,1), delta = 1e-3, 6 digits, FP64",
            "us_per_transform_eager": round(wall * 1e3, 2), "us_median_event_eager": round(med * 1e3, 2),
            "us_per_transform_graph": round(gwall * 1e3, 2), "us_median_event_graph": round(gmed * 1e3, 2),
            "transforms_per_s": 1e3 / min(wall, gwall)}


def scan_row(phases, calls, alg_bytes):
    """Time of the scan (tile reduce, carries, final sweeps) per call and its HBM fraction."""
    ms = sum(phases.get(k, 0.0) for k in ("tiles_reduce", "carry", "tiles_final")) / calls
    return {"ms": round(ms, 5), "alg_bytes": int(alg_bytes),
            "hbm_frac": round(alg_bytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4) if ms > 0 else None}


def bench_clustered(args, fgt, W, torch, np, dev):
    """2^24 sources from a 64-component Gaussian mixture, 2^22 uniform targets, delta 1e-5."""
    pr = W.clustered()
    rows = []
    for dt, name in ((torch.float64, "f64"), (torch.float32, "f32")):
        esz = 8 if dt == torch.float64 else 4
        p = fgt.plan(pr.delta, 6, dt)
        X, Y, A = (torch.from_numpy(v).to(dev, dt) for v in (pr.x, pr.y, pr.alpha))
        ws = fgt.workspace(p, pr.M, pr.N, dev)
        u = torch.empty(pr.M, dtype=dt, device=dev)
        fn = lambda: fgt.eval(X, Y, A, p, out=u, ws=ws)   # noqa: E731
        wall, med = timed(fn, args.steps, args.warmup, torch)
        fgt.profile_begin()
        for _ in range(args.steps):
            fn()
        phases, calls = fgt.profile_end()
        if fgt.last_device_status(ws) != fgt.FGT_OK:
            raise RuntimeError("device status after the clustered workload")
        P = pr.M + pr.N
        rows.append({"dtype": name, "digits": 6, "n_modes": p.n_modes,
                     "ms_per_transform": round(wall, 5), "ms_median_event": round(med, 5),
                     "value": P * p.n_modes / (wall * 1e-3), "unit": "point-modes/s",
                     "phase_ms": {k: round(v / calls, 5) for k, v in phases.items()},
                     "scan": scan_row(phases, calls, (esz + 4) * P + esz * (pr.N + pr.M))})
        del X, Y, A, ws, u
    return {"workload": ("N = 2^24 sources from a 64-component Gaussian mixture (centres U[0,1), "
                         "sigma log-uniform in [1e-5, 1e-2]), M = 2^22 targets U[0,1), "
                         "alpha ~ U(-1,1), delta = 1e-5"),
            "rows": rows}


def bench_diff(args, fgt, W, torch, np, dev):
    """M = N = 2^22, delta 1e-4: forward against forward + adjoint (all four gradients)."""
    rows = []
    for dt, name, digits in ((torch.float64, "f64", 9), (torch.float32, "f32", 4)):
        pr, g = W.grad_problem(22, 1e-4, digits)
        p = fgt.plan(pr.delta, digits, dt)
        X, Y, A, G = (torch.from_numpy(v).to(dev, dt) for v in (pr.x, pr.y, pr.alpha, g))
        ws = fgt.workspace(p, pr.M, pr.N, dev)
        u = torch.empty(pr.M, dtype=dt, device=dev)

        def fwd():
            fgt.eval(X, Y, A, p, out=u, ws=ws)

        def fwd_bwd():
            fgt.eval(X, Y, A, p, out=u, ws=ws)
            fgt.backward(X, Y, A, G, p, ws=ws, sorted=True)

        wf, mf = timed(fwd, args.steps, args.warmup, torch)
        wb, mb = timed(fwd_bwd, args.steps, args.warmup, torch)
        if fgt.last_device_status(ws) != fgt.FGT_OK:
            raise RuntimeError("device status after the differentiation workload")
        P = pr.M + pr.N
        rows.append({"dtype": name, "digits": digits, "n_modes": p.n_modes,
                     "fwd_ms": round(wf, 5), "fwd_ms_median_event": round(mf, 5),
                     "fwd_bwd_ms": round(wb, 5), "fwd_bwd_ms_median_event": round(mb, 5),
                     "ratio": round(wb / wf, 4),
                     "fwd_value": P * p.n_modes / (wf * 1e-3),
                     "fwd_bwd_value": P * p.n_modes / (wb * 1e-3), "unit": "point-modes/s"})
    return {"workload": ("M = N = 2^22 uniform on [0,1), alpha, g ~ N(0,1), delta = 1e-4, "
                         "L = g . u; backward = dL/dalpha, dL/dx, dL/dy, dL/ddelta"),
            "rows": rows}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (requested --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the transform is not sharded across GPUs in this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1909_09825_amd as fgt
    from paper_1909_09825_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dtype = torch.float32 if args.fp32 else torch.float64
    pr = W.large_plain(args.delta, args.digits, args.log2n)
    M, N = pr.M, pr.N
    P = M + N
    dev = torch.device("cuda:0")
    X = torch.from_numpy(pr.x).to(dev, dtype)
    Y = torch.from_numpy(pr.y).to(dev, dtype)
    A = torch.from_numpy(pr.alpha).to(dev, dtype)
    p = fgt.plan(args.delta, args.digits, dtype)
    ws = fgt.workspace(p, M, N, dev)
    u = torch.empty(M, dtype=dtype, device=dev)

    def step():
        fgt.eval(X, Y, A, p, out=u, ws=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    status = fgt.last_device_status(ws)
    if status != fgt.FGT_OK:
        raise RuntimeError(f"device status {status} after warmup")
    # An untimed profiled session first: the library then reuses its events and
    # creates none while the timed calls are enqueued.
    fgt.profile_begin()
    for _ in range(args.steps):
        step()
    fgt.profile_end()

    # Timed region: K steps bracketed by synchronisation, with per-step HIP
    # events on the current stream; the library records no events of its own.
    ms_step, ms_med = timed(step, args.steps, 0, torch)
    # Kernel times: K more steps right after, with the library's phase events on
    # its stream.  Each phase boundary costs a few microseconds, so these steps
    # are kept out of `value`.
    fgt.profile_begin()
    ms_prof, _ = timed(step, args.steps, 0, torch)
    phases, calls = fgt.profile_end()

    if args.copy_bytes > 0:
        src = torch.empty(args.copy_bytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    esz = 4 if args.fp32 else 8
    n_modes = p.n_modes
    per_step = {k: v / calls for k, v in phases.items()}
    radix = {k: v for k, v in per_step.items() if k.startswith("radix")}
    # Passes whose digit is constant or below the key resolution return at once;
    # only the data-moving launches count as launches of the sort kernel.
    longest = max(radix.values()) if radix else 0.0
    moving = [k for k, v in radix.items() if v > 0.05 * longest]
    n_run = len(moving)
    groups = {
        "k_onesweep": sum(radix[k] for k in moving),
        "k_final": per_step.get("tiles_final", 0.0),
        "k_reduce": per_step.get("tiles_reduce", 0.0),
        "setup": per_step.get("setup", 0.0),
        "k_carry": per_step.get("carry", 0.0),
    }
    dominant = max(groups, key=groups.get)
    # Algorithmic bytes per launch.  First pass: read the coordinate, write key
    # and index; middle passes: read and write key and index; last pass: read
    # key and index, write coordinate and index.  The tile reduce reads the
    # coordinates and merged ids, gathers alpha for the sources and writes the
    # sorted strengths; the final kernel reads coordinates, strengths and ids
    # and scatters u.
    first = P * (esz + esz + 4)
    middle = P * 2 * (esz + 4)
    if n_run <= 1:
        sort_bytes = P * (2 * esz + 4)
    else:
        sort_bytes = (first + (n_run - 1) * middle) / n_run
    alg = {
        "k_onesweep": sort_bytes,
        "k_final": P * (2 * esz + 4) + M * esz,
        "k_reduce": P * (esz + 4) + N * esz + P * esz,
    }
    launches = {"k_onesweep": max(n_run, 1), "k_final": 1, "k_reduce": 1}
    counter_name = {"k_onesweep": "k_onesweep", "k_final": "k_wfinal_fast", "k_reduce": "k_wreduce"}

    def roof(kernel):
        ms_launch = groups[kernel] / launches[kernel]
        gbs = alg[kernel] / (ms_launch * 1e-3) / 1e9
        return gbs, ms_launch

    dom = dominant if dominant in alg else "k_onesweep"
    gbs, ms_launch = roof(dom)
    traffic = traffic_for(counter_name[dom])
    kernels = {}
    for k in ("k_onesweep", "k_reduce", "k_final"):
        g, ms = roof(k)
        kernels[k] = {"ms_per_launch": round(ms, 5), "launches_per_step": launches[k],
                      "alg_bytes_per_launch": int(alg[k]), "GBps": round(g, 1),
                      "hbm_frac": round(g / HBM_PEAK_GBS, 4),
                      "valu_frac": valu_frac(counter_name[k], ms) if not args.fp32 else None,
                      "fp64_frac": fp64_frac(counter_name[k], ms) if not args.fp32 else None}
    out = {
        "metric": METRIC,
        "value": P * n_modes / (ms_step * 1e-3),
        "unit": "point-modes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "ms_median_event": round(ms_med, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.fp32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"plain FGT, M = N = 2^{args.log2n} uniform on [0,1), alpha ~ N(0,1), "
                         f"delta = {args.delta:g}, {args.digits} digits ({n_modes} modes), forward"),
            "M": M, "N": N, "delta": args.delta, "digits": args.digits, "n_modes": n_modes,
            "transforms_per_s": 1e3 / ms_step,
            "ms_per_step_with_phase_events": round(ms_prof, 5),
            "phase_ms_per_step": {k: round(v, 5) for k, v in per_step.items()},
            "kernels": kernels,
            # one pass over the sorted points: coordinates and ids read once,
            # alpha read once, u written once
            "scan": scan_row(phases, calls, P * (esz + 4) + N * esz + M * esz),
        },
        "roofline": {
            "kernel": dom,
            "ms_per_launch": round(ms_launch, 5),
            "bound": "hbm",
            "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
    }
    if not args.no_grad:
        G = torch.from_numpy(np.random.default_rng(5).standard_normal(M)).to(dev, dtype)

        def fwd_bwd():
            fgt.eval(X, Y, A, p, out=u, ws=ws)
            fgt.backward(X, Y, A, G, p, ws=ws, sorted=True)

        ms_fb, med_fb = timed(fwd_bwd, args.steps, args.warmup, torch)
        out["fwd_bwd"] = {
            "ms_per_step": round(ms_fb, 5),
            "ms_median_event": round(med_fb, 5),
            "value": P * n_modes / (ms_fb * 1e-3),
            "unit": "point-modes/s",
            "ratio_to_fwd": round(ms_fb / ms_step, 4),
            "step": "fgt_eval + fgt_backward(FGT_SORTED) giving dL/dalpha, dL/dx, dL/dy, dL/ddelta",
        }
    # plan reuse: new strengths on the sorted points
    A2 = torch.from_numpy(np.random.default_rng(6).standard_normal(N)).to(dev, dtype)
    step()
    ms_reuse, med_reuse = timed(lambda: fgt.eval_sorted(A2, p, ws, M, out=u), args.steps,
                                args.warmup, torch)
    out["plan_reuse"] = {"ms_per_step": round(ms_reuse, 5), "ms_median_event": round(med_reuse, 5),
                         "value": P * n_modes / (ms_reuse * 1e-3), "unit": "point-modes/s",
                         "step": "fgt_eval_sorted: strengths gathered into the kept sort, then the scans"}
    if fgt.last_device_status(ws) != fgt.FGT_OK:
        raise RuntimeError("device status after the headline workload")
    del ws
    if not args.no_small and not args.fp32:
        out["small"] = bench_small(args, fgt, W, torch, np, dev)
    if not args.no_clustered and not args.fp32:
        out["clustered"] = bench_clustered(args, fgt, W, torch, np, dev)
    if not args.no_diff and not args.fp32:
        out["differentiation"] = bench_diff(args, fgt, W, torch, np, dev)
    if not args.no_identical and not args.fp32:
        out["identical_points"] = bench_identical(args, fgt, W, torch, np, dev)
    if not args.no_batched and not args.fp32:
        out["batched"] = bench_batched(args, fgt, W, torch, np, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pr.x, pr.y, pr.alpha, args.delta, args.digits, n_modes,
                                           min(args.cpu_sample_log2n, args.log2n))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
