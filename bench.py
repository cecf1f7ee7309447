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
`roofline` describes
the kernel with the largest share of the step, timed with HIP events recorded
by the library on its own stream during the timed steps; `cpu_baseline` is
the CPU oracle's SOE recurrence timed on a bounded sample of the same inputs.

    python bench.py [--steps K] [--warmup W] [--delta D] [--digits G] [--log2n L]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X FP64 vector
METRIC = "(M+N)·modes/s and transforms/s at 6 digits, fwd vs fwd+bwd, % HBM roofline"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")


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
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one plain device copy of this many bytes (counter calibration)")
    return ap.parse_args()


def traffic_for(kernel: str):
    """HBM bytes per launch from committed counter runs, if the kernel source is unchanged."""
    from paper_1909_09825_amd.profiling import source_hash
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != source_hash(rec["sources"]):
        return None
    return int(rec["bytes_per_launch"])


def cpu_baseline(x, y, a, delta, digits, n_modes, k):
    """The CPU oracle's SOE recurrence (sort + per-mode sweeps) on the first 2^k points."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle
    from conftest import load_oracle_tables
    t = load_oracle_tables()[n_modes]
    n = 1 << k
    xs, ys, as_ = x[:n].copy(), y[:n].copy(), a[:n].copy()
    t0 = time.perf_counter()
    oracle.soe_recurrence(xs, ys, as_, delta, t["tau0"], t["omega"])
    dt = time.perf_counter() - t0
    threads = oracle.max_threads()
    return {
        "value": (2 * n) * n_modes / dt, "unit": "point-modes/s",
        "cores": int(min(threads, 2 * n_modes)), "kind": "oracle",
        "sample": (f"first 2^{k} targets and 2^{k} sources of the same inputs, {digits} digits "
                   f"({n_modes} modes): O2 SOE recurrence in C (qsort, then one sweep per mode and "
                   f"direction, OpenMP over the {2 * n_modes} sweeps), {dt:.2f} s wall"),
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
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fgt.eval_batch(X, Y, A, bp, out=U, ws=ws)
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / args.steps
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
    return {
        "workload": (f"{B} transforms, N_b and M_b log-uniform in [256, 65536], delta_b "
                     f"log-uniform in [1e-6, 1e-2], points uniform on [0,1), alpha [N][{R}] ~ N(0,1), "
                     f"{bt.digits} digits ({bp.n_modes} modes), FP64"),
        "total_points": bp.total_points,
        "ms_per_batch_eager": round(ms_eager, 4),
        "ms_per_batch_graph": round(ms_graph, 4),
        "transforms_per_s": B / (ms * 1e-3),
        "column_transforms_per_s": B * R / (ms * 1e-3),
        "value": bp.total_points * bp.n_modes * R / (ms * 1e-3),
        "unit": "point-mode-columns/s",
        "loop_of_fgt_eval_ms": round(ms_loop, 2),
        "loop_sample": (f"fgt_eval once per column on 32 sampled transforms ({pts32} points), "
                        f"{ms_loop32:.1f} ms, scaled by total points"),
        "speedup_vs_loop": round(ms_loop / ms, 1),
        "tuned_config": {"points_per_lane": config[0], "bucket_points": config[1],
                         "tuning_s": round(tune_s, 2)},
    }


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

    for _ in range(args.warmup):
        fgt.eval(X, Y, A, p, out=u, ws=ws)
    torch.cuda.synchronize()
    status = fgt.last_device_status(ws)
    if status != fgt.FGT_OK:
        raise RuntimeError(f"device status {status} after warmup")

    fgt.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fgt.eval(X, Y, A, p, out=u, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases, calls = fgt.profile_end()
    ms_step = (t1 - t0) * 1e3 / args.steps

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
    # key and index, gather alpha for the sources, write key, strength, slot.
    first = P * (esz + esz + 4)
    middle = P * 2 * (esz + 4)
    last = P * (esz + 4) + N * esz + P * (2 * esz + 4)
    if n_run <= 1:
        sort_bytes = P * esz + N * esz + P * (2 * esz + 4)
    else:
        sort_bytes = (first + (n_run - 2) * middle + last) / n_run
    scan_read = P * (2 * esz)                        # keys and strengths
    alg = {
        "k_onesweep": sort_bytes,
        "k_final": scan_read + P * 4 + M * esz,      # + slots, + u scattered
        "k_reduce": scan_read,
    }
    launches = {"k_onesweep": max(n_run, 1), "k_final": 1, "k_reduce": 1}

    def roof(kernel):
        ms_launch = groups[kernel] / launches[kernel]
        gbs = alg[kernel] / (ms_launch * 1e-3) / 1e9
        return gbs, ms_launch

    dom = dominant if dominant in alg else "k_onesweep"
    gbs, ms_launch = roof(dom)
    traffic = traffic_for(dom)
    kernels = {}
    for k in ("k_onesweep", "k_reduce", "k_final"):
        g, ms = roof(k)
        kernels[k] = {"ms_per_launch": round(ms, 5), "launches_per_step": launches[k],
                      "alg_bytes_per_launch": int(alg[k]), "GBps": round(g, 1),
                      "hbm_frac": round(g / HBM_PEAK_GBS, 4)}
    out = {
        "metric": METRIC,
        "value": P * n_modes / (ms_step * 1e-3),
        "unit": "point-modes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
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
            "phase_ms_per_step": {k: round(v, 5) for k, v in per_step.items()},
            "kernels": kernels,
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
        for _ in range(args.warmup):
            fgt.eval(X, Y, A, p, out=u, ws=ws)
            fgt.backward(X, Y, A, G, p, ws=ws, sorted=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fgt.eval(X, Y, A, p, out=u, ws=ws)
            fgt.backward(X, Y, A, G, p, ws=ws, sorted=True)
        torch.cuda.synchronize()
        ms_fb = (time.perf_counter() - t0) * 1e3 / args.steps
        out["fwd_bwd"] = {
            "ms_per_step": round(ms_fb, 5),
            "value": P * n_modes / (ms_fb * 1e-3),
            "unit": "point-modes/s",
            "ratio_to_fwd": round(ms_fb / ms_step, 4),
            "step": "fgt_eval + fgt_backward(FGT_SORTED) giving dL/dalpha, dL/dx, dL/dy, dL/ddelta",
        }
    # plan reuse: new strengths on the sorted points
    A2 = torch.from_numpy(np.random.default_rng(6).standard_normal(N)).to(dev, dtype)
    fgt.eval(X, Y, A, p, out=u, ws=ws)
    for _ in range(args.warmup):
        fgt.eval_sorted(A2, p, ws, M, out=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fgt.eval_sorted(A2, p, ws, M, out=u)
    torch.cuda.synchronize()
    ms_reuse = (time.perf_counter() - t0) * 1e3 / args.steps
    out["plan_reuse"] = {"ms_per_step": round(ms_reuse, 5),
                         "value": P * n_modes / (ms_reuse * 1e-3), "unit": "point-modes/s",
                         "step": "fgt_eval_sorted: strengths gathered into the kept sort, then the scans"}
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
