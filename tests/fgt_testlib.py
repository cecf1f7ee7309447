"""Helpers shared by the GPU tests: run the HIP path, run the oracle, compare."""
import math
import sys
import time

import numpy as np
import torch

import oracle
import paper_1909_09825_amd as fgt
from conftest import load_oracle_tables

OTABLES = load_oracle_tables()
EPS64 = 2.0 ** -53
EPS32 = 2.0 ** -24


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def gpu_eval(x, y, alpha, delta, digits, dtype=torch.float64, case=""):
    """Run fgt_eval through the C ABI; returns (u as float64 numpy, plan, device status)."""
    say(f"[gpu] fgt_eval {case} M={len(x)} N={len(y)} delta={delta:g} digits={digits} {dtype}")
    p = fgt.plan(delta, digits, dtype)
    X, Y, A = to_dev(x, dtype), to_dev(y, dtype), to_dev(alpha, dtype)
    ws = fgt.workspace(p, len(x), len(y), X.device)
    u = fgt.eval(X, Y, A, p, ws=ws)
    status = fgt.last_device_status(ws)
    return u.double().cpu().numpy(), p, status


def oracle_table(p):
    """The oracle's own table with the plan's mode count."""
    return OTABLES[p.n_modes]


def oracle_E(p) -> float:
    """E_n of the oracle's table with the plan's mode count: the (3.1) measurement
    that every parity bar here uses (never the library's own stated bound)."""
    return float(OTABLES[p.n_modes]["E"])


def oracle_Eprime(p) -> float:
    """E'_n = sup |S' - G'| of the oracle's table (units of 1/sqrt(delta))."""
    return float(OTABLES[p.n_modes]["Eprime"])


def oracle_sum_omega(p) -> float:
    """sum_k |omega_k| of the oracle's table with the plan's mode count."""
    return float(np.sum(np.abs(OTABLES[p.n_modes]["omega"])))


def oracle_sum_dom(p) -> float:
    """sum_k |tau_k omega_k| (tau_k = tau0_k / sqrt(delta)) of the oracle's table."""
    t = OTABLES[p.n_modes]
    return float(np.sum(np.abs(t["tau0"] * t["omega"]))) / math.sqrt(p.delta)


def impl_tol(alpha, p, P, eps=EPS64):
    """Tolerance for GPU vs the oracle's SOE recurrence (same table, different
    summation order): each of the ~2 log2(P) levels of the scan and the
    sequential sweeps adds a few rounding errors of size eps |omega_k| |alpha|;
    the recurrences damp, never amplify (|e| <= 1).  On top, the library may
    leave points closer than its key resolution unordered, which it bounds by
    1e-6 E_n sum|alpha|."""
    s_alpha = float(np.sum(np.abs(alpha)))
    s_omega = oracle_sum_omega(p)
    return (64.0 * eps * s_alpha * s_omega * max(1.0, math.log2(max(P, 2)))
            + 1e-6 * oracle_E(p) * s_alpha)


def check_direct(u, x_sel, y, alpha, delta, p, factor=2.0):
    """|u - O1| <= factor * E_n * sum|alpha| at the selected targets."""
    t0 = time.time()
    ref = oracle.direct(x_sel, y, alpha, delta)
    s_alpha = float(np.sum(np.abs(alpha)))
    err = float(np.max(np.abs(u - ref))) / s_alpha if len(u) else 0.0
    say(f"   O1 check: max err / sum|alpha| = {err:.3e}  (bound {factor} E = {factor * oracle_E(p):.3e}, "
        f"{len(x_sel)} targets, {time.time() - t0:.1f}s)")
    return err, ref
