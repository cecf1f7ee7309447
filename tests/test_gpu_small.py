"""The small-transform path that fgt_eval takes for P = M + N <= 4096.

One workgroup per mode sorts (bitonic, exact, stable in the merged order) and
scans; a second launch adds the modes and scatters; the first workgroup leaves
the sorted state in the workspace.  Checked here:
  * O1 (direct sum) within 2 E_n sum|alpha| and O2 (the oracle's SOE recurrence)
    within the rounding tolerance, over shapes at and around the size limit and
    the power-of-two padding (P = 1, 2, 3, 2047, 2048, 4095, 4096, 4097), ties
    between sources and targets, duplicates, -0 beside +0, negative coordinates,
    FP32;
  * non-finite coordinates reported;
  * the sorted state it leaves: fgt_eval_sorted with new strengths and
    fgt_backward(FGT_SORTED) after it, against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1909_09825_amd as fgt
from paper_1909_09825_amd import workloads as W
from fgt_testlib import (EPS32, check_direct, gpu_eval, impl_tol, oracle_E, oracle_sum_omega,
                         oracle_table, say, to_dev)

pytestmark = pytest.mark.gpu


def parity(x, y, a, delta, digits, case, dtype=torch.float64):
    u, p, st = gpu_eval(x, y, a, delta, digits, dtype=dtype, case=case)
    assert st == fgt.FGT_OK
    if dtype == torch.float32:   # the oracle runs on the FP32-rounded inputs
        x, y, a = (np.asarray(v, np.float32).astype(np.float64) for v in (x, y, a))
    t = oracle_table(p)
    u2 = oracle.soe_recurrence(x, y, a, delta, t["tau0"], t["omega"])
    eps = EPS32 if dtype == torch.float32 else 2.0 ** -53
    tol = impl_tol(a, p, len(x) + len(y), eps)
    e2 = float(np.max(np.abs(u - u2))) if len(u) else 0.0
    say(f"   O2: {e2:.3e} (tol {tol:.3e})")
    assert e2 <= tol
    e1, _ = check_direct(u, x, y, a, delta, p)
    assert e1 <= 2 * oracle_E(p) + (64 * EPS32 * oracle_sum_omega(p) if dtype == torch.float32 else 0)
    return u, p


@pytest.mark.parametrize("M,N", [(1, 1), (1, 2), (2, 1), (2, 3), (1000, 1000), (1, 2046),
                                 (1024, 1024), (2047, 2048), (2048, 2048), (4095, 1), (1, 4095),
                                 (2048, 2049)])
def test_small_shapes(M, N):
    pr = W.plain(M, N, 1e-3, 6, cfg=13, sub=(M * 7 + N) % 1009)
    parity(pr.x, pr.y, pr.alpha, 1e-3, 6, f"small {M}x{N}")


@pytest.mark.parametrize("delta,digits", [(1e-6, 3), (1e-4, 9), (1.0, 6), (10.0, 9)])
def test_small_settings(delta, digits):
    g = np.random.default_rng(31 + digits)
    x, y = g.uniform(-0.5, 1.5, 1500), g.uniform(-0.5, 1.5, 2500)
    a = g.standard_normal(2500)
    parity(x, y, a, delta, digits, f"settings {delta:g}/{digits}")


def test_small_ties_duplicates_signed_zero():
    g = np.random.default_rng(32)
    grid = lambda n: np.round(g.uniform(-1, 1, n) * 30) / 30   # noqa: E731 - many exact ties
    x, y = grid(1700), grid(2300)
    x[::9] = -0.0
    y[::7] = 0.0
    y[1::11] = -0.0
    a = g.standard_normal(2300)
    parity(x, y, a, 1e-2, 6, "ties")


@pytest.mark.parametrize("digits", [3, 6])
def test_small_fp32(digits):
    g = np.random.default_rng(33)
    x, y = g.random(2000), g.random(2000)
    a = g.standard_normal(2000)
    parity(x, y, a, 1e-3, digits, f"fp32 {digits}", dtype=torch.float32)


def test_small_nonfinite_is_reported():
    g = np.random.default_rng(34)
    x, y = g.random(500), g.random(600)
    x[5] = np.nan
    _, _, st = gpu_eval(x, y, np.ones(600), 1e-3, 6, case="small nan")
    assert st == fgt.FGT_ENONFINITE
    x[5] = 0.5
    y[7] = -np.inf
    _, _, st = gpu_eval(x, y, np.ones(600), 1e-3, 6, case="small inf")
    assert st == fgt.FGT_ENONFINITE
    y[7] = 0.25
    _, _, st = gpu_eval(x, y, np.ones(600), 1e-3, 6, case="small finite again")
    assert st == fgt.FGT_OK


def test_small_sorted_state_serves_reuse_and_backward():
    """After a small fgt_eval, the workspace holds the sorted state: new strengths
    through fgt_eval_sorted, and the gradients with FGT_SORTED, match the oracle."""
    g = np.random.default_rng(35)
    M, N, delta = 1800, 2200, 1e-3
    x, y = g.random(M), g.random(N)
    a, a2, gt = g.standard_normal(N), g.standard_normal(N), g.standard_normal(M)
    say(f"[gpu] small eval, then eval_sorted and backward(sorted), M={M} N={N}")
    p = fgt.plan(delta, 6)
    X, Y, A, A2, G = (to_dev(v, torch.float64) for v in (x, y, a, a2, gt))
    ws = fgt.workspace(p, M, N, X.device)
    fgt.eval(X, Y, A, p, ws=ws)
    u2 = fgt.eval_sorted(A2, p, ws, M).cpu().numpy()
    assert fgt.last_device_status(ws) == fgt.FGT_OK
    t = oracle_table(p)
    ref = oracle.soe_recurrence(x, y, a2, delta, t["tau0"], t["omega"])
    assert float(np.max(np.abs(u2 - ref))) <= impl_tol(a2, p, M + N)
    fgt.eval(X, Y, A, p, ws=ws)
    da, dx, dy, dd = fgt.backward(X, Y, A, G, p, ws=ws, sorted=True)
    db, ex, ey, de = fgt.backward(X, Y, A, G, p, sorted=False)
    assert fgt.last_device_status(ws) == fgt.FGT_OK
    # same sorted order up to the multi-kernel sort's resolution: equal to rounding
    for s_, f_, w in ((da, db, gt), (dx, ex, None), (dy, ey, None)):
        s_, f_ = s_.cpu().numpy(), f_.cpu().numpy()
        scale = float(np.max(np.abs(f_))) + 1e-300
        assert float(np.max(np.abs(s_ - f_))) <= 1e-10 * scale
    o_da, _, _, _ = oracle.direct_gradients(x, y, a, gt, delta)
    assert float(np.max(np.abs(da.cpu().numpy() - o_da))) <= (
        2 * oracle_E(p) * float(np.abs(gt).sum()) + impl_tol(gt, p, M + N))
    assert abs(float(dd.item()) - float(de.item())) <= 1e-9 * abs(float(de.item())) + 1e-12
