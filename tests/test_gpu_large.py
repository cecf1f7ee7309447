"""Parity at full size, in the launch configuration bench.py times.

* M = N = 2^24 uniform points, alpha ~ N(0,1), delta in {1e-2, 1e-4, 1e-6},
  3 / 6 / 9 digits: O1 (direct Gaussian sum) on sampled targets, within
  2 E_n sum|alpha|; O2 (the oracle's SOE recurrence) on every target for
  6 digits.
* 2^24 sources from a 64-component Gaussian mixture, 2^22 uniform targets,
  alpha ~ U(-1,1), delta = 1e-5: FP64 at 3 / 6 / 9 digits (O1 on sampled
  targets plus the targets inside the 8 narrowest clusters; O2 at 6 digits),
  FP32 at 3 / 6 digits with the error stated against O1 on the FP32-rounded
  inputs.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1909_09825_amd as fgt
from paper_1909_09825_amd import workloads as W
from fgt_testlib import (EPS32, check_direct, gpu_eval, impl_tol, oracle_E, oracle_sum_omega,
                         oracle_table, say)

pytestmark = pytest.mark.gpu

# Sampled targets per delta: the direct sum costs (targets) x (sources within
# 16.6 sqrt(delta)); these keep each check to a few seconds on the host.
SAMPLES = {1e-2: 384, 1e-4: 2048, 1e-6: 4096}

_cache = {}


def large(delta):
    if delta not in _cache:
        _cache.clear()
        _cache[delta] = W.large_plain(delta, 6)
    return _cache[delta]


@pytest.mark.parametrize("digits", [3, 6, 9])
@pytest.mark.parametrize("delta", [1e-2, 1e-4, 1e-6])
def test_large_uniform(delta, digits):
    pr = large(delta)
    u, p, st = gpu_eval(pr.x, pr.y, pr.alpha, delta, digits, case="large")
    assert st == fgt.FGT_OK
    idx = W.sample_indices(pr.M, SAMPLES[delta], cfg=2, sub=int(digits))
    e1, _ = check_direct(u[idx], pr.x[idx], pr.y, pr.alpha, delta, p)
    assert e1 <= 2 * oracle_E(p)
    if digits == 6:
        t = oracle_table(p)
        u2 = oracle.soe_recurrence(pr.x, pr.y, pr.alpha, delta, t["tau0"], t["omega"])
        e2 = float(np.max(np.abs(u - u2)))
        tol = impl_tol(pr.alpha, p, pr.M + pr.N)
        say(f"   O2 check (all {pr.M} targets): {e2:.3e} (tol {tol:.3e})")
        assert e2 <= tol


_ccache = {}


def clustered():
    if "p" not in _ccache:
        _ccache["p"] = W.clustered()
    return _ccache["p"]


def cluster_targets(pr, k=8):
    """Targets within 10 sigma of the k narrowest cluster centres."""
    centers, sig = W.clustered_meta()
    order = np.argsort(sig)[:k]
    sel = np.zeros(pr.M, bool)
    for m in order:
        sel |= np.abs(pr.x - centers[m]) <= 10 * sig[m]
    return np.nonzero(sel)[0]


@pytest.mark.parametrize("digits", [3, 6, 9])
def test_clustered_fp64(digits):
    pr = clustered()
    u, p, st = gpu_eval(pr.x, pr.y, pr.alpha, pr.delta, digits, case="clustered")
    assert st == fgt.FGT_OK
    idx = np.union1d(W.sample_indices(pr.M, 2048, cfg=3, sub=digits), cluster_targets(pr))
    e1, _ = check_direct(u[idx], pr.x[idx], pr.y, pr.alpha, pr.delta, p)
    assert e1 <= 2 * oracle_E(p)
    if digits == 6:
        t = oracle_table(p)
        u2 = oracle.soe_recurrence(pr.x, pr.y, pr.alpha, pr.delta, t["tau0"], t["omega"])
        e2 = float(np.max(np.abs(u - u2)))
        tol = impl_tol(pr.alpha, p, pr.M + pr.N)
        say(f"   O2 check (all {pr.M} targets): {e2:.3e} (tol {tol:.3e})")
        assert e2 <= tol


@pytest.mark.parametrize("digits", [3, 6])
def test_clustered_fp32(digits):
    """FP32 inputs and arithmetic; the error is stated against O1 evaluated on
    the same FP32-rounded inputs (cast exactly to FP64), and bounded by
    E_n + 64 eps32 sum|omega| relative to sum|alpha|."""
    pr = clustered()
    x32, y32, a32 = pr.x.astype(np.float32), pr.y.astype(np.float32), pr.alpha.astype(np.float32)
    u, p, st = gpu_eval(x32, y32, a32, pr.delta, digits, dtype=torch.float32, case="clustered-fp32")
    assert st == fgt.FGT_OK
    idx = np.union1d(W.sample_indices(pr.M, 2048, cfg=3, sub=10 + digits), cluster_targets(pr))
    ref = oracle.direct(x32[idx].astype(np.float64), y32.astype(np.float64),
                        a32.astype(np.float64), pr.delta)
    s_alpha = float(np.sum(np.abs(a32.astype(np.float64))))
    err = float(np.max(np.abs(u[idx] - ref))) / s_alpha
    ref64 = oracle.direct(pr.x[idx], pr.y, pr.alpha, pr.delta)
    err64 = float(np.max(np.abs(u[idx] - ref64))) / float(np.sum(np.abs(pr.alpha)))
    bound = oracle_E(p) + 64 * EPS32 * oracle_sum_omega(p)
    say(f"   FP32 error / sum|alpha| = {err:.3e} vs rounded inputs, {err64:.3e} vs FP64 inputs "
        f"(E = {oracle_E(p):.2e}, bound {bound:.2e})")
    assert err <= bound


def test_plan_reuse_full_size():
    """fgt_eval_sorted (the sort kept, new strengths) at 2^24 + 2^24, delta 1e-4,
    6 digits -- the launch the benchmark's plan-reuse line times -- against O1 on
    sampled targets and O2 on every target, for strengths the sort never saw."""
    pr = large(1e-4)
    p = fgt.plan(1e-4, 6)
    X, Y, A = (torch.from_numpy(v).to("cuda") for v in (pr.x, pr.y, pr.alpha))
    ws = fgt.workspace(p, pr.M, pr.N, X.device)
    say("[gpu] fgt_eval then fgt_eval_sorted with new alpha, 2^24 + 2^24")
    fgt.eval(X, Y, A, p, ws=ws)
    a2 = W.rng(2, 50).standard_normal(pr.N)
    u = fgt.eval_sorted(torch.from_numpy(a2).to("cuda"), p, ws, pr.M).cpu().numpy()
    assert fgt.last_device_status(ws) == fgt.FGT_OK
    idx = W.sample_indices(pr.M, 2048, cfg=2, sub=50)
    e1, _ = check_direct(u[idx], pr.x[idx], pr.y, a2, 1e-4, p)
    assert e1 <= 2 * oracle_E(p)
    t = oracle_table(p)
    u2 = oracle.soe_recurrence(pr.x, pr.y, a2, 1e-4, t["tau0"], t["omega"])
    e2 = float(np.max(np.abs(u - u2)))
    tol = impl_tol(a2, p, pr.M + pr.N)
    say(f"   O2 check (all {pr.M} targets): {e2:.3e} (tol {tol:.3e})")
    assert e2 <= tol
