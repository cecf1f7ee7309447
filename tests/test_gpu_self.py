"""Targets identical to the sources (fgt_eval_self), Section 5's first case.

Checked against O1 (direct sum over the same points, self term included)
within 2 E_n sum|alpha| and against O2 with x = y (ties counted once, in h+)
within the rounding tolerance; Chebyshev points in order with the sort
skipped; the device check of the order; agreement with fgt_eval(x, x).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1909_09825_amd as fgt
from paper_1909_09825_amd import workloads as W
from fgt_testlib import EPS32, impl_tol, oracle_E, oracle_table, say, to_dev

pytestmark = pytest.mark.gpu


def run_self(x, a, delta, digits, presorted=False, dtype=torch.float64, case=""):
    say(f"[gpu] fgt_eval_self {case} N={len(x)} delta={delta:g} digits={digits} presorted={presorted}")
    p = fgt.plan(delta, digits, dtype)
    X, A = to_dev(x, dtype), to_dev(a, dtype)
    ws = fgt.workspace(p, 0, len(x), X.device)
    u = fgt.eval_self(X, A, p, presorted=presorted, ws=ws)
    st = fgt.last_device_status(ws)
    return u.double().cpu().numpy(), p, st


@pytest.mark.parametrize("digits", [3, 6, 9])
@pytest.mark.parametrize("delta", [1e-5, 1e-3, 1.0])
def test_self_uniform(delta, digits):
    g = np.random.default_rng(300 + digits)
    N = 20011
    x, a = g.random(N), g.standard_normal(N)
    u, p, st = run_self(x, a, delta, digits, case="uniform")
    assert st == fgt.FGT_OK
    ref = oracle.direct(x, x, a, delta)
    e1 = np.max(np.abs(u - ref)) / np.abs(a).sum()
    t = oracle_table(p)
    ref2 = oracle.soe_recurrence(x, x, a, delta, t["tau0"], t["omega"])
    e2 = np.max(np.abs(u - ref2))
    tol = impl_tol(a, p, N)
    say(f"   O1 err / sum|alpha| = {e1:.3e} (2E = {2 * oracle_E(p):.3e}); O2 err {e2:.3e} (tol {tol:.3e})")
    assert e1 <= 2 * oracle_E(p) and e2 <= tol


def test_self_matches_general_path():
    g = np.random.default_rng(310)
    N = 30000
    x, a = g.random(N), g.standard_normal(N)
    u, p, _ = run_self(x, a, 1e-4, 6, case="vs eval(x, x)")
    X, A = to_dev(x, torch.float64), to_dev(a, torch.float64)
    ref = fgt.eval(X, X, A, p).cpu().numpy()
    assert np.max(np.abs(u - ref)) <= impl_tol(a, p, 2 * N)


@pytest.mark.parametrize("N", [1, 2047, 65536, 100003])
def test_self_chebyshev_presorted(N):
    x = W.chebyshev(N)
    a = np.random.default_rng(320).standard_normal(N)
    u1, p, st1 = run_self(x, a, 1e-4, 6, presorted=True, case="chebyshev")
    u2, _, st2 = run_self(x, a, 1e-4, 6, presorted=False, case="chebyshev sorted anyway")
    assert st1 == fgt.FGT_OK and st2 == fgt.FGT_OK
    np.testing.assert_array_equal(u1, u2)
    ref = oracle.direct(x, x, a, 1e-4)
    assert np.max(np.abs(u1 - ref)) / np.abs(a).sum() <= 2 * oracle_E(p)


def test_self_presorted_flag_checks_order():
    x = W.chebyshev(5000)[::-1].copy()
    a = np.ones(5000)
    _, _, st = run_self(x, a, 1e-3, 6, presorted=True, case="descending")
    assert st == fgt.FGT_EUNSORTED


def test_self_fp32_and_ties():
    g = np.random.default_rng(330)
    N = 40000
    x = np.round(g.random(N) * 1000) / 1000          # many coincident points
    a = g.standard_normal(N)
    x32 = x.astype(np.float32).astype(np.float64)
    a32 = a.astype(np.float32).astype(np.float64)
    u, p, st = run_self(x32, a32, 1e-4, 5, dtype=torch.float32, case="fp32 ties")
    assert st == fgt.FGT_OK
    ref = oracle.direct(x32, x32, a32, 1e-4)
    err = np.max(np.abs(u - ref)) / np.abs(a32).sum()
    say(f"   fp32 err / sum|alpha| = {err:.3e} (E = {oracle_E(p):.3e})")
    assert err <= 2 * oracle_E(p) + impl_tol(a32, p, N, EPS32) / np.abs(a32).sum()


def test_self_empty():
    say("[gpu] fgt_eval_self N = 0")
    p = fgt.plan(1e-3, 6)
    x = torch.empty(0, dtype=torch.float64, device="cuda")
    u = fgt.eval_self(x, x, p)
    assert u.shape == (0,)


@pytest.mark.parametrize("delta,digits", [(1.0, 6), (1e-4, 6)])
def test_self_full_size(delta, digits):
    """N = 10^7 (the Table 1 size; 77 chunks of 64 scan tiles, so the carries
    cross chunks): O1 on sampled points, O2 on every point."""
    x, a = W.identical_uniform(10_000_000)
    u, p, st = run_self(x, a, delta, digits, case="10^7")
    assert st == fgt.FGT_OK
    idx = W.sample_indices(len(x), 256 if delta == 1.0 else 2048, cfg=6, sub=digits)
    ref = oracle.direct(x[idx], x, a, delta)
    e1 = float(np.max(np.abs(u[idx] - ref))) / float(np.abs(a).sum())
    t = oracle_table(p)
    ref2 = oracle.soe_recurrence(x, x, a, delta, t["tau0"], t["omega"])
    e2 = float(np.max(np.abs(u - ref2)))
    tol = impl_tol(a, p, len(x))
    say(f"   O1 err / sum|alpha| = {e1:.3e} (2E = {2 * oracle_E(p):.3e}); O2 err {e2:.3e} (tol {tol:.3e})")
    assert e1 <= 2 * oracle_E(p) and e2 <= tol
