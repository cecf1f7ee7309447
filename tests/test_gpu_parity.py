"""Parity of the HIP path (through the C ABI) with the CPU oracle.

* O1 (direct Gaussian sum): |u - u_O1| <= 2 E_n sum|alpha|, the tolerance
  the transform is specified to meet (E_n = the plan's stated table error).
* O2 (the oracle's SOE recurrence with its own, independently built table of
  the same mode count): agreement to rounding, see fgt_testlib.impl_tol.
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


def full_check(x, y, a, delta, digits, case, direct=True):
    u, p, st = gpu_eval(x, y, a, delta, digits, case=case)
    assert st == fgt.FGT_OK
    t = oracle_table(p)
    u2 = oracle.soe_recurrence(x, y, a, delta, t["tau0"], t["omega"])
    e2 = float(np.max(np.abs(u - u2))) if len(u) else 0.0
    tol = impl_tol(a, p, len(x) + len(y))
    say(f"   O2 check: max |u - u_O2| = {e2:.3e} (tol {tol:.3e})")
    assert e2 <= tol
    if direct:
        e1, _ = check_direct(u, x, y, a, delta, p)
        assert e1 <= 2 * oracle_E(p)
    return u, p


def test_small_config():
    """1000 targets, 1000 sources uniform on [0,1), alpha ~ N(0,1), delta 1e-3, 6 digits."""
    pr = W.small_plain()
    full_check(pr.x, pr.y, pr.alpha, pr.delta, pr.digits, "small")


@pytest.mark.parametrize("digits", [3, 6, 9])
@pytest.mark.parametrize("delta", [1e-6, 1e-3, 1.0])
def test_ragged_multi_tile(delta, digits):
    """Several sort and scan tiles plus a ragged tail, M != N."""
    pr = W.plain(20011, 30007, delta, digits, cfg=10, sub=int(digits))
    full_check(pr.x, pr.y, pr.alpha, delta, digits, "ragged", direct=True)


@pytest.mark.parametrize("M,N", [(1, 1), (1, 4097), (4097, 1), (2048, 2048), (4096, 4096),
                                 (2047, 2050), (12288, 4096)])
def test_shapes(M, N):
    pr = W.plain(M, N, 1e-3, 6, cfg=11, sub=M % 97)
    full_check(pr.x, pr.y, pr.alpha, 1e-3, 6, f"shape{M}x{N}")


@pytest.mark.parametrize("dtype,off", [(torch.float64, 1), (torch.float32, 1), (torch.float32, 2),
                                       (torch.float32, 3)])
def test_misaligned_inputs(dtype, off):
    """Coordinates and strengths given as views that start off a 16-byte boundary
    (the setup kernels then take single loads instead of 16-byte ones): results
    bit-identical to the same values in aligned arrays."""
    pr = W.plain(30001, 20003, 1e-4, 6, cfg=12, sub=off)
    say(f"[gpu] misaligned views, {dtype}, offset {off} elements")
    p = fgt.plan(1e-4, 6, dtype)
    dev = torch.device("cuda")
    def view(v):
        buf = torch.zeros(len(v) + off, dtype=dtype, device=dev)
        buf[off:] = torch.from_numpy(v).to(dev, dtype)
        return buf[off:]
    X, Y, A = view(pr.x), view(pr.y), view(pr.alpha)
    assert X.data_ptr() % 16 != 0 and Y.data_ptr() % 16 != 0
    u1 = fgt.eval(X, Y, A, p)
    u0 = fgt.eval(X.clone(), Y.clone(), A.clone(), p)
    assert torch.equal(u0.view(torch.int64 if dtype == torch.float64 else torch.int32),
                       u1.view(torch.int64 if dtype == torch.float64 else torch.int32))


def test_no_sources_gives_zero():
    say("[gpu] N = 0")
    p = fgt.plan(1e-3, 6)
    x = torch.rand(100, dtype=torch.float64, device="cuda")
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    u = fgt.eval(x, e, e, p, out=torch.full((100,), 7.0, dtype=torch.float64, device="cuda"))
    assert torch.all(u == 0)


def test_no_targets():
    say("[gpu] M = 0")
    p = fgt.plan(1e-3, 6)
    y = torch.rand(100, dtype=torch.float64, device="cuda")
    u = fgt.eval(torch.empty(0, dtype=torch.float64, device="cuda"), y, y, p)
    assert u.numel() == 0


def test_all_coordinates_equal():
    x = np.full(3000, 0.25)
    y = np.full(5000, 0.25)
    a = np.random.default_rng(1).standard_normal(5000)
    u, p = full_check(x, y, a, 1e-2, 6, "all-equal")
    s0 = float(np.sum(oracle_table(p)["omega"]).real)
    np.testing.assert_allclose(u, s0 * np.sum(a), rtol=0, atol=1e-12 * np.sum(np.abs(a)))


def test_ties_duplicates_negative_and_signed_zero():
    g = np.random.default_rng(2)
    grid = np.arange(-300, 301) / 256.0
    y = np.concatenate([g.choice(grid, 9000), [0.0, -0.0, 0.0]])
    x = np.concatenate([g.choice(y, 4000), g.choice(grid, 3000), [-0.0, 0.0]])
    a = g.standard_normal(len(y))
    full_check(x, y, a, 1e-4, 9, "ties")


def test_wide_spread_small_delta():
    """Gaps far beyond the decay length: exponentials underflow, general exp path."""
    g = np.random.default_rng(3)
    y = g.uniform(-1e6, 1e6, 20000)
    x = np.concatenate([y[:500] + g.normal(0, 1e-4, 500), g.uniform(-1e6, 1e6, 9500)])
    a = g.standard_normal(len(y))
    full_check(x, y, a, 1e-6, 6, "spread")


@pytest.mark.parametrize("delta", [1e-4, 1e-10])
def test_near_duplicates_below_key_resolution(delta):
    """Points a few ulps apart: the library may leave them unordered (its
    key resolution); the result must stay within the stated bounds."""
    g = np.random.default_rng(6)
    base = g.random(300)
    y = (base[g.integers(0, 300, 20000)] + g.integers(0, 64, 20000) * 2.0 ** -52)
    x = (base[g.integers(0, 300, 15000)] + g.integers(0, 64, 15000) * 2.0 ** -52)
    a = g.standard_normal(len(y))
    full_check(x, y, a, delta, 6, "near-dup")


def _code_case(kind, g):
    if kind == "far_positive":      # range far from 0: offsets from its aligned start
        y, x = 1e6 + g.random(20000), 1e6 + g.random(15000)
    elif kind == "far_negative":
        y, x = -5e3 - 2 * g.random(20000), -5e3 - 2 * g.random(15000)
    elif kind == "straddle_tiny":   # points below the grid step near 0 move by < g
        tiny = np.array([1e-20, -1e-20, 3e-310, -3e-310, 0.0, -0.0, 2.0 ** -70])
        y = np.concatenate([g.uniform(-1, 1, 20000), tiny])
        x = np.concatenate([g.uniform(-1, 1, 15000), tiny, -tiny])
    else:                           # "two_points": the smallest non-degenerate range
        y, x = np.array([0.25, 0.75]), np.array([0.75, 0.25, 0.5])
    return x, y, g.standard_normal(len(y))


@pytest.mark.parametrize("kind", ["far_positive", "far_negative", "straddle_tiny", "two_points"])
@pytest.mark.parametrize("delta,digits", [(1e-4, 6), (1e-6, 11)])
def test_fp64_key_code_ranges(kind, delta, digits):
    """FP64 keys are coded on a grid fitted to the points' range where that
    moves no point by more than the plan allows (else IEEE keys): ranges far
    from 0 on either side, ranges through 0 with values below the grid step,
    tiny sets; 11 digits at delta 1e-6 keeps IEEE keys for ranges through 0."""
    x, y, a = _code_case(kind, np.random.default_rng(12))
    full_check(x, y, a, delta, digits, f"code-{kind}")


def test_clustered_small():
    pr = W.clustered(log2n=15, log2m=13, delta=1e-5, digits=6, n_comp=16)
    full_check(pr.x, pr.y, pr.alpha, pr.delta, 6, "clustered-small")


def test_deterministic():
    pr = W.plain(50000, 60000, 1e-4, 6, cfg=12)
    u1, _, _ = gpu_eval(pr.x, pr.y, pr.alpha, 1e-4, 6, case="det-1")
    u2, _, _ = gpu_eval(pr.x, pr.y, pr.alpha, 1e-4, 6, case="det-2")
    assert np.array_equal(u1.view(np.int64), u2.view(np.int64))


def test_nonfinite_is_reported():
    x = np.random.default_rng(4).random(1000)
    y = np.random.default_rng(5).random(1000)
    x[17] = np.nan
    _, _, st = gpu_eval(x, y, np.ones(1000), 1e-3, 6, case="nan")
    assert st == fgt.FGT_ENONFINITE
    y[3] = np.inf
    x[17] = 0.5
    _, _, st = gpu_eval(x, y, np.ones(1000), 1e-3, 6, case="inf")
    assert st == fgt.FGT_ENONFINITE


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_nonfinite_is_reported_multi_kernel(dtype):
    """Above 4096 points fgt_eval runs the range, histogram and radix kernels;
    a NaN or an infinity among the coordinates is reported there too, and a
    finite call after it reads OK."""
    g = np.random.default_rng(6)
    x, y = g.random(5000), g.random(6000)
    x[1234] = np.nan
    _, _, st = gpu_eval(x, y, np.ones(6000), 1e-3, 6, dtype=dtype, case="nan, multi-kernel")
    assert st == fgt.FGT_ENONFINITE
    x[1234] = 0.5
    y[77] = -np.inf
    _, _, st = gpu_eval(x, y, np.ones(6000), 1e-3, 6, dtype=dtype, case="-inf, multi-kernel")
    assert st == fgt.FGT_ENONFINITE
    y[77] = 0.25
    _, _, st = gpu_eval(x, y, np.ones(6000), 1e-3, 6, dtype=dtype, case="finite, multi-kernel")
    assert st == fgt.FGT_OK


@pytest.mark.parametrize("digits", [3, 4, 6])
def test_fp32(digits):
    """FP32 inputs (the FP32-rounded values, cast exactly to FP64 for the oracle).

    Stated error: E_n plus FP32 rounding of the recurrences, bounded here by
    E_n + 64 eps32 sum|omega| (relative to sum|alpha|)."""
    pr = W.plain(30001, 40003, 1e-4, digits, cfg=13, sub=digits)
    x32 = pr.x.astype(np.float32)
    y32 = pr.y.astype(np.float32)
    a32 = pr.alpha.astype(np.float32)
    u, p, st = gpu_eval(x32, y32, a32, 1e-4, digits, dtype=torch.float32, case="fp32")
    assert st == fgt.FGT_OK
    ref = oracle.direct(x32.astype(np.float64), y32.astype(np.float64), a32.astype(np.float64), 1e-4)
    s_alpha = float(np.sum(np.abs(a32.astype(np.float64))))
    err = float(np.max(np.abs(u - ref))) / s_alpha
    bound = oracle_E(p) + 64 * EPS32 * oracle_sum_omega(p)
    say(f"   FP32 error / sum|alpha| = {err:.3e} (E = {oracle_E(p):.2e}, bound {bound:.2e})")
    assert err <= bound
