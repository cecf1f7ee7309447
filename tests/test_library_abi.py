"""The C ABI on the CPU: the library loads, exports every function the header
declares, and its host-side paths (plans, tables, validation) behave as
documented.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1909_09825_amd as fgt
from paper_1909_09825_amd import _lib
from oracle import soe_table

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fgt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fgt_\w+)\s*\(", text)))


def test_header_symbols_are_exported():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_plan_selects_smallest_table():
    expect = {3: 2, 6: 4, 9: 6, 11: 7}
    for d, m in expect.items():
        p = fgt.plan(1e-4, d)
        assert p.n_modes == m
        assert p.err_bound <= 10.0 ** (-d)


def test_plan_scales_nodes_by_sqrt_delta():
    a = fgt.plan(1.0, 6)
    b = fgt.plan(1e-4, 6)
    np.testing.assert_allclose(b.tau, a.tau / 1e-2, rtol=1e-15)
    np.testing.assert_array_equal(a.omega, b.omega)
    assert a.err_bound == b.err_bound


@pytest.mark.parametrize("delta,digits,dtype,exc", [
    (0.0, 6, "f64", ValueError), (-1.0, 6, "f64", ValueError), (float("nan"), 6, "f64", ValueError),
    (float("inf"), 6, "f64", ValueError), (1e-3, 0, "f64", ValueError), (1e-3, 99, "f64", ValueError),
    (1e-3, 9, "f32", fgt.FGTError),
])
def test_plan_rejects_bad_arguments(delta, digits, dtype, exc):
    import torch
    dt = torch.float64 if dtype == "f64" else torch.float32
    with pytest.raises(exc):
        fgt.plan(delta, digits, dt)


def test_plan_codes_through_the_c_abi():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.fgt_plan(1e-3, 6, 0, None) == fgt.FGT_EINVAL
    assert lib.fgt_plan(1e-3, 6, 7, ctypes.byref(h)) == fgt.FGT_EINVAL
    assert lib.fgt_plan(1e-3, 7, fgt.FGT_F32, ctypes.byref(h)) == fgt.FGT_EUNSUPPORTED
    assert lib.fgt_plan(1e-3, 6, fgt.FGT_F64, ctypes.byref(h)) == fgt.FGT_OK
    assert lib.fgt_plan_info(None, None, None, None, None, None, None) == fgt.FGT_EINVAL
    assert lib.fgt_workspace_size(None, 10, 10) == 0
    assert lib.fgt_workspace_size(h, -1, 10) == 0
    assert lib.fgt_workspace_size(h, 10, 10) > 0
    assert lib.fgt_max_digits(fgt.FGT_F32) == 6 and lib.fgt_max_digits(5) == 0
    assert lib.fgt_strerror(fgt.FGT_ENONFINITE).decode() == "non-finite coordinate"
    lib.fgt_plan_destroy(h)
    lib.fgt_plan_destroy(None)


def test_eval_validation_happens_before_any_launch():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.fgt_plan(1e-3, 6, fgt.FGT_F64, ctypes.byref(h)) == fgt.FGT_OK
    dummy = ctypes.c_void_p(256)
    ok_ws = lib.fgt_workspace_size(h, 4, 4)
    # bad plan, negative sizes, too many points, null pointers, small or misaligned workspace
    assert lib.fgt_eval(None, dummy, 4, dummy, dummy, 4, dummy, dummy, ok_ws, None) == fgt.FGT_EINVAL
    assert lib.fgt_eval(h, dummy, -1, dummy, dummy, 4, dummy, dummy, ok_ws, None) == fgt.FGT_EINVAL
    assert lib.fgt_eval(h, dummy, 1 << 31, dummy, dummy, 1 << 31, dummy, dummy, ok_ws, None) == fgt.FGT_EINVAL
    assert lib.fgt_eval(h, None, 4, dummy, dummy, 4, dummy, dummy, ok_ws, None) == fgt.FGT_EINVAL
    assert lib.fgt_eval(h, dummy, 4, None, dummy, 4, dummy, dummy, ok_ws, None) == fgt.FGT_EINVAL
    assert lib.fgt_eval(h, dummy, 4, dummy, dummy, 4, dummy, None, ok_ws, None) == fgt.FGT_EINVAL
    assert lib.fgt_eval(h, dummy, 4, dummy, dummy, 4, dummy, dummy, ok_ws - 1, None) == fgt.FGT_EINVAL
    assert lib.fgt_eval(h, dummy, 4, dummy, dummy, 4, dummy, ctypes.c_void_p(257), ok_ws, None) == fgt.FGT_EINVAL
    assert lib.fgt_eval(h, dummy, 0, dummy, dummy, 4, dummy, dummy, ok_ws, None) == fgt.FGT_OK   # M = 0: nothing
    lib.fgt_plan_destroy(h)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7])
def test_shipped_tables_equal_the_oracles(otables, m):
    """The library's generator and the oracle's build the same tables independently."""
    digits = {1: 1, 2: 3, 3: 5, 4: 6, 5: 8, 6: 10, 7: 11}[m]
    p = fgt.plan(1.0, digits)
    assert p.n_modes == m
    np.testing.assert_array_equal(p.tau, otables[m]["tau0"])
    np.testing.assert_array_equal(p.omega, otables[m]["omega"])


@pytest.mark.parametrize("digits", [1, 3, 5, 6, 8, 10, 11])
def test_stated_bound_is_honest(digits):
    """The oracle re-measures the shipped table on the (3.1) grid and a finer one."""
    p = fgt.plan(1.0, digits)
    e, ep, _ = soe_table.table_errors(p.tau, p.omega)
    fine = np.concatenate([[0.0], np.logspace(-8.0, 2.0, 400001)])
    e2, ep2, _ = soe_table.table_errors(p.tau, p.omega, fine)
    assert max(e, e2) <= p.err_bound * (1 + 1e-12)
    assert max(ep, ep2) <= p.deriv_err_bound * 1.01


@pytest.mark.parametrize("digits", [1, 3, 4, 5, 6, 8, 9, 10, 11])
def test_stated_bounds_sit_on_the_oracles(otables, digits):
    """The plan states E_n and E'_n from its own generator; they may carry a
    small margin over the oracle's measurement but not inflate it: every GPU
    parity bar takes the oracle's values, and this keeps the two within
    [1, 1.002] (E_n) and [1, 1.02] (E'_n) of each other.  The table the plan
    picks for `digits` is the one the oracle's reading of "digits" picks."""
    p = fgt.plan(1.0, digits)
    assert soe_table.modes_for_digits(otables, digits) == p.n_modes
    t = otables[p.n_modes]
    assert t["E"] <= p.err_bound <= 1.002 * t["E"], (p.err_bound, t["E"])
    assert t["Eprime"] <= p.deriv_err_bound <= 1.02 * t["Eprime"], (p.deriv_err_bound, t["Eprime"])


def test_backward_and_eval_sorted_validation():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.fgt_plan(1e-3, 6, fgt.FGT_F64, ctypes.byref(h)) == fgt.FGT_OK
    d = ctypes.c_void_p(256)
    ws_ok = lib.fgt_workspace_size(h, 4, 4)
    # unknown flags; null g; small workspace; sorting needs x, y and alpha
    assert lib.fgt_backward(h, d, 4, d, d, 4, d, d, d, d, d, 2, d, ws_ok, None) == fgt.FGT_EINVAL
    assert lib.fgt_backward(h, d, 4, d, None, 4, d, d, d, d, d, 0, d, ws_ok, None) == fgt.FGT_EINVAL
    assert lib.fgt_backward(h, d, 4, d, d, 4, None, d, d, d, d, 0, d, ws_ok, None) == fgt.FGT_EINVAL
    assert lib.fgt_backward(h, d, 4, d, d, 4, d, d, d, d, d, 0, d, ws_ok - 1, None) == fgt.FGT_EINVAL
    assert lib.fgt_backward(h, None, 4, d, d, 4, d, d, d, d, None, 0, d, ws_ok, None) == fgt.FGT_EINVAL
    assert lib.fgt_backward(None, d, 4, d, d, 4, d, d, d, d, d, 0, d, ws_ok, None) == fgt.FGT_EINVAL
    assert lib.fgt_backward(h, None, 4, None, None, 4, d, d, d, d, d, fgt.FGT_SORTED,
                            ctypes.c_void_p(257), ws_ok, None) == fgt.FGT_EINVAL
    # nothing requested: nothing to do
    assert lib.fgt_backward(h, d, 4, d, d, 4, d, None, None, None, None, 0, d, ws_ok, None) == fgt.FGT_OK
    assert lib.fgt_eval_sorted(h, 4, 4, None, d, d, ws_ok, None) == fgt.FGT_EINVAL
    assert lib.fgt_eval_sorted(h, 4, 4, d, d, ctypes.c_void_p(257), ws_ok, None) == fgt.FGT_EINVAL
    assert lib.fgt_eval_sorted(h, 4, 4, d, d, d, ws_ok - 1, None) == fgt.FGT_EINVAL
    assert lib.fgt_eval_sorted(h, 0, 4, d, d, d, ws_ok, None) == fgt.FGT_OK
    lib.fgt_plan_destroy(h)


def _i64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def test_batch_plan_validation():
    lib = _lib.load()
    h = ctypes.c_void_p()
    delta = np.array([1e-3, 1e-4, 1e-2])
    xo = np.array([0, 10, 10, 25], np.int64)
    yo = np.array([0, 5, 17, 17], np.int64)
    bad = [
        (3, delta, 6, fgt.FGT_F64, xo, yo, 0),                                  # R = 0
        (3, delta, 6, fgt.FGT_F64, xo, yo, 65),                                 # R too large
        (3, delta, 0, fgt.FGT_F64, xo, yo, 4),                                  # digits
        (3, np.array([1e-3, -1.0, 1e-2]), 6, fgt.FGT_F64, xo, yo, 4),           # delta <= 0
        (3, np.array([1e-3, np.nan, 1e-2]), 6, fgt.FGT_F64, xo, yo, 4),         # delta NaN
        (3, delta, 6, fgt.FGT_F64, np.array([1, 10, 10, 25], np.int64), yo, 4),  # x_off[0] != 0
        (3, delta, 6, fgt.FGT_F64, np.array([0, 10, 9, 25], np.int64), yo, 4),   # decreasing
        (3, delta, 6, 7, xo, yo, 4),                                             # dtype
        (-1, delta, 6, fgt.FGT_F64, xo, yo, 4),                                  # B < 0
    ]
    for B, d, dig, dt, x_off, y_off, R in bad:
        assert lib.fgt_batch_plan(B, _dp(d), dig, dt, _i64p(x_off), _i64p(y_off), R,
                                  ctypes.byref(h)) == fgt.FGT_EINVAL
    assert lib.fgt_batch_plan(3, _dp(delta), 6, fgt.FGT_F32, _i64p(xo), _i64p(yo), 4,
                              ctypes.byref(h)) == fgt.FGT_EUNSUPPORTED
    assert lib.fgt_batch_plan(3, None, 6, fgt.FGT_F64, _i64p(xo), _i64p(yo), 4,
                              ctypes.byref(h)) == fgt.FGT_EINVAL
    assert lib.fgt_batch_eval(None, None, None, None, None, None, 0, None) == fgt.FGT_EINVAL
    assert lib.fgt_batch_sorted(None, None, 0, None, None, None, None) == fgt.FGT_EINVAL
    assert lib.fgt_batch_workspace_size(None) == 0
    lib.fgt_batch_destroy(None)


def test_batch_workspace_size_grows_with_points_and_columns():
    lib = _lib.load()
    xo = np.array([0, 1000, 1000, 5000], np.int64)
    yo = np.array([0, 300, 9000, 9000], np.int64)
    s1 = lib.fgt_eval_batched_workspace_size(3, _i64p(xo), _i64p(yo), 1, 6)
    s16 = lib.fgt_eval_batched_workspace_size(3, _i64p(xo), _i64p(yo), 16, 6)
    big = lib.fgt_eval_batched_workspace_size(3, _i64p(xo * 4), _i64p(yo * 4), 16, 6)
    assert 0 < s1 < s16 < big
    assert lib.fgt_eval_batched_workspace_size(3, _i64p(xo), _i64p(yo), 0, 6) == 0
    assert lib.fgt_eval_batched_workspace_size(3, _i64p(xo), _i64p(yo), 4, 0) == 0


def test_noalloc_host_checks():
    """fgt_eval_noalloc's host checks: the limit is the header's, sizes are refused
    before any HIP call (no device needed here)."""
    text = open(HEADER).read()
    m = re.search(r"#define FGT_NOALLOC_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.FGT_NOALLOC_BYTES
    lib = _lib.load()
    p = fgt.plan(1e-3, 6)
    assert lib.fgt_eval_noalloc(None, None, 10, None, None, 10, None, None) == _lib.FGT_EINVAL
    assert lib.fgt_eval_noalloc(p.handle, None, -1, None, None, 5, None, None) == _lib.FGT_EINVAL
    assert (lib.fgt_eval_noalloc(p.handle, None, 1_000_000, None, None, 1_000_000, None, None)
            == _lib.FGT_ENOSPACE)
    assert lib.fgt_eval_noalloc(p.handle, None, 0, None, None, 5, None, None) == _lib.FGT_OK
    # the header states that 1.5e6 points fit at any digits, FP64 and FP32
    import torch
    for dt in (torch.float64, torch.float32):
        for d in range(1, fgt.max_digits(dt) + 1):
            q = fgt.plan(1e-3, d, dt)
            assert q.workspace_size(750_000, 750_000) <= _lib.FGT_NOALLOC_BYTES
            assert q.workspace_size(1_000_000, 1_000_000) > _lib.FGT_NOALLOC_BYTES or dt == torch.float32
    assert "fixed workspace" in _lib.strerror(_lib.FGT_ENOSPACE)


@pytest.mark.parametrize("digits", [3, 4, 6, 9, 11])
@pytest.mark.parametrize("delta", [1e-6, 1e-3, 1.0])
def test_sort_resolution_from_oracle_table(delta, digits, otables):
    """The key width the sort may leave unordered, pinned by the oracle's table:
    a source and a target at scaled distance s that swap places change a value
    by exactly |Re sum_k omega_k (e^{tau0_k s} - e^{-tau0_k s})| per unit strength
    (S evaluated at -s instead of s); at s = width / sqrt(delta) this must stay
    within 1e-6 E_n (and not be pointlessly small).  The FP64 code tolerance c
    moves each end of a pair by < c, changing a term by at most
    (max|G'| + E'_n) 2 c / sqrt(delta) per unit strength, which must stay within
    0.5e-6 E_n."""
    p = fgt.plan(delta, digits)
    kw, ctol = fgt.sort_resolution(p)
    t = otables[p.n_modes]
    E, Ep = float(t["E"]), float(t["Eprime"])
    s = kw / np.sqrt(delta)
    swap = abs(float(np.sum(t["omega"] * 2.0 * np.sinh(t["tau0"] * s)).real))   # no cancellation
    assert 0.5e-6 * E <= swap <= 1.002e-6 * E
    r = np.linspace(0.0, 10.0, 200001)
    max_dg = float(np.max(np.abs(0.5 * r * np.exp(-r * r / 4))))
    shift = (max_dg + Ep) * 2 * ctol / np.sqrt(delta)
    assert 0.2e-6 * E <= shift <= 0.5e-6 * E * 1.002
    # exact mode reports zero widths; unknown flags are refused
    res = (ctypes.c_double * 2)()
    lib = _lib.load()
    assert lib.fgt_sort(p.handle, None, 0, None, None, 0, _lib.FGT_SORT_EXACT, None, None, res,
                        None, 0, None) == _lib.FGT_OK
    assert res[0] == 0.0 and res[1] == 0.0
    assert lib.fgt_sort(p.handle, None, 0, None, None, 0, 8, None, None, res, None, 0,
                        None) == _lib.FGT_EINVAL
