"""The sort step (Section 4) on its own, as index work: bit-exact checks.

* FGT_SORT_EXACT: the permutation must equal numpy's stable argsort of the
  merged coordinates [y; x] (-0 read as +0) element for element, and the
  sorted coordinates must be the inputs bit for bit -- on ties, negatives,
  duplicates, signed zeros, wide exponent ranges, FP32, and the full
  2^24 + 2^24 benchmark input.
* The plan's resolution (what fgt_eval runs): the permutation is a
  permutation, every inversion spans less than the key width, and each
  coordinate moves by less than the code tolerance (exactly 0 for points on
  the key grid, which the benchmark's points are).
"""
import numpy as np
import pytest
import torch

import paper_1909_09825_amd as fgt
from paper_1909_09825_amd import workloads as W
from fgt_testlib import say, to_dev

pytestmark = pytest.mark.gpu


def merged(x, y, dtype):
    v = np.concatenate([y, x]).astype(dtype)
    v[v == 0] = 0.0          # -0 -> +0
    return v


def run_sort(x, y, exact, dtype=np.float64, delta=1e-4, digits=6, case=""):
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    say(f"[gpu] fgt_sort {case} M={len(x)} N={len(y)} exact={exact} {tdt}")
    p = fgt.plan(delta, digits, tdt)
    X, Y = to_dev(np.asarray(x, dtype), tdt), to_dev(np.asarray(y, dtype), tdt)
    ws = fgt.workspace(p, len(x), len(y), X.device)
    perm, z, res = fgt.sort(X, Y, p, exact=exact, ws=ws)
    assert fgt.last_device_status(ws) == fgt.FGT_OK
    return perm.cpu().numpy(), z.cpu().numpy(), res


def check_exact(x, y, dtype=np.float64, case=""):
    perm, z, res = run_sort(x, y, True, dtype, case=case)
    assert res == (0.0, 0.0)
    v = merged(x, y, dtype)
    ref = np.argsort(v, kind="stable")
    bad = np.nonzero(perm != ref)[0]
    assert bad.size == 0, f"{bad.size} positions differ, first at {bad[:5]}"
    assert np.array_equal(z.view(np.uint64 if dtype == np.float64 else np.uint32),
                          v[ref].view(np.uint64 if dtype == np.float64 else np.uint32))


def cases(dtype):
    g = np.random.default_rng(77)
    out = {
        "uniform ragged": (g.random(30007), g.random(20011)),
        "ties on a 1e-3 grid": (np.round(g.random(40000), 3), np.round(g.random(25000), 3)),
        "negatives and duplicates": (np.repeat(g.standard_normal(5000), 3),
                                     np.repeat(g.standard_normal(7000), 2)),
        "signed zeros": (np.array([0.0, -0.0, 1.0, -1.0, -0.0] * 3000),
                         np.array([-0.0, 0.0, -1.0] * 4000)),
        "all equal": (np.full(9000, 0.375), np.full(11000, 0.375)),
        "one point each": (np.array([0.5]), np.array([0.5])),
        # radix tiles hold 8192 points: whole tiles only, and one point past them
        "two whole tiles": (g.random(10000), g.random(6384)),
        "one tile and a point": (g.random(4096), g.random(4097)),
    }
    if dtype == np.float64:
        e = g.integers(-300, 300, 30000).astype(np.float64)
        out["wide exponents"] = (np.sign(g.standard_normal(30000)) * 10.0 ** e,
                                 np.sign(g.standard_normal(17000)) * 10.0 ** e[:17000][::-1])
        out["denormals"] = (g.random(5000) * 1e-310, -g.random(6000) * 1e-310)
    else:
        out["wide exponents"] = (np.sign(g.standard_normal(30000)) *
                                 10.0 ** g.integers(-37, 37, 30000),
                                 np.sign(g.standard_normal(17000)) *
                                 10.0 ** g.integers(-37, 37, 17000))
    return out


@pytest.mark.parametrize("name", list(cases(np.float64)))
def test_exact_sort_fp64(name):
    x, y = cases(np.float64)[name]
    check_exact(x, y, np.float64, name)


@pytest.mark.parametrize("name", list(cases(np.float32)))
def test_exact_sort_fp32(name):
    x, y = cases(np.float32)[name]
    check_exact(x, y, np.float32, name)


def test_exact_sort_full_size():
    pr = W.large_plain(1e-4, 6)
    check_exact(pr.x, pr.y, np.float64, "2^24 + 2^24")


def check_resolution(x, y, delta, digits, case, dtype=np.float64):
    perm, z, (kw, ctol) = run_sort(x, y, False, dtype, delta, digits, case)
    v = merged(x, y, dtype).astype(np.float64)
    P = len(v)
    assert np.array_equal(np.sort(perm), np.arange(P))
    t = v[perm]
    # every inversion spans less than the key width
    span = float(np.max(np.maximum.accumulate(t) - t))
    moved = float(np.max(np.abs(z.astype(np.float64) - t)))
    say(f"   largest inversion {span:.3e} (key width {kw:.3e}); largest move {moved:.3e} "
        f"(code tolerance {ctol:.3e})")
    assert span < kw
    assert moved < ctol or moved == 0.0
    return moved


@pytest.mark.parametrize("delta,digits", [(1e-4, 6), (1e-2, 3), (1e-6, 9)])
def test_resolution_sort_full_size(delta, digits):
    pr = W.large_plain(delta, 6)
    moved = check_resolution(pr.x, pr.y, delta, digits, "2^24 + 2^24")
    assert moved == 0.0      # k 2^-53 points lie on the key grid


def test_resolution_sort_clustered():
    pr = W.clustered()
    check_resolution(pr.x, pr.y, pr.delta, 6, "clustered 2^22 + 2^24")


def test_resolution_sort_off_grid():
    """Points finer than the key grid (a range far wider than their spacing near 0)."""
    g = np.random.default_rng(78)
    x = np.concatenate([g.random(50000) * 1e-9, 1e3 + g.random(50000)])
    y = np.concatenate([-g.random(40000) * 1e-9, g.random(40000) * 1e3])
    check_resolution(x, y, 1e-2, 6, "off grid")
