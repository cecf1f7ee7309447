"""The batched sort step (fgt_batch_sorted) as index work.

For every transform of a batch, the sorted codes must be a permutation of its
sources and targets, each carrying its coordinate bit for bit; their order
must equal numpy's stable argsort of the key the header documents (the
range-normalised 62-bit key of the scaled coordinate with the bits below the
sort resolution dropped), computed here on the host with the same FP64
operations; and two points out of coordinate order must lie closer than the
stated resolution plus the key's rounding.  Section 4 sorts sources and targets
together; equal keys keep the merged order [sources; targets], so a source
coinciding with a target comes first, the split the recurrences assume.

Cases: mixed sizes with empty transforms and deltas from 1e-12 to 10; exact
ties between sources and targets, duplicates and -0 beside +0; a transform
whose points all coincide; buckets above the LDS sort's capacity (coincident
points and a 1e-7-wide cluster), which take the block-global path.
"""
import math

import numpy as np
import pytest
import torch

import paper_1909_09825_amd as fgt
from fgt_testlib import say, to_dev

pytestmark = pytest.mark.gpu

TWO62 = 4.611686018427387904e18


def host_keys(z, scale):
    """The documented key of every coordinate of one transform, and its range factor."""
    zp = z * scale
    lo, hi = float(zp.min()), float(zp.max())
    qs = TWO62 / (hi - lo) if hi > lo else 0.0
    if not math.isfinite(qs):
        qs = 0.0
    v = np.clip((zp - lo) * qs, 0.0, TWO62)
    return v.astype(np.uint64), qs


def low_bit_choices(qs, s_allow):
    """Lowest sorted key bit(s): floor(log2(s 2^62 / range)) in [0, 62], both
    neighbours when that logarithm is within rounding of an integer."""
    if qs == 0.0:
        return [64]
    units = s_allow * qs
    if not units >= 1.0:
        return [0]
    l2 = math.log2(units)
    out = {min(int(math.floor(l2)), 62)}
    if abs(l2 - round(l2)) < 1e-9:
        out |= {min(int(round(l2)) - 1, 62), min(int(round(l2)), 62)}
    return sorted(b for b in out if b >= 0)


def check_batch(xs, ys, deltas, digits=6, case=""):
    x_off = np.concatenate([[0], np.cumsum([len(v) for v in xs])]).astype(np.int64)
    y_off = np.concatenate([[0], np.cumsum([len(v) for v in ys])]).astype(np.int64)
    x = np.concatenate(xs) if xs else np.zeros(0)
    y = np.concatenate(ys) if ys else np.zeros(0)
    SN = int(y_off[-1])
    g = np.random.default_rng(3)
    a = g.standard_normal((SN, 1))
    say(f"[gpu] fgt_batch_sorted {case}: B={len(deltas)} sumM={x_off[-1]} sumN={SN}")
    bp = fgt.batch_plan(np.asarray(deltas, np.float64), digits, x_off, y_off, 1)
    X, Y, A = to_dev(x, torch.float64), to_dev(y, torch.float64), to_dev(a, torch.float64)
    ws = fgt.batch_workspace(bp, X.device)
    fgt.eval_batch(X, Y, A, bp, ws=ws)
    assert fgt.last_device_status(ws) == fgt.FGT_OK
    codes, zs, s_allow = fgt.batch_sorted(bp, ws)
    codes, zs = codes.cpu().numpy(), zs.cpu().numpy()
    assert s_allow > 0.0
    base = 0
    for b, delta in enumerate(deltas):
        xb, yb = xs[b], ys[b]
        N, M = len(yb), len(xb)
        got = codes[base:base + M + N]
        zb = zs[base:base + M + N]
        merged_codes = np.concatenate([y_off[b] + np.arange(N), SN + x_off[b] + np.arange(M)])
        merged_z = np.concatenate([yb, xb])
        # a permutation of this transform's points, coordinates carried bit for bit
        assert np.array_equal(np.sort(got), np.sort(merged_codes)), (case, b)
        pos = np.where(got < SN, got - y_off[b], N + (got - SN - x_off[b]))
        assert np.array_equal(zb.view(np.uint64), merged_z[pos].view(np.uint64)), (case, b)
        if M + N == 0:
            continue
        scale = 1.0 / math.sqrt(delta)
        keys, qs = host_keys(merged_z, scale)
        # the documented order: stable in the key above the resolution bits
        ok = []
        for lb in low_bit_choices(qs, s_allow):
            shift = 8 * (lb // 8) if lb < 64 else 64
            kk = keys >> np.uint64(shift) if shift < 64 else np.zeros_like(keys)
            ok.append(np.array_equal(got, merged_codes[np.argsort(kk, kind="stable")]))
        assert any(ok), (case, b, delta, M, N)
        # order up to the resolution in coordinate units, plus the key's rounding:
        # |computed - exact key| <= 2^10 units + |z| scale qs 2^-53 per point
        unit = (1.0 / qs if qs > 0 else 0.0) / scale
        bound = s_allow / scale + (2**11 + 1) * unit + 2 * float(np.abs(merged_z).max()) * 2.0**-53
        back = np.maximum.accumulate(zb) - zb
        assert float(back.max()) <= bound, (case, b, float(back.max()), bound)
        base += M + N
    return codes


def test_batch_sort_mixed():
    g = np.random.default_rng(21)
    sizes = [(0, 50), (40, 0), (0, 0), (1, 1), (3000, 5000), (20000, 17000), (257, 9001),
             (5, 70000), (33000, 1)]
    deltas = [1e-3, 1e-2, 1.0, 1e-4, 1e-5, 1e-7, 3e-2, 10.0, 1e-12]
    xs = [g.uniform(-0.7, 0.9, m) for m, _ in sizes]
    ys = [g.uniform(-0.7, 0.9, n) for _, n in sizes]
    check_batch(xs, ys, deltas, case="mixed")


def test_batch_sort_ties_duplicates_signed_zero():
    g = np.random.default_rng(22)
    grid = lambda n: np.round(g.uniform(-1, 1, n) * 40) / 40   # 81 values: many exact ties
    xs, ys = [], []
    for n in (3000, 12000, 700):
        xv, yv = grid(n), grid(n + 500)
        xv[::7] = -0.0
        yv[::11] = 0.0
        yv[1::13] = -0.0
        xs.append(xv)
        ys.append(yv)
    xs.append(np.full(5000, 0.3))   # every point of the transform equal
    ys.append(np.full(6000, 0.3))
    check_batch(xs, ys, [1e-3, 1e-5, 1.0, 1e-2], case="ties")


def test_batch_sort_large_buckets():
    g = np.random.default_rng(23)
    xs = [np.concatenate([np.full(9000, 0.25), g.random(3000)]),
          np.concatenate([0.5 + 1e-7 * g.random(15000), g.random(2000)]),
          g.random(500)]
    ys = [np.concatenate([np.full(7000, 0.25), g.random(4000)]),
          np.concatenate([0.5 + 1e-7 * g.random(12000), g.random(3000)]),
          np.full(20000, -1.0)]
    check_batch(xs, ys, [1e-3, 1e-12, 1.0], case="large buckets")


@pytest.mark.parametrize("digits", [3, 9])
def test_batch_sort_digits(digits):
    """The resolution follows the digits; the order rule holds at each."""
    g = np.random.default_rng(24 + digits)
    xs = [g.random(40000), 0.5 + 1e-6 * g.standard_normal(30000)]
    ys = [g.random(35000), 0.5 + 1e-6 * g.standard_normal(25000)]
    check_batch(xs, ys, [1e-4, 1e-6], digits=digits, case=f"digits {digits}")
