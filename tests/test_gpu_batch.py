"""Batched transforms (fgt_batch_plan / fgt_batch_eval) against the oracle.

Every transform b and column r of a batch is checked on its own:
  * against O1 (direct Gaussian sum) within 2 E_n sum_j |alpha_jr|;
  * against O2 (the oracle's SOE recurrence, same table) within the rounding
    tolerance of the single-transform tests.
Cases: mixed sizes with empty transforms, deltas from 1e-7 to 10, negative
coordinates; buckets larger than the LDS sort (coincident and clustered
points); HIP-graph capture and replay; determinism; non-finite input; and the
4096-transform, 16-column workload on sampled transforms and targets.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1909_09825_amd as fgt
from paper_1909_09825_amd import workloads as W
from fgt_testlib import impl_tol, oracle_E, oracle_table, say, to_dev

pytestmark = pytest.mark.gpu


def make_batch(sizes, deltas, R, seed, spread=(0.0, 1.0)):
    g = np.random.default_rng(seed)
    Ms = np.array([m for m, _ in sizes], np.int64)
    Ns = np.array([n for _, n in sizes], np.int64)
    x_off = np.concatenate([[0], np.cumsum(Ms)]).astype(np.int64)
    y_off = np.concatenate([[0], np.cumsum(Ns)]).astype(np.int64)
    x = g.uniform(*spread, int(x_off[-1]))
    y = g.uniform(*spread, int(y_off[-1]))
    a = g.standard_normal((int(y_off[-1]), R))
    return W.Batch(x, y, a, x_off, y_off, np.asarray(deltas, np.float64), 6)


def run_batch(bt, digits, case=""):
    B, R = len(bt.delta), bt.alpha.shape[1]
    say(f"[gpu] fgt_batch_eval {case} B={B} R={R} sumM={bt.x_off[-1]} sumN={bt.y_off[-1]} digits={digits}")
    bp = fgt.batch_plan(bt.delta, digits, bt.x_off, bt.y_off, R)
    X, Y = to_dev(bt.x, torch.float64), to_dev(bt.y, torch.float64)
    A = to_dev(bt.alpha, torch.float64)
    ws = fgt.batch_workspace(bp, X.device)
    u = fgt.eval_batch(X, Y, A, bp, ws=ws)
    st = fgt.last_device_status(ws)
    return u.cpu().numpy(), bp, st


def check_transform(bt, u, b, digits, targets=None, recurrence=True):
    xs, xe = bt.x_off[b], bt.x_off[b + 1]
    ys, ye = bt.y_off[b], bt.y_off[b + 1]
    x, y, delta = bt.x[xs:xe], bt.y[ys:ye], float(bt.delta[b])
    if len(x) == 0:
        return 0.0, 0.0
    p = fgt.plan(delta, digits)
    t = oracle_table(p)
    ti = np.arange(len(x)) if targets is None else targets
    worst1 = worst2 = 0.0
    for r in range(bt.alpha.shape[1]):
        a = bt.alpha[ys:ye, r]
        got = u[xs:xe, r][ti]
        s_a = float(np.abs(a).sum())
        if len(y) == 0:
            assert np.all(got == 0.0)
            continue
        ref = oracle.direct(x[ti], y, a, delta)
        e1 = float(np.max(np.abs(got - ref))) / s_a
        assert e1 <= 2 * oracle_E(p), (b, r, e1, oracle_E(p))
        worst1 = max(worst1, e1 / oracle_E(p))
        if recurrence:
            ref2 = oracle.soe_recurrence(x, y, a, delta, t["tau0"], t["omega"])[ti]
            tol = impl_tol(a, p, len(x) + len(y))
            e2 = float(np.max(np.abs(got - ref2)))
            assert e2 <= tol, (b, r, e2, tol)
            worst2 = max(worst2, e2 / tol)
    return worst1, worst2


SIZES = [(0, 50), (40, 0), (0, 0), (1, 1), (3000, 5000), (20000, 17000), (257, 9001), (5, 70000),
         (33000, 1)]
DELTAS = [1e-3, 1e-2, 1.0, 1e-4, 1e-5, 1e-7, 3e-2, 10.0, 1e-6]


@pytest.mark.parametrize("digits", [3, 6, 9])
def test_batch_mixed(digits):
    bt = make_batch(SIZES, DELTAS, R=3, seed=100 + digits, spread=(-0.7, 0.9))
    u, bp, st = run_batch(bt, digits, case="mixed")
    assert st == fgt.FGT_OK
    w1 = w2 = 0.0
    for b in range(len(SIZES)):
        e1, e2 = check_transform(bt, u, b, digits)
        w1, w2 = max(w1, e1), max(w2, e2)
    say(f"   worst O1 err / E_n = {w1:.3e}, worst O2 err / tol = {w2:.3e}")


def test_batch_matches_single_transform_path():
    bt = make_batch([(4000, 3000), (1000, 12000), (7000, 7000)], [1e-4, 1e-3, 1e-5], R=1, seed=7)
    u, bp, _ = run_batch(bt, 6, case="vs single")
    for b in range(3):
        xs, xe, ys, ye = bt.x_off[b], bt.x_off[b + 1], bt.y_off[b], bt.y_off[b + 1]
        p = fgt.plan(float(bt.delta[b]), 6)
        ref = fgt.eval(to_dev(bt.x[xs:xe], torch.float64), to_dev(bt.y[ys:ye], torch.float64),
                       to_dev(bt.alpha[ys:ye, 0], torch.float64), p).cpu().numpy()
        tol = 2 * impl_tol(bt.alpha[ys:ye, 0], p, (xe - xs) + (ye - ys))
        assert np.max(np.abs(u[xs:xe, 0] - ref)) <= tol


def test_batch_large_buckets():
    """Buckets above the LDS capacity: coincident points and a narrow cluster."""
    g = np.random.default_rng(11)
    xs = [np.concatenate([np.full(9000, 0.25), g.random(3000)]),
          np.concatenate([0.5 + 1e-7 * g.random(15000), g.random(2000)]),
          g.random(500)]
    ys = [np.concatenate([np.full(7000, 0.25), g.random(4000)]),
          np.concatenate([0.5 + 1e-7 * g.random(12000), g.random(3000)]),
          np.full(20000, -1.0)]
    x_off = np.concatenate([[0], np.cumsum([len(v) for v in xs])]).astype(np.int64)
    y_off = np.concatenate([[0], np.cumsum([len(v) for v in ys])]).astype(np.int64)
    a = g.standard_normal((int(y_off[-1]), 2))
    bt = W.Batch(np.concatenate(xs), np.concatenate(ys), a, x_off, y_off,
                 np.array([1e-3, 1e-12, 1.0]), 6)
    u, bp, st = run_batch(bt, 6, case="large buckets")
    assert st == fgt.FGT_OK
    for b in range(3):
        # O1 only: O2's recurrence over exact ties follows a different (valid) order
        check_transform(bt, u, b, 6, recurrence=False)


def test_batch_deterministic_and_graph_replay():
    bt = make_batch([(3000, 2000), (0, 10), (9000, 11000), (64, 64)], [1e-3, 1e-2, 1e-5, 0.1],
                    R=16, seed=12)
    say("[gpu] batch eager x2, then HIP graph capture and replays")
    bp = fgt.batch_plan(bt.delta, 6, bt.x_off, bt.y_off, 16)
    X, Y = to_dev(bt.x, torch.float64), to_dev(bt.y, torch.float64)
    A = to_dev(bt.alpha, torch.float64)
    ws = fgt.batch_workspace(bp, X.device)
    u1 = fgt.eval_batch(X, Y, A, bp, ws=ws).clone()
    u2 = fgt.eval_batch(X, Y, A, bp, ws=ws).clone()
    assert torch.equal(u1, u2)
    out = torch.empty_like(u1)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fgt.eval_batch(X, Y, A, bp, out=out, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fgt.eval_batch(X, Y, A, bp, out=out, ws=ws)
    for rep in range(3):
        out.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()   # eager work between
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, u1), f"replay {rep}"
        del junk


def test_batch_nonfinite_is_reported():
    bt = make_batch([(100, 100), (50, 60)], [1e-3, 1e-3], R=1, seed=13)
    bt.y[70] = np.nan
    _, _, st = run_batch(bt, 6, case="nan")
    assert st == fgt.FGT_ENONFINITE


def test_batch_one_shot_entry_point():
    bt = make_batch([(500, 800), (300, 0), (1200, 700)], [1e-3, 1e-2, 1e-4], R=2, seed=14)
    say("[gpu] fgt_eval_batched (one shot)")
    lib = fgt._lib.load()
    X, Y = to_dev(bt.x, torch.float64), to_dev(bt.y, torch.float64)
    A = to_dev(bt.alpha, torch.float64)
    U = torch.empty((int(bt.x_off[-1]), 2), dtype=torch.float64, device="cuda")
    i64p = lambda v: v.ctypes.data_as(__import__("ctypes").POINTER(__import__("ctypes").c_int64))  # noqa: E731
    dp = bt.delta.ctypes.data_as(__import__("ctypes").POINTER(__import__("ctypes").c_double))
    need = lib.fgt_eval_batched_workspace_size(3, i64p(bt.x_off), i64p(bt.y_off), 2, 6)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rc = lib.fgt_eval_batched(3, dp, 6, fgt.FGT_F64, i64p(bt.x_off), i64p(bt.y_off), X.data_ptr(),
                              Y.data_ptr(), A.data_ptr(), 2, U.data_ptr(), ws.data_ptr(), need,
                              torch.cuda.current_stream().cuda_stream)
    assert rc == fgt.FGT_OK
    ref, _, _ = run_batch(bt, 6, case="plan path")
    assert np.array_equal(U.cpu().numpy(), ref)


def test_batch_4096_transforms_16_columns():
    """The batched workload: 4096 transforms, N_b and M_b log-uniform in
    [256, 65536], delta_b log-uniform in [1e-6, 1e-2], 16 columns, 6 digits;
    64 sampled transforms x 256 targets x 16 columns against O1."""
    bt = W.batched()
    u, bp, st = run_batch(bt, 6, case="4096x16")
    assert st == fgt.FGT_OK
    g = np.random.default_rng(15)
    picks = g.choice(len(bt.delta), 64, replace=False)
    worst = 0.0
    for b in picks:
        M = int(bt.x_off[b + 1] - bt.x_off[b])
        ti = np.sort(g.choice(M, min(256, M), replace=False))
        e1, _ = check_transform(bt, u, int(b), 6, targets=ti, recurrence=False)
        worst = max(worst, e1)
    say(f"   64 transforms x 256 targets x 16 columns: worst O1 err / E_n = {worst:.3e}")


def test_batch_tuner_choices_agree_and_cache(tmp_path):
    """Every kernel choice gives the same transform (to rounding); the tuner
    picks one of them and records it in the JSON cache, which a second plan
    of the same shape reads back."""
    bt = make_batch([(3000, 2000), (0, 10), (9000, 11000), (64, 64), (40000, 30000)],
                    [1e-3, 1e-2, 1e-5, 0.1, 1e-4], R=16, seed=17)
    say("[gpu] batch tuner: 4 choices, then tune with a cache")
    bp = fgt.batch_plan(bt.delta, 6, bt.x_off, bt.y_off, 16)
    X, Y = to_dev(bt.x, torch.float64), to_dev(bt.y, torch.float64)
    A = to_dev(bt.alpha, torch.float64)
    ws = fgt.batch_workspace(bp, X.device)
    outs = {}
    for chunk in (8, 16):
        for bucket in (1024, 2048):
            bp.set_config(chunk, bucket)
            outs[(chunk, bucket)] = fgt.eval_batch(X, Y, A, bp, ws=ws).cpu().numpy()
    ref = outs[(16, 2048)]
    scale = np.abs(bt.alpha).sum(axis=0).max()
    for k, v in outs.items():
        assert np.max(np.abs(v - ref)) <= 1e-12 * scale, k
    with pytest.raises(fgt.FGTError):
        bp.set_config(12, 2048)
    cache = str(tmp_path / "tune.json")
    cfg = bp.tune(X, Y, A, ws=ws, cache=cache)
    assert cfg in outs
    text = open(cache).read()
    assert "gfx950:" in text and f'"chunk": {cfg[0]}' in text
    bp2 = fgt.batch_plan(bt.delta, 6, bt.x_off, bt.y_off, 16)
    bp2.set_config(8 if cfg[0] == 16 else 16, 1024 if cfg[1] == 2048 else 2048)
    assert bp2.tune(X, Y, A, ws=ws, cache=cache) == cfg
