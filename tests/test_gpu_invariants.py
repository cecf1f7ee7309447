"""Invariants of the transform (1.1) and of its SOE form (1.3), run against the
HIP path at the small configuration (M = N = 1000 uniform on [0,1), alpha ~
N(0,1), delta = 1e-3, 6 digits) and at sizes with several tiles.

* alpha = e_j gives u_i = S(x_i - y_j) (the oracle's SOE kernel, pair by pair)
  and |u_i - G(x_i - y_j)| <= E_n;
* linearity in alpha, permutation invariance, translation by a shift that is
  exact on the points' grid, exact scaling u(sx, sy; s^2 delta) = u(x, y; delta)
  for a power of two s;
* the transpose identity <g, K alpha> = <K^T g, alpha> (K^T: the same transform
  with targets and sources swapped; the kernel is symmetric);
* the large- and small-delta limits: u_i -> S(0) sum alpha, and u_i -> the sum
  of the strengths at x_i.

Rounding tolerances come from fgt_testlib.impl_tol (the O2 bar).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1909_09825_amd as fgt
from paper_1909_09825_amd import workloads as W
from fgt_testlib import impl_tol, oracle_E, oracle_table, say, to_dev

pytestmark = pytest.mark.gpu


class Runner:
    def __init__(self, delta, digits):
        self.p = fgt.plan(delta, digits)
        self.delta = delta

    def __call__(self, x, y, a, delta=None):
        p = self.p if delta is None else fgt.plan(delta, self.p.digits)
        X, Y, A = (to_dev(v, torch.float64) for v in (x, y, a))
        ws = fgt.workspace(p, len(x), len(y), X.device)
        u = fgt.eval(X, Y, A, p, ws=ws)
        assert fgt.last_device_status(ws) == fgt.FGT_OK
        return u.cpu().numpy()


def small():
    pr = W.small_plain()
    return pr.x, pr.y, pr.alpha, pr.delta, pr.digits


def test_unit_strength_gives_kernel():
    x, y, _, delta, digits = small()
    run = Runner(delta, digits)
    t = oracle_table(run.p)
    say("[gpu] alpha = e_j, j in 5 positions")
    for j in (0, 1, 499, 998, 999):
        a = np.zeros(len(y))
        a[j] = 1.0
        u = run(x, y, a)
        s = oracle.soe_brute(x, y[j:j + 1], np.ones(1), delta, t["tau0"], t["omega"])
        gk = np.exp(-(x - y[j]) ** 2 / (4 * delta))
        assert np.max(np.abs(u - s)) <= impl_tol(a, run.p, len(x) + len(y))
        assert np.max(np.abs(u - gk)) <= oracle_E(run.p) + impl_tol(a, run.p, len(x) + len(y))


def test_linearity():
    x, y, a, delta, digits = small()
    run = Runner(delta, digits)
    b = np.random.default_rng(21).standard_normal(len(y))
    say("[gpu] linearity 2.5 a - 0.75 b")
    u = run(x, y, 2.5 * a - 0.75 * b)
    v = 2.5 * run(x, y, a) - 0.75 * run(x, y, b)
    tol = impl_tol(np.abs(2.5 * a) + np.abs(0.75 * b), run.p, len(x) + len(y))
    assert np.max(np.abs(u - v)) <= 3 * tol


@pytest.mark.parametrize("M,N", [(1000, 1000), (20011, 30007)])
def test_permutation_invariance(M, N):
    pr = W.plain(M, N, 1e-3, 6, cfg=15, sub=M % 7)
    run = Runner(1e-3, 6)
    g = np.random.default_rng(22)
    px, py = g.permutation(M), g.permutation(N)
    say(f"[gpu] permutation M={M} N={N}")
    u = run(pr.x, pr.y, pr.alpha)
    v = run(pr.x[px], pr.y[py], pr.alpha[py])
    assert np.max(np.abs(v - u[px])) <= impl_tol(pr.alpha, run.p, M + N)


@pytest.mark.parametrize("c", [0.5, -3.0, 1024.0])
def test_translation_invariance(c):
    # points on the 2^-40 grid, so x + c is exact for these shifts
    pr = W.plain(20011, 30007, 1e-4, 6, cfg=15, sub=3)
    x = np.round(pr.x * 2.0 ** 40) / 2.0 ** 40
    y = np.round(pr.y * 2.0 ** 40) / 2.0 ** 40
    assert np.array_equal((x + c) - c, x) and np.array_equal((y + c) - c, y)
    run = Runner(1e-4, 6)
    say(f"[gpu] translation by {c}")
    u = run(x, y, pr.alpha)
    v = run(x + c, y + c, pr.alpha)
    assert np.max(np.abs(u - v)) <= impl_tol(pr.alpha, run.p, len(x) + len(y))


@pytest.mark.parametrize("s", [0.25, 8.0])
def test_exact_scaling(s):
    """u(s x, s y; s^2 delta) = u(x, y; delta): S's nodes scale as 1/sqrt(delta)."""
    pr = W.plain(20011, 30007, 1e-4, 6, cfg=15, sub=4)
    run = Runner(1e-4, 6)
    say(f"[gpu] scaling by {s}")
    u = run(pr.x, pr.y, pr.alpha)
    v = run(s * pr.x, s * pr.y, pr.alpha, delta=s * s * 1e-4)
    assert np.max(np.abs(u - v)) <= impl_tol(pr.alpha, run.p, len(pr.x) + len(pr.y))


@pytest.mark.parametrize("M,N", [(1000, 1000), (20011, 30007)])
def test_transpose_identity(M, N):
    pr = W.plain(M, N, 1e-3, 6, cfg=15, sub=5)
    gw = np.random.default_rng(23).standard_normal(M)
    run = Runner(1e-3, 6)
    say(f"[gpu] transpose identity M={M} N={N}")
    u = run(pr.x, pr.y, pr.alpha)            # K alpha at the targets
    w = run(pr.y, pr.x, gw)                  # K^T g at the sources
    lhs, rhs = float(gw @ u), float(w @ pr.alpha)
    tol = impl_tol(pr.alpha, run.p, M + N) * float(np.abs(gw).sum()) \
        + impl_tol(gw, run.p, M + N) * float(np.abs(pr.alpha).sum())
    assert abs(lhs - rhs) <= tol


def test_large_delta_limit():
    """delta >> range^2: every pair sits near 0, u_i -> S(0) sum alpha (within E_n)."""
    x, y, a, _, _ = small()
    run = Runner(1e6, 6)
    say("[gpu] delta = 1e6")
    u = run(x, y, a)
    s0 = float(np.sum(oracle_table(run.p)["omega"]).real)
    s_alpha = float(np.abs(a).sum())
    # |S(r) - S(0)| <= |S - G|(r) + |G(r) - G(0)| + |G - S|(0) <= 2 E_n + r^2 / (4 delta), r < 1
    assert np.max(np.abs(u - s0 * a.sum())) <= (2 * oracle_E(run.p) + 0.25e-6) * s_alpha \
        + impl_tol(a, run.p, 2000)
    assert abs(s0 - 1.0) <= oracle_E(run.p)


def test_small_delta_limit():
    """delta << spacing^2: only coincident sources contribute (weight S(0))."""
    g = np.random.default_rng(24)
    grid = np.arange(5000) / 5000.0
    y = g.choice(grid, 8000)
    x = np.concatenate([g.choice(y, 3000), grid[:2000] + 0.5 / 5000.0])
    a = g.standard_normal(len(y))
    run = Runner(1e-14, 6)
    say("[gpu] delta = 1e-14")
    u = run(x, y, a)
    s0 = float(np.sum(oracle_table(run.p)["omega"]).real)
    exact = np.array([a[y == xi].sum() for xi in x]) * s0
    assert np.max(np.abs(u - exact)) <= impl_tol(a, run.p, len(x) + len(y))


def test_one_source_one_target():
    run = Runner(1e-3, 9)
    t = oracle_table(run.p)
    say("[gpu] M = N = 1")
    for x, y in ((0.3, 0.31), (0.3, 0.3), (-2.0, 5.0)):
        u = run(np.array([x]), np.array([y]), np.array([1.75]))
        s = oracle.soe_brute(np.array([x]), np.array([y]), np.array([1.75]), 1e-3, t["tau0"],
                             t["omega"])
        assert abs(u[0] - s[0]) <= impl_tol(np.array([1.75]), run.p, 2)
