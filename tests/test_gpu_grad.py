"""Gradients on the GPU (fgt_backward and the autograd function) against the oracle.

L = sum_i g_i u_i.  Two references:
  * the SOE gradients themselves (the oracle's transposed O3 for dL/dalpha,
    O5 / O2 with derivative weights for dL/dx and dL/dy), to rounding;
  * the direct Gaussian gradients (O4), within the table's bounds:
      |dalpha_j err| <= 2 E_n sum|g|,
      |dx_i err|     <= 2 |g_i| E'_n / sqrt(delta) sum|alpha|,
      |dy_j err|     <= 2 |alpha_j| E'_n / sqrt(delta) sum|g|,
      |ddelta err|   <= 2 E''_n / (2 delta) sum|g| sum|alpha|,  E''_n = sup_r |r (S' - G')(r)|.
At the full size (N = M = 2^22, delta = 1e-4) O4 runs on 4096 sampled points
and O2 with derivative weights on every point; dL/ddelta is also checked by
central differences of the GPU forward.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1909_09825_amd as fgt
from paper_1909_09825_amd import workloads as W
from fgt_testlib import (EPS32, EPS64, impl_tol, oracle_E, oracle_Eprime, oracle_sum_dom, oracle_table,
                         say, to_dev)

pytestmark = pytest.mark.gpu


def impl_tol_der(w, p, P, eps=EPS64):
    """Rounding tolerance of a derivative field: impl_tol with |tau_k omega_k| in place of |omega_k|."""
    s_w = float(np.sum(np.abs(w)))
    s_dom = oracle_sum_dom(p)
    tie = 2.0 * oracle_Eprime(p) / math.sqrt(p.delta) * 1e-6 * s_w
    return 64.0 * eps * s_w * s_dom * max(1.0, math.log2(max(P, 2))) + tie


def e_second(p):
    """sup_r |r (S'(r) - G'(r))| at delta = 1 on a dense grid (the bound used for dL/ddelta)."""
    t = oracle_table(p)
    r = np.concatenate([np.linspace(0, 1, 20001), np.logspace(0, 2.3, 40001)])
    ds = np.zeros_like(r, dtype=np.complex128)
    for tk, wk in zip(t["tau0"], t["omega"]):
        ds += -wk * tk * np.exp(-tk * r)
    dg = -(r / 2) * np.exp(-r * r / 4)
    return float(np.max(np.abs(r * (ds.real - dg))))


def gpu_backward(x, y, a, g, delta, digits, dtype=torch.float64, sorted_after_eval=True, case=""):
    say(f"[gpu] fgt_backward {case} M={len(x)} N={len(y)} delta={delta:g} digits={digits} {dtype} "
        f"sorted={sorted_after_eval}")
    p = fgt.plan(delta, digits, dtype)
    X, Y, A, G = to_dev(x, dtype), to_dev(y, dtype), to_dev(a, dtype), to_dev(g, dtype)
    ws = fgt.workspace(p, len(x), len(y), X.device)
    u = fgt.eval(X, Y, A, p, ws=ws)
    da, dx, dy, dd = fgt.backward(X, Y, A, G, p, ws=ws, sorted=sorted_after_eval)
    st = fgt.last_device_status(ws)
    out = [t.double().cpu().numpy() for t in (da, dx, dy)] + [float(dd.item())]
    return out, u.double().cpu().numpy(), p, st


def soe_refs(x, y, a, g, p):
    """SOE-exact gradients from the oracle (no coincident points assumed)."""
    t = oracle_table(p)
    delta = p.delta
    da = oracle.soe_brute(y, x, g, delta, t["tau0"], t["omega"])
    dx = g * oracle.soe_deriv_brute(x, y, a, delta, t["tau0"], t["omega"])
    dy = a * oracle.soe_deriv_brute(y, x, g, delta, t["tau0"], t["omega"])
    c = 0.5 * (min(x.min(), y.min()) + max(x.max(), y.max()))
    dd = -(np.dot(x - c, dx) + np.dot(y - c, dy)) / (2 * delta)
    return da, dx, dy, dd


def check_all(got, x, y, a, g, p, eps=EPS64, soe=True, factor=2.0, case=""):
    da, dx, dy, dd = got
    delta = p.delta
    P = len(x) + len(y)
    sa, sg = float(np.abs(a).sum()), float(np.abs(g).sum())
    rd = math.sqrt(delta)
    if soe:
        r_da, r_dx, r_dy, r_dd = soe_refs(x, y, a, g, p)
        tda = impl_tol(g, p, P, eps)
        tdx = np.abs(g) * impl_tol_der(a, p, P, eps)
        tdy = np.abs(a) * impl_tol_der(g, p, P, eps)
        e = [np.max(np.abs(da - r_da)) / tda, np.max(np.abs(dx - r_dx) / tdx),
             np.max(np.abs(dy - r_dy) / tdy)]
        c = 0.5 * (min(x.min(), y.min()) + max(x.max(), y.max()))
        scale = (np.dot(np.abs(x - c), np.abs(r_dx)) + np.dot(np.abs(y - c), np.abs(r_dy))) / (2 * delta)
        tdd = (np.dot(np.abs(x - c), tdx) + np.dot(np.abs(y - c), tdy)) / (2 * delta) + 64 * eps * scale
        e.append(abs(dd - r_dd) / tdd)
        say(f"   {case} vs SOE oracle, err/tol: dalpha {e[0]:.2e} dx {e[1]:.2e} dy {e[2]:.2e} "
            f"ddelta {e[3]:.2e}")
        assert max(e) <= 1.0
    o_da, o_dx, o_dy, o_dd = oracle.direct_gradients(x, y, a, g, delta)
    ep = oracle_Eprime(p) / rd
    r = [np.max(np.abs(da - o_da)) / (factor * oracle_E(p) * sg + impl_tol(g, p, P, eps)),
         np.max(np.abs(dx - o_dx) / (np.abs(g) * (factor * ep * sa + impl_tol_der(a, p, P, eps)) + 1e-300)),
         np.max(np.abs(dy - o_dy) / (np.abs(a) * (factor * ep * sg + impl_tol_der(g, p, P, eps)) + 1e-300)),
         abs(dd - o_dd) / (factor * e_second(p) / (2 * delta) * sa * sg)]
    say(f"   {case} vs direct gradients, err/bound: dalpha {r[0]:.3e} dx {r[1]:.3e} dy {r[2]:.3e} "
        f"ddelta {r[3]:.3e}")
    assert max(r) <= 1.0


# ---------------------------------------------------------------------------
# small and ragged sizes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("digits", [3, 6, 9])
@pytest.mark.parametrize("delta", [1e-5, 1e-3, 1.0])
def test_grad_small(delta, digits):
    g0 = np.random.default_rng(1000 + digits)
    M, N = 3001, 4093
    x, y = g0.random(M), g0.random(N)
    a, g = g0.standard_normal(N), g0.standard_normal(M)
    got, _, p, st = gpu_backward(x, y, a, g, delta, digits, case="small")
    assert st == fgt.FGT_OK
    check_all(got, x, y, a, g, p, case=f"delta={delta:g} digits={digits}")


def test_grad_several_sort_tiles_and_fresh_sort():
    g0 = np.random.default_rng(7)
    M, N = 9000, 7777
    x, y = g0.uniform(-2, 3, M), g0.uniform(-2, 3, N)
    a, g = g0.standard_normal(N), g0.standard_normal(M)
    got, _, p, st = gpu_backward(x, y, a, g, 1e-3, 6, sorted_after_eval=False, case="tiles")
    assert st == fgt.FGT_OK
    check_all(got, x, y, a, g, p, case="P=16777")


def test_sorted_reuse_is_bitwise_identical():
    g0 = np.random.default_rng(8)
    M, N = 5000, 6000
    x, y = g0.random(M), g0.random(N)
    a, g = g0.standard_normal(N), g0.standard_normal(M)
    r1, u1, _, _ = gpu_backward(x, y, a, g, 1e-4, 6, sorted_after_eval=True, case="reuse")
    r2, u2, _, _ = gpu_backward(x, y, a, g, 1e-4, 6, sorted_after_eval=False, case="resort")
    for k in range(3):
        np.testing.assert_array_equal(r1[k], r2[k])
    assert r1[3] == r2[3]


def test_eval_sorted_matches_eval():
    g0 = np.random.default_rng(9)
    M, N = 4000, 7000
    x, y = g0.random(M), g0.random(N)
    a1, a2 = g0.standard_normal(N), g0.standard_normal(N)
    say("[gpu] eval then eval_sorted with new strengths")
    p = fgt.plan(1e-4, 6)
    X, Y = to_dev(x, torch.float64), to_dev(y, torch.float64)
    ws = fgt.workspace(p, M, N, X.device)
    fgt.eval(X, Y, to_dev(a1, torch.float64), p, ws=ws)
    u2s = fgt.eval_sorted(to_dev(a2, torch.float64), p, ws, M).cpu().numpy()
    u2 = fgt.eval(X, Y, to_dev(a2, torch.float64), p).cpu().numpy()
    np.testing.assert_array_equal(u2s, u2)


def test_grad_ties_and_translation_invariance():
    """Coincident points: the sort puts a source before a target, so the pair's
    derivative takes one side's value S'(0+) ~ E'_n (the Gaussian's is 0); the
    two scans take opposite sides, so sum dx + sum dy still vanishes."""
    g0 = np.random.default_rng(10)
    M, N = 2500, 3000
    y = g0.random(N)
    x = np.concatenate([y[:1200], g0.random(M - 1200)])
    a, g = g0.standard_normal(N), g0.standard_normal(M)
    (da, dx, dy, dd), _, p, st = gpu_backward(x, y, a, g, 1e-3, 6, case="ties")
    assert st == fgt.FGT_OK
    # one extra E'_n per coincident pair on top of the 2 E'_n bound
    check_all((da, dx, dy, dd), x, y, a, g, p, soe=False, factor=3.0, case="ties")
    s = dx.sum() + dy.sum()
    scale = np.abs(dx).sum() + np.abs(dy).sum()
    say(f"   sum dx + sum dy = {s:.3e} (scale {scale:.3e})")
    assert abs(s) <= 1e-12 * scale


def test_grad_all_points_equal():
    M, N = 700, 900
    x = np.full(M, 0.25)
    y = np.full(N, 0.25)
    g0 = np.random.default_rng(11)
    a, g = g0.standard_normal(N), g0.standard_normal(M)
    (da, dx, dy, dd), _, p, st = gpu_backward(x, y, a, g, 1e-2, 6, case="all-equal")
    assert st == fgt.FGT_OK
    np.testing.assert_allclose(da, np.full(N, g.sum()), rtol=0, atol=2 * oracle_E(p) * np.abs(g).sum())
    ep = oracle_Eprime(p) / 0.1
    assert np.all(np.abs(dx) <= np.abs(g) * ep * np.abs(a).sum())
    assert np.all(np.abs(dy) <= np.abs(a) * ep * np.abs(g).sum())


@pytest.mark.parametrize("M,N", [(0, 50), (40, 0), (0, 0)])
def test_grad_empty(M, N):
    say(f"[gpu] fgt_backward empty M={M} N={N}")
    p = fgt.plan(1e-3, 6)
    g0 = np.random.default_rng(12)
    X, Y = to_dev(g0.random(M), torch.float64), to_dev(g0.random(N), torch.float64)
    A, G = to_dev(g0.standard_normal(N), torch.float64), to_dev(g0.standard_normal(M), torch.float64)
    da, dx, dy, dd = fgt.backward(X, Y, A, G, p)
    assert torch.all(da == 0) and torch.all(dx == 0) and torch.all(dy == 0) and float(dd) == 0.0
    assert da.shape == (N,) and dx.shape == (M,) and dy.shape == (N,)


# ---------------------------------------------------------------------------
# FP32
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("digits", [3, 4, 6])
def test_grad_fp32(digits):
    g0 = np.random.default_rng(2000 + digits)
    M, N = 3001, 4093
    delta = 1e-4
    x = g0.random(M).astype(np.float32).astype(np.float64)
    y = g0.random(N).astype(np.float32).astype(np.float64)
    a = g0.standard_normal(N).astype(np.float32).astype(np.float64)
    g = g0.standard_normal(M).astype(np.float32).astype(np.float64)
    got, _, p, st = gpu_backward(x, y, a, g, delta, digits, dtype=torch.float32, case="fp32")
    assert st == fgt.FGT_OK
    check_all(got, x, y, a, g, p, eps=EPS32, case=f"fp32 digits={digits}")


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------

def test_autograd_matches_backward_and_oracle():
    g0 = np.random.default_rng(13)
    M, N = 2000, 2600
    delta = 1e-3
    x, y = g0.random(M), g0.random(N)
    a, g = g0.standard_normal(N), g0.standard_normal(M)
    say("[gpu] gauss_transform autograd")
    X = to_dev(x, torch.float64).requires_grad_()
    Y = to_dev(y, torch.float64).requires_grad_()
    A = to_dev(a, torch.float64).requires_grad_()
    D = torch.tensor(delta, dtype=torch.float64, device="cuda", requires_grad=True)
    G = to_dev(g, torch.float64)
    u = fgt.gauss_transform(X, Y, A, D, 9)
    (u * G).sum().backward()
    got = (A.grad.cpu().numpy(), X.grad.cpu().numpy(), Y.grad.cpu().numpy(), float(D.grad))
    p = fgt.plan(delta, 9)
    ref, _, _, _ = fgt.backward(X.detach(), Y.detach(), A.detach(), G, p)
    np.testing.assert_array_equal(got[0], ref.cpu().numpy())
    check_all(got, x, y, a, g, p, case="autograd")


def test_autograd_partial_requirements():
    g0 = np.random.default_rng(14)
    M, N = 500, 700
    x, y = g0.random(M), g0.random(N)
    a = g0.standard_normal(N)
    say("[gpu] gauss_transform autograd, alpha only")
    X, Y = to_dev(x, torch.float64), to_dev(y, torch.float64)
    A = to_dev(a, torch.float64).requires_grad_()
    u = fgt.gauss_transform(X, Y, A, 1e-3, 6)
    u.sum().backward()
    ref = oracle.direct(y, x, np.ones(M), 1e-3)
    p = fgt.plan(1e-3, 6)
    assert np.max(np.abs(A.grad.cpu().numpy() - ref)) <= 2 * oracle_E(p) * M


def test_autograd_reuses_plan_and_workspace():
    """A second forward of the same shape allocates only its output; forwards
    that share the cached workspace before their backwards still get their own
    gradients (the later backward sorts again)."""
    g0 = np.random.default_rng(16)
    M, N = 30000, 40000
    delta = 1e-3
    say("[gpu] gauss_transform workspace cache")
    fgt.api._gt_cache.clear()
    Y = to_dev(g0.random(N), torch.float64)
    A = to_dev(g0.standard_normal(N), torch.float64)
    X1 = to_dev(g0.random(M), torch.float64)
    X2 = to_dev(g0.random(M), torch.float64)
    G = to_dev(g0.standard_normal(M), torch.float64)
    u1 = fgt.gauss_transform(X1, Y, A, delta, 6)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    u2 = fgt.gauss_transform(X2, Y, A, delta, 6)
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - m0
    assert grown <= ((M * 8 + 511) // 512) * 512, grown
    # interleaved: forward 1, forward 2 (same cached workspace), backward 1, backward 2
    x1 = X1.clone().requires_grad_()
    x2 = X2.clone().requires_grad_()
    a1 = A.clone().requires_grad_()
    a2 = A.clone().requires_grad_()
    v1 = fgt.gauss_transform(x1, Y, a1, delta, 6)
    v2 = fgt.gauss_transform(x2, Y, a2, delta, 6)
    (v1 * G).sum().backward()
    (v2 * G).sum().backward()
    p = fgt.plan(delta, 6)
    for xs, xg, ag in ((X1, x1.grad, a1.grad), (X2, x2.grad, a2.grad)):
        da, dx, _, _ = fgt.backward(xs, Y, A, G, p)
        np.testing.assert_allclose(xg.cpu().numpy(), dx.cpu().numpy(), rtol=0,
                                   atol=1e-12 * float(dx.abs().max()))
        np.testing.assert_allclose(ag.cpu().numpy(), da.cpu().numpy(), rtol=0,
                                   atol=1e-12 * float(da.abs().max()))
    np.testing.assert_array_equal(u1.cpu().numpy(), v1.detach().cpu().numpy())
    np.testing.assert_array_equal(u2.cpu().numpy(), v2.detach().cpu().numpy())


def test_gradcheck_tiny():
    g0 = np.random.default_rng(15)
    say("[gpu] torch.autograd.gradcheck, 11 digits")
    X = to_dev(g0.random(7), torch.float64).requires_grad_()
    Y = to_dev(g0.random(9), torch.float64).requires_grad_()
    A = to_dev(g0.standard_normal(9), torch.float64).requires_grad_()
    D = torch.tensor(0.02, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x, y, a, d: fgt.gauss_transform(x, y, a, d, 11),
                                    (X, Y, A, D), eps=1e-6, atol=1e-6, rtol=1e-5)


# ---------------------------------------------------------------------------
# full size: N = M = 2^22 uniform, delta = 1e-4, FP64 at 9 digits, FP32 at 4
# ---------------------------------------------------------------------------

_big = {}


def big():
    if "p" not in _big:
        _big["p"] = W.grad_problem()
    return _big["p"]


def test_grad_full_size_fp64():
    pr, g = big()
    delta, digits = pr.delta, pr.digits
    (da, dx, dy, dd), u, p, st = gpu_backward(pr.x, pr.y, pr.alpha, g, delta, digits, case="full")
    assert st == fgt.FGT_OK
    P = pr.M + pr.N
    t = oracle_table(p)
    # every point against O2 with derivative weights, and the transposed O2
    say("   O2 derivative fields on every point ...")
    r_dx = g * oracle.soe_recurrence_deriv(pr.x, pr.y, pr.alpha, delta, t["tau0"], t["omega"])
    r_dy = pr.alpha * oracle.soe_recurrence_deriv(pr.y, pr.x, g, delta, t["tau0"], t["omega"])
    r_da = oracle.soe_recurrence(pr.y, pr.x, g, delta, t["tau0"], t["omega"])
    e_da = np.max(np.abs(da - r_da)) / impl_tol(g, p, P)
    e_dx = np.max(np.abs(dx - r_dx) / (np.abs(g) * impl_tol_der(pr.alpha, p, P)))
    e_dy = np.max(np.abs(dy - r_dy) / (np.abs(pr.alpha) * impl_tol_der(g, p, P)))
    c = 0.5 * (min(pr.x.min(), pr.y.min()) + max(pr.x.max(), pr.y.max()))
    r_dd = -(np.dot(pr.x - c, r_dx) + np.dot(pr.y - c, r_dy)) / (2 * delta)
    tdd = (np.dot(np.abs(pr.x - c), np.abs(g)) * impl_tol_der(pr.alpha, p, P)
           + np.dot(np.abs(pr.y - c), np.abs(pr.alpha)) * impl_tol_der(g, p, P)) / (2 * delta)
    e_dd = abs(dd - r_dd) / tdd
    say(f"   vs O2 (all points), err/tol: dalpha {e_da:.2e} dx {e_dx:.2e} dy {e_dy:.2e} ddelta {e_dd:.2e}")
    assert max(e_da, e_dx, e_dy, e_dd) <= 1.0
    # 4096 sampled targets and sources against the direct Gaussian gradients
    ti = W.sample_indices(pr.M, 4096, cfg=5, sub=1)
    sj = W.sample_indices(pr.N, 4096, cfg=5, sub=2)
    o_da, o_dx, o_dy, _ = oracle.direct_gradients(pr.x, pr.y, pr.alpha, g, delta, targets=ti, sources=sj)
    sa, sg = np.abs(pr.alpha).sum(), np.abs(g).sum()
    ep = oracle_Eprime(p) / math.sqrt(delta)
    r1 = np.max(np.abs(da[sj] - o_da)) / (2 * oracle_E(p) * sg)
    r2 = np.max(np.abs(dx[ti] - o_dx) / (np.abs(g[ti]) * 2 * ep * sa))
    r3 = np.max(np.abs(dy[sj] - o_dy) / (np.abs(pr.alpha[sj]) * 2 * ep * sg))
    say(f"   vs direct gradients (4096 sampled), err/bound: dalpha {r1:.3e} dx {r2:.3e} dy {r3:.3e}")
    assert max(r1, r2, r3) <= 1.0


def test_grad_full_size_ddelta_finite_difference():
    pr, g = big()
    delta, digits = pr.delta, pr.digits
    X, Y, A, G = (to_dev(v, torch.float64) for v in (pr.x, pr.y, pr.alpha, g))
    D = torch.tensor(delta, dtype=torch.float64, device="cuda", requires_grad=True)
    say("[gpu] full-size dL/ddelta vs central differences of the forward")
    u = fgt.gauss_transform(X, Y, A, D, digits)
    (u * G).sum().backward()
    h = 1e-4 * delta
    lp = float((fgt.gauss_transform(X, Y, A, delta + h, digits) * G).sum())
    lm = float((fgt.gauss_transform(X, Y, A, delta - h, digits) * G).sum())
    fd = (lp - lm) / (2 * h)
    err = abs(float(D.grad) - fd) / abs(fd)
    say(f"   dL/ddelta {float(D.grad):.10e} vs FD {fd:.10e}: rel {err:.2e}")
    assert err <= 1e-6


def test_grad_full_size_fp32_4digits():
    pr, g = big()
    delta = pr.delta
    x32 = pr.x.astype(np.float32).astype(np.float64)
    y32 = pr.y.astype(np.float32).astype(np.float64)
    a32 = pr.alpha.astype(np.float32).astype(np.float64)
    g32 = g.astype(np.float32).astype(np.float64)
    (da, dx, dy, dd), _, p, st = gpu_backward(x32, y32, a32, g32, delta, 4, dtype=torch.float32,
                                              case="full fp32")
    assert st == fgt.FGT_OK
    P = pr.M + pr.N
    ti = W.sample_indices(pr.M, 4096, cfg=5, sub=3)
    sj = W.sample_indices(pr.N, 4096, cfg=5, sub=4)
    o_da, o_dx, o_dy, _ = oracle.direct_gradients(x32, y32, a32, g32, delta, targets=ti, sources=sj)
    sa, sg = np.abs(a32).sum(), np.abs(g32).sum()
    ep = oracle_Eprime(p) / math.sqrt(delta)
    m1 = np.max(np.abs(da[sj] - o_da)) / sg
    m2 = np.max(np.abs(dx[ti] - o_dx) / np.abs(g32[ti])) / (sa / math.sqrt(delta))
    m3 = np.max(np.abs(dy[sj] - o_dy) / np.abs(a32[sj])) / (sg / math.sqrt(delta))
    say(f"   fp32 4 digits, measured max err: dalpha {m1:.3e} x sum|g| (E {oracle_E(p):.2e}); "
        f"dx {m2:.3e}, dy {m3:.3e} x sum|w|/sqrt(delta) (E' {oracle_Eprime(p):.2e})")
    r1 = np.max(np.abs(da[sj] - o_da)) / (2 * oracle_E(p) * sg + impl_tol(g32, p, P, EPS32))
    r2 = np.max(np.abs(dx[ti] - o_dx) / (np.abs(g32[ti]) * (2 * ep * sa + impl_tol_der(a32, p, P, EPS32))))
    r3 = np.max(np.abs(dy[sj] - o_dy) / (np.abs(a32[sj]) * (2 * ep * sg + impl_tol_der(g32, p, P, EPS32))))
    assert max(r1, r2, r3) <= 1.0


def test_partial_requests_match_full():
    """Any subset of outputs gives the same values as the full request."""
    g0 = np.random.default_rng(16)
    M, N = 6000, 5000
    x, y = g0.random(M), g0.random(N)
    a, g = g0.standard_normal(N), g0.standard_normal(M)
    say("[gpu] fgt_backward partial requests")
    p = fgt.plan(1e-4, 6)
    X, Y, A, G = (to_dev(v, torch.float64) for v in (x, y, a, g))
    ws = fgt.workspace(p, M, N, X.device)
    fgt.eval(X, Y, A, p, ws=ws)
    full = fgt.backward(X, Y, A, G, p, ws=ws, sorted=True)
    only_dd = fgt.backward(X, Y, A, G, p, ws=ws, sorted=True, dalpha=False, dx=False, dy=False)
    only_da = fgt.backward(X, Y, A, G, p, ws=ws, sorted=True, dx=False, dy=False, ddelta=False)
    only_dx = fgt.backward(X, Y, A, G, p, ws=ws, sorted=True, dalpha=False, dy=False, ddelta=False)
    assert only_dd[:3] == (None, None, None) and float(only_dd[3]) == float(full[3])
    assert torch.equal(only_da[0], full[0]) and only_da[1] is None
    assert torch.equal(only_dx[1], full[1]) and only_dx[2] is None
