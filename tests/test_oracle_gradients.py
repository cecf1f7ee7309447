"""Pins of the gradient oracle (O4: direct gradients, O5: SOE derivative field).

L = sum_i g_i u_i with u from (1.1)-(1.2).  The pins are facts that do not
depend on the oracle's own formulas:
  * central finite differences of the forward oracle O1 (itself pinned in
    test_oracle_pins.py) in every coordinate, strength and delta;
  * translation invariance (u depends on x_i - y_j only):   sum dx + sum dy = 0;
  * the scaling identity u(c x, c y; c^2 delta) = u(x, y; delta):
        2 delta dL/ddelta + sum x dx + sum y dy = 0;
  * bilinearity: sum_j alpha_j dL/dalpha_j = L = g . u;
  * for the SOE field, finite differences of O3 away from coincident points,
    the table's derivative bound E'_n against O4, oddness (a configuration
    symmetric about a target has zero field there, coincident source included).
Each planted mistake in O4/O5 fails at least one of these.
"""
import numpy as np
import pytest

import oracle


def problem(seed, M=30, N=34, delta=2e-3, spread=0.3):
    g = np.random.default_rng(seed)
    x = g.uniform(0, spread, M)
    y = g.uniform(0, spread, N)
    alpha = g.standard_normal(N)
    gg = g.standard_normal(M)
    return x, y, alpha, gg, delta


def loss(x, y, alpha, g, delta):
    return float(np.dot(g, oracle.direct(x, y, alpha, delta, cutoff=0)))


def fd_gradients(x, y, alpha, g, delta):
    """Central differences of L through O1 (step sizes relative to the scale sqrt(delta))."""
    h = 1e-5 * np.sqrt(delta)
    dx = np.empty_like(x)
    for i in range(x.size):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        dx[i] = (loss(xp, y, alpha, g, delta) - loss(xm, y, alpha, g, delta)) / (2 * h)
    dy = np.empty_like(y)
    for j in range(y.size):
        yp, ym = y.copy(), y.copy()
        yp[j] += h
        ym[j] -= h
        dy[j] = (loss(x, yp, alpha, g, delta) - loss(x, ym, alpha, g, delta)) / (2 * h)
    da = np.empty_like(alpha)
    for j in range(alpha.size):
        ap, am = alpha.copy(), alpha.copy()
        ap[j] += 1.0
        am[j] -= 1.0
        da[j] = (loss(x, y, ap, g, delta) - loss(x, y, am, g, delta)) / 2.0
    hd = 1e-5 * delta
    dd = (loss(x, y, alpha, g, delta + hd) - loss(x, y, alpha, g, delta - hd)) / (2 * hd)
    return da, dx, dy, dd


def rel(a, b):
    a, b = np.atleast_1d(a), np.atleast_1d(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------------------
# pins of O4, each returning (ok, detail)
# ---------------------------------------------------------------------------

def pin_finite_differences(plant=0):
    x, y, a, g, delta = problem(1)
    got = oracle.direct_gradients(x, y, a, g, delta, plant=plant)
    ref = fd_gradients(x, y, a, g, delta)
    errs = [rel(got[k], ref[k]) for k in range(4)]
    return max(errs) < 1e-6, "fd rel errs " + ", ".join(f"{e:.1e}" for e in errs)


def pin_translation(plant=0):
    x, y, a, g, delta = problem(2)
    _, dx, dy, _ = oracle.direct_gradients(x, y, a, g, delta, plant=plant)
    s = dx.sum() + dy.sum()
    scale = np.abs(dx).sum() + np.abs(dy).sum()
    return abs(s) <= 1e-13 * scale, f"sum dx + sum dy = {s:.2e} (scale {scale:.2e})"


def pin_scaling(plant=0):
    x, y, a, g, delta = problem(3)
    _, dx, dy, dd = oracle.direct_gradients(x, y, a, g, delta, plant=plant)
    lhs = 2 * delta * dd
    rhs = -(np.dot(x, dx) + np.dot(y, dy))
    return abs(lhs - rhs) <= 1e-12 * max(abs(rhs), 1e-300), f"2 delta dL/ddelta {lhs:.6e} vs {rhs:.6e}"


def pin_bilinear(plant=0):
    x, y, a, g, delta = problem(4)
    da, _, _, _ = oracle.direct_gradients(x, y, a, g, delta, plant=plant)
    L = loss(x, y, a, g, delta)
    return abs(np.dot(a, da) - L) <= 1e-13 * np.abs(a).sum() * np.abs(g).sum(), "alpha . dalpha = L"


GRAD_PINS = {"fd": pin_finite_differences, "translation": pin_translation,
             "scaling": pin_scaling, "bilinear": pin_bilinear}


@pytest.mark.parametrize("name", list(GRAD_PINS))
def test_gradient_pin(name):
    ok, detail = GRAD_PINS[name]()
    assert ok, detail


def test_gradient_subsets_match_full():
    x, y, a, g, delta = problem(5)
    full = oracle.direct_gradients(x, y, a, g, delta)
    ti, sj = np.array([3, 0, 17]), np.array([5, 33, 2])
    part = oracle.direct_gradients(x, y, a, g, delta, targets=ti, sources=sj)
    np.testing.assert_array_equal(part[0], full[0][sj])
    np.testing.assert_array_equal(part[1], full[1][ti])
    np.testing.assert_array_equal(part[2], full[2][sj])
    assert part[3] is None


@pytest.mark.parametrize("plant", [1, 2, 3])
def test_planted_gradient_mistake_is_caught(plant):
    failed = [n for n, f in GRAD_PINS.items() if not f(plant)[0]]
    assert failed, f"plant {plant} passed every gradient pin"


# ---------------------------------------------------------------------------
# pins of O5 (the SOE derivative field)
# ---------------------------------------------------------------------------

def soe_fd(x, y, w, delta, tau0, omega):
    h = 1e-6 * np.sqrt(delta)
    return (oracle.soe_brute(x + h, y, w, delta, tau0, omega)
            - oracle.soe_brute(x - h, y, w, delta, tau0, omega)) / (2 * h)


def pin_soe_fd(otables, plant=0):
    x, y, a, _, delta = problem(6)
    t = otables[4]
    d = oracle.soe_deriv_brute(x, y, a, delta, t["tau0"], t["omega"], plant=plant)
    ref = soe_fd(x, y, a, delta, t["tau0"], t["omega"])
    e = rel(d, ref)
    return e < 1e-6, f"SOE field vs FD of O3: {e:.1e}"


def pin_soe_odd_with_tie(otables, plant=0):
    """Sources placed symmetrically about the target, one on it: the field is zero."""
    t = otables[4]
    delta = 1e-3
    off = np.array([0.01, 0.03, 0.05, 0.08])
    x = np.array([0.5])
    y = np.concatenate([0.5 - off, [0.5], 0.5 + off])
    w = np.concatenate([np.ones(4) * 0.7, [2.0], np.ones(4) * 0.7])
    d = oracle.soe_deriv_brute(x, y, w, delta, t["tau0"], t["omega"], plant=plant)
    scale = np.abs(w).sum() / np.sqrt(delta)
    return abs(d[0]) <= 1e-13 * scale, f"field at centre {d[0]:.2e}"


def pin_soe_vs_gaussian(otables, plant=0):
    """|sum w S' - sum w G'| <= E'_n / sqrt(delta) sum |w| (table bound, delta = 1 units)."""
    x, y, a, _, delta = problem(7, M=60, N=50)
    worst = 0.0
    for m in (2, 4, 6):
        t = otables[m]
        d = oracle.soe_deriv_brute(x, y, a, delta, t["tau0"], t["omega"], plant=plant)
        ref = oracle._field(x, y, a, delta, 1)
        ratio = np.max(np.abs(d - ref)) / (t["Eprime"] / np.sqrt(delta) * np.abs(a).sum())
        worst = max(worst, ratio)
    return worst <= 1.0, f"worst |S'-G'| / bound = {worst:.3f}"


SOE_PINS = {"fd": pin_soe_fd, "odd_tie": pin_soe_odd_with_tie, "gaussian": pin_soe_vs_gaussian}


@pytest.mark.parametrize("name", list(SOE_PINS))
def test_soe_field_pin(otables, name):
    ok, detail = SOE_PINS[name](otables)
    assert ok, detail


@pytest.mark.parametrize("plant", [1, 2])
def test_planted_soe_field_mistake_is_caught(otables, plant):
    failed = [n for n, f in SOE_PINS.items() if not f(otables, plant)[0]]
    assert failed, f"plant {plant} passed every SOE field pin"


# ---------------------------------------------------------------------------
# O2 with derivative weights, pinned to O5 (itself pinned above)
# ---------------------------------------------------------------------------

def pin_recurrence_deriv(otables, plant=0):
    worst = 0.0
    for seed, (M, N, delta, m) in enumerate([(40, 50, 2e-3, 4), (33, 17, 1e-4, 6), (25, 60, 1.0, 2)]):
        x, y, a, _, _ = problem(20 + seed, M=M, N=N, delta=delta)
        t = otables[m]
        d = oracle.soe_recurrence_deriv(x, y, a, delta, t["tau0"], t["omega"], plant=plant)
        ref = oracle.soe_deriv_brute(x, y, a, delta, t["tau0"], t["omega"])
        scale = np.abs(a).sum() * np.sum(np.abs(t["tau0"] * t["omega"])) / np.sqrt(delta)
        worst = max(worst, float(np.max(np.abs(d - ref))) / scale)
    return worst < 1e-13, f"O2' vs O5: {worst:.2e}"


def test_recurrence_deriv_pin(otables):
    ok, detail = pin_recurrence_deriv(otables)
    assert ok, detail


@pytest.mark.parametrize("plant", [2, 3, 4, 5, 6, 7])
def test_planted_recurrence_deriv_mistake_is_caught(otables, plant):
    ok, detail = pin_recurrence_deriv(otables, plant)
    assert not ok, f"plant {plant} passed: {detail}"
