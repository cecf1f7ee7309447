"""Pins of the oracle's SOE tables (Sections 2-3 of the paper).

* the contour of Section 3.4 really represents the Gaussian: adaptive
  quadrature of the integral (2.2) along it returns exp(-x^2/4);
* the printed weights (2.9), taken with u increasing, give S_n(0) = -1, so
  the orientation reading (weights negated) is forced;
* balanced truncation at full rank is a similarity transform (the SOE is
  reproduced), and the Hankel singular values satisfy sum sigma^2 = tr(PQ);
* the reduced tables converge at a rate between the paper's contour+BT rate
  (about 6.3^-n, Section 3.2) and Halphen's bound (9.28903^-n, Section 2.3),
  and meet the Section 3.3 digit claims.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import soe_table as ST


@pytest.mark.parametrize("x", [0.0, 0.7, 2.5, 6.0])
def test_contour_integral_is_the_gaussian(x):
    with mp.workdps(30):
        _, a, lam, _ = ST.contour_parameters(48)
        # beyond |u| = a + 2.5, Re z < -1000: the integrand is below e^-1000
        ends = [-a - mp.mpf(2.5), -a, -a / 2, 0, a / 2, a, a + mp.mpf(2.5)]
        val = mp.quad(lambda u: ST.contour_integrand(u, x, lam), ends)
        assert abs(mp.re(val) - mp.exp(-mp.mpf(x) ** 2 / 4)) < mp.mpf("1e-20")
        assert abs(mp.im(val)) < mp.mpf("1e-20")


def test_printed_orientation_gives_minus_one():
    """(2.9) summed with u increasing gives -G; the oracle's weights are negated."""
    t, w = ST.contour_soe(32)
    with mp.workdps(ST.DPS):
        s0 = mp.fsum(w)
    assert abs(s0 - 1) < 1e-8            # negated weights: S_n(0) = +1
    assert abs((-s0) - 1) > 1.9          # as printed: S_n(0) = -1, not G(0) = 1


def test_midpoint_rule_matches_weights():
    """h * sum of the integrand at the midpoints equals the SOE built from (2.9)."""
    n = 24
    t, w = ST.contour_soe(n)
    with mp.workdps(40):
        _, a, lam, h = ST.contour_parameters(n)
        for x in (0.0, 0.3, 1.7):
            quad = h * mp.fsum(ST.contour_integrand(-a + (k - mp.mpf(1) / 2) * h, x, lam)
                               for k in range(1, n + 1))
            soe = mp.fsum(wk * mp.exp(-tk * x) for tk, wk in zip(t, w))
            assert abs(quad - soe) < mp.mpf("1e-30")


def test_contour_soe_accuracy():
    """The stabilised contour reaches far below the ~13-digit saturation of Section 3.1."""
    t, w = ST.contour_soe(48)
    tau = np.array([complex(v) for v in t])
    om = np.array([complex(v) for v in w])
    e, _, _ = ST.table_errors(tau, om)
    assert e < 1e-11


def test_balanced_truncation_full_rank_is_identity():
    n = 12
    t, w = ST.contour_soe(n)
    tr, wr = ST.balanced_truncation(n, n)
    with mp.workdps(ST.DPS):
        for x in (0.0, 0.4, 2.0):
            a = mp.fsum(wk * mp.exp(-tk * x) for tk, wk in zip(t, w))
            b = mp.fsum(wk * mp.exp(-tk * x) for tk, wk in zip(tr, wr))
            assert abs(a - b) < mp.mpf("1e-60")


def test_hankel_singular_values_trace_identity():
    n = 12
    t, w = ST.contour_soe(n)
    sig = ST.hankel_singular_values(n)
    with mp.workdps(ST.DPS):
        tr = mp.mpf(0)
        for j in range(n):
            for k in range(n):
                p = 1 / (t[j] + mp.conj(t[k]))
                q = mp.conj(w[k]) * w[j] / (mp.conj(t[k]) + t[j])
                tr += p * q
        assert abs(mp.fsum(s ** 2 for s in sig) - tr) < mp.mpf("1e-60") * abs(tr)


def test_grid_is_the_papers():
    g = ST.paper_grid()
    assert g.shape == (100001,)
    assert g[0] == 0.0 and g[1] == pytest.approx(1e-5) and g[-1] == pytest.approx(1e2)
    r = g[2:] / g[1:-1]
    assert np.allclose(r, r[0])


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7])
def test_table_properties(otables, m):
    t = otables[m]
    tau0, om = t["tau0"], t["omega"]
    e, ep, _ = ST.table_errors(tau0, om)
    assert e == pytest.approx(t["E"], rel=1e-9)
    assert np.all(tau0.real > 0)
    assert np.all(tau0.imag >= 0)
    assert abs(float(np.sum(om).real) - 1.0) <= e * (1 + 1e-9)
    assert t["Eprime"] == pytest.approx(ep, rel=1e-9)


def test_fixture_matches_a_fresh_build(otables):
    t = ST.gaussian_table(3)
    np.testing.assert_allclose(t["tau0"], otables[3]["tau0"], rtol=1e-14, atol=0)
    np.testing.assert_allclose(t["omega"], otables[3]["omega"], rtol=1e-13, atol=0)


def test_convergence_rate_between_paper_bounds(otables, paper):
    """Fitted rate per exponential (n = 2 n_e) over n_e = 2..6."""
    ne = np.arange(2, 7)
    logs = np.log([otables[m]["E"] for m in ne])
    slope = np.polyfit(2 * ne, logs, 1)[0]
    rate = math.exp(-slope)
    assert paper["rates"]["bt_contour_rate"] <= rate <= paper["rates"]["halphen"], rate


def test_digit_claims(otables, paper):
    c = paper["digits_claims"]
    assert otables[c["modes_for_4_digits"]]["E"] <= 1e-4
    assert otables[c["modes_for_10_digits"]]["E"] <= 1e-10
    assert ST.modes_for_digits(otables, 3) == 2
    assert ST.modes_for_digits(otables, 6) == 4
    assert ST.modes_for_digits(otables, 9) == 6


# ---------------------------------------------------------------------------
# E'_n pinned from both sides by a route other than the derivative formula:
# slopes of the error function eps(x) = S_n(x) - G(x) itself, taken as forward
# difference quotients in mpmath (step 1e-20 at 50 digits, so the quotient is
# the derivative to ~1e-17 absolute).  By the mean value theorem every quotient
# is a value of eps', so their maximum is a lower bound of sup|eps'|; on a grid
# this dense (and at x = 0, where the quotient is the one-sided slope of the
# cusp, G'(0) = 0) it is also within a fraction of a percent of it.  A planted
# inflation of E'_n (the complex modulus instead of the real part, or a dropped
# factor tau0) misses the window by orders of magnitude.
# ---------------------------------------------------------------------------
def fd_slope_sup(tau0, omega, dps=50):
    with mp.workdps(dps):
        ts = [mp.mpc(complex(t)) for t in tau0]
        ws = [mp.mpc(complex(w)) for w in omega]
        h = mp.mpf("1e-20")

        def eps(x):
            return mp.re(mp.fsum(w * mp.exp(-t * x) for t, w in zip(ts, ws))) - mp.exp(-x * x / 4)

        xs = ([mp.mpf(0)] + [mp.mpf(float(v)) for v in np.linspace(0.002, 2.0, 1000)]
              + [mp.mpf(float(v)) for v in np.linspace(2.01, 30.0, 2800)])
        return float(max(abs((eps(x + h) - eps(x)) / h) for x in xs))


FD_SUP = {}


def _fd(otables, m):
    if m not in FD_SUP:
        FD_SUP[m] = fd_slope_sup(otables[m]["tau0"], otables[m]["omega"])
    return FD_SUP[m]


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7])
def test_deriv_error_pinned_by_slopes(otables, m):
    fd = _fd(otables, m)
    ep = otables[m]["Eprime"]
    assert fd * (1 - 1e-6) <= ep <= fd * 1.005, (ep, fd)


@pytest.mark.parametrize("plant", [1, 2])
@pytest.mark.parametrize("m", [2, 4, 6])
def test_planted_deriv_error_is_caught(otables, m, plant):
    t = otables[m]
    _, ep, _ = ST.table_errors(t["tau0"], t["omega"], plant=plant)
    fd = _fd(otables, m)
    assert not (fd * (1 - 1e-6) <= ep <= fd * 1.005), (plant, ep, fd)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
def test_deriv_error_is_the_cusp(otables, m):
    """Up to 6 modes the largest slope error sits at the origin: E'_n = |Re sum omega tau0|."""
    t = otables[m]
    cusp = abs(float(np.sum(t["omega"] * t["tau0"]).real))
    assert t["Eprime"] == pytest.approx(cusp, rel=1e-12)
    assert _fd(otables, m) == pytest.approx(cusp, rel=1e-6)
