"""ORACLE -- sum-of-exponentials (SOE) tables for the Gaussian, built from the paper.

Test infrastructure only (see ``oracle/__init__.py``).  Shares no code with
the GPU library's own table generator.

Steps, in the paper's order:

1. Integral representation (2.2): G(x; delta) is the contour integral
   (1/(2 pi i)) int_Gamma e^z sqrt(pi/z) exp(-sqrt(z)|x|/sqrt(delta)) dz over a
   contour that starts at -infinity in the third quadrant, winds around 0 and
   returns to -infinity in the second quadrant (principal square root).
2. The stabilised hyperbolic contour of Section 3.4:
   z(u) = lambda (1 - sin(0.8 + i u)), a = acosh(2/((1-theta) sin 0.8)),
   lambda = 0.6 pi (1-theta) n / a, h = 2a/n, theta = 1/4 (n <= 16) else 12/n.
3. Midpoint rule (2.7) on u in [-a, a], giving the SOE (2.8) with the weights
   and nodes of (2.9).  As u increases, z(u) runs from the second quadrant
   to the third, the reverse of the orientation (2.2) asks for, so every
   weight of (2.9) changes sign (reading: S_n(0) must be +1, not -1).
4. Balanced truncation (Section 2.4) of the SOE viewed as the impulse
   response C exp(A x) B of A = diag(-t), B = 1, C = w: Gramians
   P_jk = 1/(t_j + conj t_k), Q_jk = conj(w_j) w_k / (conj t_j + t_k),
   square-root projection on the leading Hankel singular values, then
   diagonalisation of the reduced A to read off new nodes and weights.
5. Keep one node of each conjugate pair (Im t > 0) with its weight doubled
   (Section 1, after (1.3)); the transform takes the real part.
6. E_n by (3.1): delta = 1, x = 0 and 100,000 log-spaced points on
   [1e-5, 1e2].

Everything before step 5 runs in mpmath at ``DPS`` decimal digits; the
Gramians are numerically singular in double precision.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

DPS = 130
PHASE = "0.8"          # the 0.8 in z(u) = lambda (1 - sin(0.8 + i u)), Section 3.4
CONTOUR_N = 48         # nodes on the contour before reduction


def contour_parameters(n: int):
    """theta, a, lambda, h of the Section 3.4 hyperbolic contour (mp numbers)."""
    theta = mp.mpf(1) / 4 if n <= 16 else mp.mpf(12) / n
    s08 = mp.sin(mp.mpf(PHASE))
    a = mp.acosh(2 / ((1 - theta) * s08))
    lam = mp.mpf("0.6") * mp.pi * (1 - theta) * n / a
    h = 2 * a / n
    return theta, a, lam, h


def contour_point(u, lam):
    """z(u) and z'(u) for z(u) = lambda (1 - sin(0.8 + i u))."""
    arg = mp.mpf(PHASE) + 1j * u
    z = lam * (1 - mp.sin(arg))
    dz = -1j * lam * mp.cos(arg)
    return z, dz


def contour_integrand(u, x, lam, delta=1):
    """Integrand of (2.4)-(2.6) for the Gaussian, with the orientation of (2.2).

    (1/(2 pi i)) e^z f(z) dz/du with f of (2.5), times -1 because increasing
    u traverses the contour backwards.
    """
    z, dz = contour_point(u, lam)
    f = mp.sqrt(mp.pi / z) * mp.exp(-mp.sqrt(z) * abs(x) / mp.sqrt(delta))
    return -mp.exp(z) * f * dz / (2j * mp.pi)


def contour_soe(n: int = CONTOUR_N):
    """Midpoint discretisation (2.7)-(2.9) of the Section 3.4 contour; mp lists (t, w)."""
    with mp.workdps(DPS):
        _, a, lam, h = contour_parameters(n)
        t, w = [], []
        for k in range(1, n + 1):
            u = -a + (k - mp.mpf(1) / 2) * h
            z, dz = contour_point(u, lam)
            sz = mp.sqrt(z)
            # (2.9) with the orientation sign of (2.2)
            w.append(-h / (2 * mp.sqrt(mp.pi) * 1j) * dz / sz * mp.exp(z))
            t.append(sz)
        return t, w


@functools.lru_cache(maxsize=None)
def _bt_factors(n: int):
    """Cholesky factors and SVD of the balanced-truncation square-root method."""
    t, w = contour_soe(n)
    with mp.workdps(DPS):
        P = mp.matrix(n, n)
        Q = mp.matrix(n, n)
        for j in range(n):
            for k in range(n):
                P[j, k] = 1 / (t[j] + mp.conj(t[k]))
                Q[j, k] = mp.conj(w[j]) * w[k] / (mp.conj(t[j]) + t[k])
        L = mp.cholesky(P)
        R = mp.cholesky(Q)
        U, S, V = mp.svd_c(R.H * L)      # R^H L = U diag(S) V
        return t, w, L, R, U, S, V


def hankel_singular_values(n: int = CONTOUR_N):
    _, _, _, _, _, S, _ = _bt_factors(n)
    return [S[i] for i in range(n)]


def balanced_truncation(r: int, n: int = CONTOUR_N):
    """Reduce the n-term contour SOE to r terms; returns mp lists (t_r, w_r)."""
    t, w, L, R, U, S, V = _bt_factors(n)
    with mp.workdps(DPS):
        Sm = mp.diag([1 / mp.sqrt(S[i]) for i in range(r)])
        Ur = U[:, :r]
        Vr = V[:r, :].H
        T = L * Vr * Sm                 # n x r
        Ti = Sm * Ur.H * R.H            # r x n, Ti T = I
        A = mp.diag([-tk for tk in t])
        Ar = Ti * A * T
        Br = Ti * mp.matrix([1] * n)
        Cr = mp.matrix([w]) * T
        E, X = mp.eig(Ar)
        Xi = mp.inverse(X)
        cx = Cr * X
        xb = Xi * Br
        tr = [-E[i] for i in range(r)]
        wr = [cx[0, i] * xb[i] for i in range(r)]
        return tr, wr


def pair_representatives(t, w, tol: float = 1e-30):
    """One node per conjugate pair (Im t > 0) with doubled weight; real nodes keep w.

    Returns numpy complex128 arrays (tau0, omega).  Raises if the nodes do not
    come in exact conjugate pairs.
    """
    with mp.workdps(DPS):
        reps = []
        for tk, wk in zip(t, w):
            if abs(mp.im(tk)) <= tol * abs(tk):
                reps.append((mp.mpc(mp.re(tk), 0), mp.mpc(mp.re(wk), 0)))
            elif mp.im(tk) > 0:
                partner = min(range(len(t)), key=lambda m: abs(t[m] - mp.conj(tk)))
                if abs(t[partner] - mp.conj(tk)) > 1e-40 * abs(tk) or abs(w[partner] - mp.conj(wk)) > 1e-40 * abs(wk):
                    raise ValueError("nodes/weights are not conjugate pairs")
                reps.append((tk, 2 * wk))
        reps.sort(key=lambda p: float(mp.re(p[0])))
        tau0 = np.array([complex(p[0]) for p in reps])
        omega = np.array([complex(p[1]) for p in reps])
        return tau0, omega


def paper_grid() -> np.ndarray:
    """x = 0 and 100,000 logarithmically spaced points on [1e-5, 1e2], as in (3.1)."""
    return np.concatenate([[0.0], np.logspace(-5.0, 2.0, 100000)])


def soe_value(tau0: np.ndarray, omega: np.ndarray, x: np.ndarray) -> np.ndarray:
    """S_n(x; 1) = Re sum_k omega_k exp(-tau0_k |x|) (complex sum returned)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    out = np.zeros(x.shape, dtype=np.complex128)
    for tk, wk in zip(tau0, omega):
        out += wk * np.exp(-tk * x)
    return out


def table_errors(tau0: np.ndarray, omega: np.ndarray, x: np.ndarray | None = None,
                 plant: int = 0):
    """(E_n, E'_n, max |Im S|) on the (3.1) grid at delta = 1.

    E'_n = sup_{x > 0} |S_n'(x) - G'(x)| with S_n' = -Re sum omega tau0 e^{-tau0 x}
    and G' = -(x/2) e^{-x^2/4}: the maximum over the grid's positive points and
    the one-sided limit x -> 0+, where G'(0) = 0 and S_n'(0+) = -Re sum omega tau0
    (the cusp of the SOE at the origin).  `plant` selects a deliberately wrong
    E'_n (tests only): 1 takes the complex modulus instead of the real part,
    2 drops the factor tau0 of the derivative.
    """
    if x is None:
        x = paper_grid()
    s = soe_value(tau0, omega, x)
    g = np.exp(-x * x / 4.0)
    e = float(np.max(np.abs(s.real - g)))
    xp = x[x > 0]
    ds = np.zeros(xp.shape, dtype=np.complex128)
    for tk, wk in zip(tau0, omega):
        ds += -wk * (tk if plant != 2 else 1.0) * np.exp(-tk * xp)
    dg = -(xp / 2.0) * np.exp(-xp * xp / 4.0)
    if plant == 1:
        ep = float(np.max(np.abs(ds - dg)))
    else:
        ep = float(np.max(np.abs(ds.real - dg)))
    cusp = abs(float(np.sum(np.asarray(omega) * np.asarray(tau0)).real))
    ep = max(ep, cusp)
    return e, ep, float(np.max(np.abs(s.imag)))


def gaussian_table(n_modes: int, n: int = CONTOUR_N) -> dict:
    """SOE table with n_modes conjugate-pair modes (2 n_modes exponentials)."""
    t, w = balanced_truncation(2 * n_modes, n)
    tau0, omega = pair_representatives(t, w)
    e, ep, im = table_errors(tau0, omega)
    return {
        "n_modes": int(n_modes),
        "tau0": tau0,
        "omega": omega,
        "E": e,
        "Eprime": ep,
        "max_imag": im,
        "sum_abs_omega": float(np.sum(np.abs(omega))),
    }


def modes_for_digits(tables: dict, digits: int) -> int:
    """Smallest table whose E_n <= 10^-digits (reading of 'digits')."""
    for m in sorted(tables):
        if tables[m]["E"] <= 10.0 ** (-digits):
            return m
    raise ValueError(f"no table reaches {digits} digits")
