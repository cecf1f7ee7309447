"""Build the SOE tables the library ships and write them as C source.

Offline, build-time only (mpmath, no GPU).  Output:

* ``paper_1909_09825_amd/csrc/soe_tables.inc`` -- hex-float constants compiled
  into the library;
* ``paper_1909_09825_amd/soe/soe_tables.json`` -- the same numbers, readable.

Construction (the paper's Sections 2.2, 2.4 and 3.4):

* Discretise the Laplace-type representation (2.2) of the Gaussian on the
  stabilised hyperbolic contour z(u) = lam (1 - sin(0.8 + i u)) with the
  midpoint rule: n = 48 nodes on [-a, a], a = acosh(2 / ((1 - th) sin 0.8)),
  lam = 0.6 pi (1 - th) n / a, th = 12/n.  Weights and nodes follow (2.9);
  the sign is flipped because increasing u runs the contour against the
  orientation (2.2) requires, which is what makes the sum equal +G(0).
* Reduce with square-root balanced truncation (Section 2.4) to 2 m
  exponentials for m = 1..7, in high precision (the Gramians are
  numerically singular in double precision).
* Keep one node per conjugate pair (Im > 0) and double its weight; the
  kernels take the real part of the mode sum (Section 1, after (1.3)).
* Measure E_m on the grid of (3.1) (delta = 1, x = 0 and 1e5 log-spaced
  points on [1e-5, 1e2]) and on a denser check grid; the shipped bound is
  the larger of the two plus a relative margin of 1e-3 (the sup between grid
  points is slightly larger than any grid maximum).  E'_m, the derivative
  error, is measured the same way, with a margin of 1e-2.

Run from the repository root:  python -m paper_1909_09825_amd.soe.gen_tables
"""
from __future__ import annotations

import json
import os

import mpmath as mp
import numpy as np

PREC = 130
N_CONTOUR = 48
MAX_MODES = 7

_HERE = os.path.dirname(os.path.abspath(__file__))
_CSRC = os.path.join(os.path.dirname(_HERE), "csrc")


def _contour(n):
    th = mp.mpf(12) / n if n > 16 else mp.mpf(1) / 4
    phi = mp.mpf("0.8")
    a = mp.acosh(2 / ((1 - th) * mp.sin(phi)))
    lam = mp.mpf(6) / 10 * mp.pi * (1 - th) * n / a
    step = 2 * a / n
    nodes, weights = [], []
    for k in range(n):
        u = -a + (k + mp.mpf(1) / 2) * step
        s = phi + mp.mpc(0, u)
        z = lam * (1 - mp.sin(s))
        dzdu = mp.mpc(0, -1) * lam * mp.cos(s)
        root = mp.sqrt(z)
        # (2.9): h z'(u) e^z / (2 sqrt(pi) i sqrt(z)), negated for the orientation
        weights.append(step * dzdu * mp.exp(z) / (2 * mp.sqrt(mp.pi) * root) * mp.mpc(0, 1))
        nodes.append(root)
    return nodes, weights


def _reduce_all(nodes, weights, ranks):
    """Square-root balanced truncation of sum_k w_k exp(-t_k x) to each rank in `ranks`."""
    n = len(nodes)
    gram_c = mp.matrix(n, n)   # controllability: B = ones
    gram_o = mp.matrix(n, n)   # observability:   C = weights
    for i in range(n):
        for j in range(n):
            gram_c[i, j] = 1 / (nodes[i] + mp.conj(nodes[j]))
            gram_o[i, j] = mp.conj(weights[i]) * weights[j] / (mp.conj(nodes[i]) + nodes[j])
    lc = mp.cholesky(gram_c)
    lo = mp.cholesky(gram_o)
    u, sv, vh = mp.svd_c(lo.H * lc)
    a_full = mp.diag([-t for t in nodes])
    ones = mp.matrix([1] * n)
    crow = mp.matrix([weights])
    out = {}
    for r in ranks:
        scale = mp.diag([sv[i] ** (-mp.mpf(1) / 2) for i in range(r)])
        right = lc * vh[:r, :].H * scale
        left = scale * u[:, :r].H * lo.H
        ar = left * a_full * right
        br = left * ones
        cr = crow * right
        lam, vec = mp.eig(ar)
        ivec = mp.inverse(vec)
        cv = cr * vec
        vb = ivec * br
        out[r] = ([-lam[i] for i in range(r)], [cv[0, i] * vb[i] for i in range(r)])
    return out


def _halve(nodes, weights):
    """(tau0, omega) with one node of each conjugate pair and its weight doubled."""
    keep = []
    for t, w in zip(nodes, weights):
        if mp.im(t) > 0:
            mate = min(zip(nodes, weights), key=lambda p: abs(p[0] - mp.conj(t)))
            if abs(mate[0] - mp.conj(t)) > mp.mpf(10) ** (-40) * abs(t):
                raise RuntimeError("reduced nodes are not conjugate pairs")
            keep.append((complex(t), complex(2 * w)))
        elif abs(mp.im(t)) <= mp.mpf(10) ** (-40) * abs(t):
            keep.append((complex(mp.re(t)), complex(mp.re(w))))
    keep.sort(key=lambda p: p[0].real)
    return np.array([p[0] for p in keep]), np.array([p[1] for p in keep])


def _errors(tau0, omega, xs):
    s = np.zeros(xs.shape, np.complex128)
    ds = np.zeros(xs.shape, np.complex128)
    for t, w in zip(tau0, omega):
        ex = np.exp(-t * xs)
        s += w * ex
        ds -= w * t * ex
    g = np.exp(-0.25 * xs * xs)
    dg = -0.5 * xs * g
    e = np.max(np.abs(s.real - g))
    pos = xs > 0
    ep = np.max(np.abs(ds.real[pos] - dg[pos]))
    return float(e), float(ep)


def build_tables():
    with mp.workdps(PREC):
        nodes, weights = _contour(N_CONTOUR)
        reduced = _reduce_all(nodes, weights, [2 * m for m in range(1, MAX_MODES + 1)])
    grid = np.concatenate([[0.0], np.logspace(-5.0, 2.0, 100000)])
    dense = np.concatenate([[0.0], np.logspace(-7.0, 2.0, 900001)])
    tables = []
    for m in range(1, MAX_MODES + 1):
        with mp.workdps(PREC):
            tau0, omega = _halve(*reduced[2 * m])
        e1, ep1 = _errors(tau0, omega, grid)
        e2, ep2 = _errors(tau0, omega, dense)
        tables.append({
            "n_modes": m,
            "tau0_re": tau0.real.tolist(), "tau0_im": tau0.imag.tolist(),
            "omega_re": omega.real.tolist(), "omega_im": omega.imag.tolist(),
            "err_grid": e1, "err_bound": max(e1, e2) * (1.0 + 1e-3),
            "deriv_err_bound": max(ep1, ep2) * (1.0 + 1e-2),
            "sum_abs_omega": float(np.sum(np.abs(omega))),
        })
    return tables


def _hex(v: float) -> str:
    return float(v).hex()


def write_c(tables, path):
    lines = [
        "// SOE tables of the Gaussian exp(-x^2/4) at delta = 1: S(x) = Re sum_k omega_k exp(-tau0_k |x|).",
        "// Generated by paper_1909_09825_amd/soe/gen_tables.py (hyperbolic contour of Section 3.4,",
        "// midpoint rule (2.7)-(2.9), balanced truncation of Section 2.4).  Do not edit.",
        f"#define FGT_SOE_NUM_TABLES {len(tables)}",
        "static const fgt_soe_table_t kSoeTables[FGT_SOE_NUM_TABLES] = {",
    ]
    for t in tables:
        m = t["n_modes"]
        pad = lambda xs: ", ".join(_hex(v) for v in list(xs) + [0.0] * (8 - m))
        lines.append("  {%d,\n   {%s},\n   {%s},\n   {%s},\n   {%s},\n   %s, %s, %s}," % (
            m, pad(t["tau0_re"]), pad(t["tau0_im"]), pad(t["omega_re"]), pad(t["omega_im"]),
            _hex(t["err_bound"]), _hex(t["deriv_err_bound"]), _hex(t["sum_abs_omega"])))
    lines.append("};")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    tables = build_tables()
    write_c(tables, os.path.join(_CSRC, "soe_tables.inc"))
    with open(os.path.join(_HERE, "soe_tables.json"), "w") as f:
        json.dump({"contour_nodes": N_CONTOUR, "tables": tables}, f, indent=1)
        f.write("\n")
    for t in tables:
        print(t["n_modes"], "E=%.3e E'=%.3e sum|w|=%.3g" % (t["err_bound"], t["deriv_err_bound"],
                                                          t["sum_abs_omega"]))


if __name__ == "__main__":
    main()
