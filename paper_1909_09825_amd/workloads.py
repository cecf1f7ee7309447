"""Seeded synthetic inputs for the 1-D Gauss transform.

This module only draws random numbers; it holds none of the transform's
arithmetic.  Both the GPU path's tests/benchmark and the CPU oracle's tests
take their inputs from here, so the two sides always see the same arrays.

The shapes follow the paper's experiments (Section 5): points uniform on
[0, 1] (Tables 1-2), here widened with a clustered, uneven case and a
batched case.  No public dataset is involved.

Every generator is keyed by ``numpy.random.SeedSequence([1909, 9825, cfg,
sub])`` so a (cfg, sub) pair always reproduces the same arrays.
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED_PREFIX = (1909, 9825)


def rng(cfg: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([*SEED_PREFIX, cfg, sub]))


@dataclasses.dataclass
class Problem:
    """One transform: targets x[M], sources y[N], strengths alpha[N] (or [N][R])."""

    x: np.ndarray
    y: np.ndarray
    alpha: np.ndarray
    delta: float
    digits: int
    name: str

    @property
    def M(self) -> int:
        return int(self.x.shape[0])

    @property
    def N(self) -> int:
        return int(self.y.shape[0])


def plain(M: int, N: int, delta: float, digits: int, cfg: int = 1, sub: int = 0,
          alpha_dist: str = "normal") -> Problem:
    """Targets and sources i.i.d. uniform on [0, 1); alpha ~ N(0,1) or U(-1,1)."""
    g = rng(cfg, sub)
    y = g.random(N)
    x = g.random(M)
    if alpha_dist == "normal":
        a = g.standard_normal(N)
    elif alpha_dist == "uniform":
        a = g.uniform(-1.0, 1.0, N)
    else:
        raise ValueError(alpha_dist)
    return Problem(x, y, a, float(delta), int(digits), f"plain_M{M}_N{N}_d{delta:g}_D{digits}")


def small_plain() -> Problem:
    """1000 targets and 1000 sources uniform on [0,1), alpha ~ N(0,1), delta 1e-3, 6 digits."""
    return plain(1000, 1000, 1e-3, 6, cfg=1, sub=0)


def large_plain(delta: float, digits: int, log2n: int = 24) -> Problem:
    """M = N = 2^24 uniform points, alpha ~ N(0,1); delta in {1e-2, 1e-4, 1e-6}."""
    n = 1 << log2n
    sub = {1e-2: 0, 1e-4: 1, 1e-6: 2}.get(delta, 3)
    return plain(n, n, delta, digits, cfg=2, sub=sub)


def clustered(log2n: int = 24, log2m: int = 22, delta: float = 1e-5, digits: int = 6,
              n_comp: int = 64, sub: int = 0) -> Problem:
    """Sources from a 64-component Gaussian mixture, targets uniform.

    Centers uniform on [0,1), widths log-uniform on [1e-5, 1e-2], equal
    component weights, no clipping; alpha ~ U(-1,1).
    """
    g = rng(3, sub)
    n = 1 << log2n
    m = 1 << log2m
    centers = g.random(n_comp)
    sig = 10.0 ** g.uniform(-5.0, -2.0, n_comp)
    comp = g.integers(0, n_comp, n)
    y = centers[comp] + sig[comp] * g.standard_normal(n)
    x = g.random(m)
    a = g.uniform(-1.0, 1.0, n)
    return Problem(x, y, a, float(delta), int(digits), f"clustered_M{m}_N{n}_d{delta:g}_D{digits}")


def clustered_meta(n_comp: int = 64, sub: int = 0):
    """Centers and widths of the mixture used by :func:`clustered` (same draws)."""
    g = rng(3, sub)
    centers = g.random(n_comp)
    sig = 10.0 ** g.uniform(-5.0, -2.0, n_comp)
    return centers, sig


@dataclasses.dataclass
class Batch:
    """CSR batch of independent transforms sharing the digits setting."""

    x: np.ndarray          # [sum M]
    y: np.ndarray          # [sum N]
    alpha: np.ndarray      # [sum N][R]
    x_off: np.ndarray      # [B+1] int64
    y_off: np.ndarray      # [B+1] int64
    delta: np.ndarray      # [B]
    digits: int


def batched(B: int = 4096, R: int = 16, lo: int = 256, hi: int = 65536, digits: int = 6,
            sub: int = 0) -> Batch:
    """B transforms with N_b, M_b log-uniform in [lo, hi], delta_b log-uniform in [1e-6, 1e-2]."""
    g = rng(4, sub)
    Ns = np.floor(np.exp(g.uniform(np.log(lo), np.log(hi), B))).astype(np.int64)
    Ms = np.floor(np.exp(g.uniform(np.log(lo), np.log(hi), B))).astype(np.int64)
    delta = 10.0 ** g.uniform(-6.0, -2.0, B)
    y_off = np.zeros(B + 1, np.int64)
    x_off = np.zeros(B + 1, np.int64)
    np.cumsum(Ns, out=y_off[1:])
    np.cumsum(Ms, out=x_off[1:])
    y = g.random(int(y_off[-1]))
    x = g.random(int(x_off[-1]))
    a = g.standard_normal((int(y_off[-1]), R))
    return Batch(x, y, a, x_off, y_off, delta, digits)


def grad_problem(log2n: int = 22, delta: float = 1e-4, digits: int = 9, sub: int = 0):
    """M = N = 2^22 uniform points, alpha and upstream weights g ~ N(0,1)."""
    g = rng(5, sub)
    n = 1 << log2n
    y = g.random(n)
    x = g.random(n)
    a = g.standard_normal(n)
    w = g.standard_normal(n)
    return Problem(x, y, a, float(delta), int(digits), f"grad_N{n}_d{delta:g}_D{digits}"), w


def identical_uniform(N: int = 10_000_000, delta: float = 1.0, digits: int = 6, sub: int = 0):
    """Targets identical to N sources uniform on [0,1), alpha ~ N(0,1) (Table 1 setting)."""
    g = rng(6, sub)
    x = g.random(N)
    a = g.standard_normal(N)
    return x, a


def chebyshev(N: int) -> np.ndarray:
    """Chebyshev points of the first kind mapped to [0,1], in ascending order."""
    i = np.arange(1, N + 1, dtype=np.float64)
    return 0.5 * (1.0 - np.cos(np.pi * (i - 0.5) / N))


def sample_indices(M: int, k: int, cfg: int, sub: int = 1) -> np.ndarray:
    """k distinct target indices drawn without replacement (sorted)."""
    g = rng(cfg, 100 + sub)
    k = min(k, M)
    return np.sort(g.choice(M, size=k, replace=False)).astype(np.int64)
