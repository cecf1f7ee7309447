"""ORACLE for the 1-D fast Gauss transform -- test infrastructure only.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline leg may import this package.  It shares no code with the GPU
library (``paper_1909_09825_amd``) and the GPU library never imports it.

* :func:`direct`          -- O1, the definition (1.1)-(1.2), Neumaier-summed.
* :func:`soe_recurrence`  -- O2, the SOE sweeps of Section 4 ((4.1)-(4.6)).
* :func:`soe_brute`       -- O3, the SOE transform summed pair by pair.
* :func:`soe_recurrence_deriv` -- O2's sweeps giving the SOE transform's x-derivative.
* :func:`direct_gradients` -- gradients of L = sum_i g_i u_i from the definition.
* :func:`soe_deriv_brute` -- the SOE transform's derivative field, pair by pair.
* :mod:`oracle.soe_table` -- the SOE tables built from Sections 2-3 and the
  E_n measurement (3.1).

The C part (``fgt_oracle.c``) is compiled with gcc by :func:`build`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fgt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# Sources farther than sqrt(4 delta * 69.1) contribute below 1e-30 |alpha_j|.
DEFAULT_CUTOFF = 69.1


def build(force: bool = True) -> str:
    """Compile fgt_oracle.c into liboracle.so with gcc (IEEE double, OpenMP)."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_direct.argtypes = [dp, i64, dp, dp, i64, ctypes.c_double, ctypes.c_double, dp,
                                      ctypes.c_int, ctypes.c_int]
        lib.oracle_direct.restype = ctypes.c_int
        lib.oracle_soe_recurrence.argtypes = [dp, i64, dp, dp, i64, ctypes.c_double, ctypes.c_int,
                                              dp, dp, dp, dp, dp, ctypes.c_int, ctypes.c_int]
        lib.oracle_soe_recurrence.restype = ctypes.c_int
        lib.oracle_soe_recurrence_field.argtypes = [dp, i64, dp, dp, i64, ctypes.c_double,
                                                    ctypes.c_int, dp, dp, dp, dp, ctypes.c_int, dp,
                                                    ctypes.c_int, ctypes.c_int]
        lib.oracle_soe_recurrence_field.restype = ctypes.c_int
        lib.oracle_soe_brute.argtypes = [dp, i64, dp, dp, i64, ctypes.c_double, ctypes.c_int,
                                         dp, dp, dp, dp, dp, ctypes.c_int]
        lib.oracle_soe_brute.restype = ctypes.c_int
        lib.oracle_direct_field.argtypes = [dp, i64, dp, dp, i64, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int, dp, ctypes.c_int, ctypes.c_int]
        lib.oracle_direct_field.restype = ctypes.c_int
        lib.oracle_soe_deriv_brute.argtypes = [dp, i64, dp, dp, i64, ctypes.c_double, ctypes.c_int,
                                               dp, dp, dp, dp, dp, ctypes.c_int, ctypes.c_int]
        lib.oracle_soe_deriv_brute.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_last_sort_seconds.argtypes = []
        lib.oracle_last_sort_seconds.restype = ctypes.c_double
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def last_sort_seconds() -> float:
    """Wall time of the sort inside the last soe_recurrence call (timing only)."""
    return float(_load().oracle_last_sort_seconds())


def direct(x, y, alpha, delta: float, cutoff: float = DEFAULT_CUTOFF, threads: int = 0,
           plant: int = 0) -> np.ndarray:
    """O1: u_i = sum_j alpha_j exp(-(x_i - y_j)^2 / (4 delta)) for every entry of x."""
    x, y, alpha = _f64(x), _f64(y), _f64(alpha)
    u = np.zeros(x.shape[0], np.float64)
    rc = _load().oracle_direct(_ptr(x), x.shape[0], _ptr(y), _ptr(alpha), y.shape[0], float(delta),
                               float(cutoff), _ptr(u), int(threads), int(plant))
    if rc:
        raise ValueError(f"oracle_direct failed ({rc})")
    return u


def _table_arrays(tau0, omega):
    tau0 = np.asarray(tau0, dtype=np.complex128)
    omega = np.asarray(omega, dtype=np.complex128)
    return (_f64(tau0.real), _f64(tau0.imag), _f64(omega.real), _f64(omega.imag))


def soe_recurrence(x, y, alpha, delta: float, tau0, omega, threads: int = 0,
                   plant: int = 0) -> np.ndarray:
    """O2: the Section 4 sweeps with the SOE table (tau0, omega)."""
    x, y, alpha = _f64(x), _f64(y), _f64(alpha)
    tr, ti, wr, wi = _table_arrays(tau0, omega)
    u = np.zeros(x.shape[0], np.float64)
    rc = _load().oracle_soe_recurrence(_ptr(x), x.shape[0], _ptr(y), _ptr(alpha), y.shape[0],
                                       float(delta), tr.shape[0], _ptr(tr), _ptr(ti), _ptr(wr),
                                       _ptr(wi), _ptr(u), int(threads), int(plant))
    if rc:
        raise ValueError(f"oracle_soe_recurrence failed ({rc})")
    return u


def soe_recurrence_deriv(x, y, alpha, delta: float, tau0, omega, threads: int = 0,
                         plant: int = 0) -> np.ndarray:
    """O2 with derivative weights: sum_j alpha_j S'(x_i - y_j), a source at x_i counted left."""
    x, y, alpha = _f64(x), _f64(y), _f64(alpha)
    tr, ti, wr, wi = _table_arrays(tau0, omega)
    u = np.zeros(x.shape[0], np.float64)
    rc = _load().oracle_soe_recurrence_field(_ptr(x), x.shape[0], _ptr(y), _ptr(alpha), y.shape[0],
                                             float(delta), tr.shape[0], _ptr(tr), _ptr(ti),
                                             _ptr(wr), _ptr(wi), 1, _ptr(u), int(threads),
                                             int(plant))
    if rc:
        raise ValueError(f"oracle_soe_recurrence_field failed ({rc})")
    return u


def soe_brute(x, y, alpha, delta: float, tau0, omega, threads: int = 0) -> np.ndarray:
    """O3: sum_j alpha_j Re sum_k omega_k exp(-tau0_k |x_i - y_j| / sqrt(delta))."""
    x, y, alpha = _f64(x), _f64(y), _f64(alpha)
    tr, ti, wr, wi = _table_arrays(tau0, omega)
    u = np.zeros(x.shape[0], np.float64)
    rc = _load().oracle_soe_brute(_ptr(x), x.shape[0], _ptr(y), _ptr(alpha), y.shape[0],
                                  float(delta), tr.shape[0], _ptr(tr), _ptr(ti), _ptr(wr), _ptr(wi),
                                  _ptr(u), int(threads))
    if rc:
        raise ValueError(f"oracle_soe_brute failed ({rc})")
    return u


def _field(x, y, w, delta, which, cutoff=DEFAULT_CUTOFF, threads=0, plant=0):
    x, y, w = _f64(x), _f64(y), _f64(w)
    out = np.zeros(x.shape[0], np.float64)
    rc = _load().oracle_direct_field(_ptr(x), x.shape[0], _ptr(y), _ptr(w), y.shape[0], float(delta),
                                     float(cutoff), int(which), _ptr(out), int(threads), int(plant))
    if rc:
        raise ValueError(f"oracle_direct_field failed ({rc})")
    return out


def direct_gradients(x, y, alpha, g, delta: float, targets=None, sources=None, threads: int = 0,
                     plant: int = 0):
    """Gradients of L = sum_i g_i u_i, u from (1.1)-(1.2), by direct summation.

    Returns (dalpha, dx, dy, ddelta):
      dalpha_j = sum_i g_i G(x_i - y_j)            (the transform with roles swapped),
      dx_i     = g_i sum_j alpha_j G'(x_i - y_j),
      dy_j     = alpha_j sum_i g_i G'(y_j - x_i),
      ddelta   = sum_ij g_i alpha_j (x_i - y_j)^2 / (4 delta^2) G(x_i - y_j).
    `targets` / `sources` restrict dx / (dalpha, dy) to index subsets (ddelta is
    then None).  `plant` is passed to the field evaluation (tests only).
    """
    x, y, alpha, g = _f64(x), _f64(y), _f64(alpha), _f64(g)
    ti = np.arange(x.shape[0]) if targets is None else np.asarray(targets)
    sj = np.arange(y.shape[0]) if sources is None else np.asarray(sources)
    dalpha = direct(y[sj], x, g, delta, threads=threads)
    dx = g[ti] * _field(x[ti], y, alpha, delta, 1, threads=threads, plant=plant)
    dy = alpha[sj] * _field(y[sj], x, g, delta, 1, threads=threads, plant=plant)
    ddelta = None
    if targets is None and sources is None:
        ddelta = float(np.dot(g, _field(x, y, alpha, delta, 2, threads=threads, plant=plant)))
    return dalpha, dx, dy, ddelta


def soe_deriv_brute(x, y, w, delta: float, tau0, omega, threads: int = 0,
                    plant: int = 0) -> np.ndarray:
    """sum_j w_j S'(x_i - y_j) with S' of the SOE (sign(0) = 0)."""
    x, y, w = _f64(x), _f64(y), _f64(w)
    tr, ti, wr, wi = _table_arrays(tau0, omega)
    out = np.zeros(x.shape[0], np.float64)
    rc = _load().oracle_soe_deriv_brute(_ptr(x), x.shape[0], _ptr(y), _ptr(w), y.shape[0],
                                        float(delta), tr.shape[0], _ptr(tr), _ptr(ti), _ptr(wr),
                                        _ptr(wi), _ptr(out), int(threads), int(plant))
    if rc:
        raise ValueError(f"oracle_soe_deriv_brute failed ({rc})")
    return out
