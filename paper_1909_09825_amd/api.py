"""Python binding of the fast Gauss transform library (torch tensors in, torch tensors out).

    import torch, paper_1909_09825_amd as fgt
    p = fgt.plan(delta=1e-4, digits=6)                     # FP64
    u = fgt.eval(x, y, alpha, p)                           # x[M], y[N], alpha[N] on cuda

PyTorch supplies device memory and the current stream; the C ABI of
include/fgt.h does all the work.  Names follow the paper: targets x,
sources y, strengths alpha, heat-kernel time delta (kernel exp(-r^2/(4 delta))).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import FGT_F32, FGT_F64, FGTError, check

_DTYPES = {torch.float64: FGT_F64, torch.float32: FGT_F32}


class Plan:
    """An SOE table chosen for `digits` and scaled to `delta` (owns the C plan)."""

    def __init__(self, delta: float, digits: int, dtype: torch.dtype = torch.float64):
        if dtype not in _DTYPES:
            raise ValueError(f"dtype must be float64 or float32, got {dtype}")
        lib = _lib.load()
        h = ctypes.c_void_p()
        rc = lib.fgt_plan(float(delta), int(digits), _DTYPES[dtype], ctypes.byref(h))
        if rc == _lib.FGT_EINVAL:
            raise ValueError(f"fgt_plan(delta={delta}, digits={digits}): {_lib.strerror(rc)}")
        check(rc, "fgt_plan")
        self._h = h
        self._lib = lib
        self.dtype = dtype
        self.digits = int(digits)
        n = ctypes.c_int()
        e, ep, d = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        tau = (ctypes.c_double * (2 * _lib.FGT_MAX_MODES))()
        om = (ctypes.c_double * (2 * _lib.FGT_MAX_MODES))()
        check(lib.fgt_plan_info(h, ctypes.byref(n), ctypes.byref(e), ctypes.byref(ep), tau, om,
                                ctypes.byref(d)), "fgt_plan_info")
        self.n_modes = n.value
        self.err_bound = e.value
        self.deriv_err_bound = ep.value
        self.delta = d.value
        t = np.array(tau[: 2 * n.value])
        w = np.array(om[: 2 * n.value])
        self.tau = t[0::2] + 1j * t[1::2]        # already divided by sqrt(delta)
        self.omega = w[0::2] + 1j * w[1::2]

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def workspace_size(self, M: int, N: int) -> int:
        return int(self._lib.fgt_workspace_size(self._h, int(M), int(N)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.fgt_plan_destroy(h)
            self._h = None

    def __repr__(self) -> str:
        return (f"Plan(delta={self.delta:g}, digits={self.digits}, dtype={self.dtype}, "
                f"n_modes={self.n_modes}, err_bound={self.err_bound:.3e})")


def plan(delta: float, digits: int, dtype: torch.dtype = torch.float64) -> Plan:
    return Plan(delta, digits, dtype)


def max_digits(dtype: torch.dtype = torch.float64) -> int:
    return int(_lib.load().fgt_max_digits(_DTYPES[dtype]))


def _vec(t: torch.Tensor, name: str, dtype: torch.dtype, device) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dim() != 1:
        raise ValueError(f"{name} must be 1-D, got shape {tuple(t.shape)}")
    if t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, plan expects {dtype}")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t.contiguous()


def workspace(p: Plan, M: int, N: int, device) -> torch.Tensor:
    """A device workspace of fgt_workspace_size bytes (torch allocations are 512-byte aligned)."""
    return torch.empty(max(p.workspace_size(M, N), 1), dtype=torch.uint8, device=device)


def eval(x: torch.Tensor, y: torch.Tensor, alpha: torch.Tensor, p: Plan,
         out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """u_i = sum_j S(x_i - y_j) alpha_j on the current stream of x's device."""
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise ValueError("x must be a CUDA (HIP) tensor")
    dev = x.device
    x = _vec(x, "x", p.dtype, dev)
    y = _vec(y, "y", p.dtype, dev)
    alpha = _vec(alpha, "alpha", p.dtype, dev)
    if y.shape[0] != alpha.shape[0]:
        raise ValueError("y and alpha must have the same length")
    M, N = x.shape[0], y.shape[0]
    if out is None:
        out = torch.empty(M, dtype=p.dtype, device=dev)
    else:
        out = _vec(out, "out", p.dtype, dev)
        if out.shape[0] != M or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor of length M")
    need = p.workspace_size(M, N)
    if ws is None:
        ws = workspace(p, M, N, dev)
    elif ws.numel() * ws.element_size() < need or not ws.is_contiguous() or ws.device != dev:
        raise ValueError(f"workspace must be a contiguous {dev} tensor of >= {need} bytes")
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = p._lib.fgt_eval(p.handle, x.data_ptr(), M, y.data_ptr(), alpha.data_ptr(), N,
                         out.data_ptr(), ws.data_ptr(), need, stream)
    check(rc, "fgt_eval")
    return out


def last_device_status(ws: torch.Tensor) -> int:
    """Synchronise the current stream; return and clear the device status of `ws` (0 = ok)."""
    stream = torch.cuda.current_stream(ws.device).cuda_stream
    return int(_lib.load().fgt_last_device_status(ws.data_ptr(), stream))


def profile_begin() -> None:
    """Record per-phase HIP events in subsequent eval calls (benchmark use)."""
    check(_lib.load().fgt_profile_begin(), "fgt_profile_begin")


def profile_end() -> tuple[dict, int]:
    """Stop recording; return ({phase: summed ms}, number of calls)."""
    lib = _lib.load()
    ms = (ctypes.c_double * 16)()
    n_ph, n_calls = ctypes.c_int(), ctypes.c_int()
    check(lib.fgt_profile_end(ms, 16, ctypes.byref(n_ph), ctypes.byref(n_calls)), "fgt_profile_end")
    out = {}
    for i in range(n_ph.value):
        name = lib.fgt_profile_phase_name(i).decode()
        if ms[i] > 0:
            out[name] = ms[i]
    return out, n_calls.value
