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


def eval_noalloc(x: torch.Tensor, y: torch.Tensor, alpha: torch.Tensor, p: Plan,
                 out: torch.Tensor) -> torch.Tensor:
    """eval() into `out` with the library's fixed per-device workspace (fgt_eval_noalloc).

    Nothing is allocated, here or in the library, so the call may run where
    allocation is not allowed (e.g. under graph capture).  Problems whose
    workspace exceeds FGT_NOALLOC_BYTES raise FGTError(FGT_ENOSPACE); calls that
    overlap in time on one device race on the shared workspace.
    """
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise ValueError("x must be a CUDA (HIP) tensor")
    dev = x.device
    for t, name in ((x, "x"), (y, "y"), (alpha, "alpha"), (out, "out")):
        if (not isinstance(t, torch.Tensor) or t.dim() != 1 or t.dtype != p.dtype
                or t.device != dev or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous 1-D {p.dtype} tensor on {dev}")
    M, N = x.shape[0], y.shape[0]
    if alpha.shape[0] != N or out.shape[0] != M:
        raise ValueError("alpha must have length N and out length M")
    stream = torch.cuda.current_stream(dev).cuda_stream
    check(p._lib.fgt_eval_noalloc(p.handle, x.data_ptr(), M, y.data_ptr(), alpha.data_ptr(), N,
                                  out.data_ptr(), stream), "fgt_eval_noalloc")
    return out


def _check_ws(p: Plan, ws: torch.Tensor, M: int, N: int, dev) -> int:
    need = p.workspace_size(M, N)
    if (not isinstance(ws, torch.Tensor) or ws.numel() * ws.element_size() < need
            or not ws.is_contiguous() or ws.device != dev):
        raise ValueError(f"workspace must be a contiguous {dev} tensor of >= {need} bytes")
    return need


def eval_self(x: torch.Tensor, alpha: torch.Tensor, p: Plan, presorted: bool = False,
              out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """u_i = sum_j S(x_i - x_j) alpha_j: targets identical to the sources.

    presorted=True skips the sort for points already in ascending order (the
    order is checked on the device; see last_device_status).
    """
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise ValueError("x must be a CUDA (HIP) tensor")
    dev = x.device
    x = _vec(x, "x", p.dtype, dev)
    alpha = _vec(alpha, "alpha", p.dtype, dev)
    N = x.shape[0]
    if alpha.shape[0] != N:
        raise ValueError("x and alpha must have the same length")
    if out is None:
        out = torch.empty(N, dtype=p.dtype, device=dev)
    else:
        out = _vec(out, "out", p.dtype, dev)
        if out.shape[0] != N:
            raise ValueError("out must have length N")
    if ws is None:
        ws = workspace(p, 0, N, dev)
    need = _check_ws(p, ws, 0, N, dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = p._lib.fgt_eval_self(p.handle, x.data_ptr(), N, alpha.data_ptr(), out.data_ptr(),
                              _lib.FGT_PRESORTED if presorted else 0, ws.data_ptr(), need, stream)
    check(rc, "fgt_eval_self")
    return out


def sort(x: torch.Tensor, y: torch.Tensor, p: Plan, alpha: torch.Tensor | None = None,
         exact: bool = False, ws: torch.Tensor | None = None):
    """The sort step alone (fgt_sort): (perm, z, (key_width, code_tol)).

    perm[p] is the merged index of sorted position p (< N: source, else target
    perm[p] - N) as an int64 tensor, z the sorted coordinates the scans use.
    exact=True sorts every key bit and keeps FP64 coordinates exact, so perm
    is the stable ascending order of [y; x].
    """
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise ValueError("x must be a CUDA (HIP) tensor")
    dev = x.device
    x = _vec(x, "x", p.dtype, dev)
    y = _vec(y, "y", p.dtype, dev)
    if alpha is not None:
        alpha = _vec(alpha, "alpha", p.dtype, dev)
        if alpha.shape[0] != y.shape[0]:
            raise ValueError("y and alpha must have the same length")
    M, N = x.shape[0], y.shape[0]
    if ws is None:
        ws = workspace(p, M, N, dev)
    need = _check_ws(p, ws, M, N, dev)
    perm = torch.empty(M + N, dtype=torch.int32, device=dev)
    z = torch.empty(M + N, dtype=p.dtype, device=dev)
    res = (ctypes.c_double * 2)()
    stream = torch.cuda.current_stream(dev).cuda_stream
    check(p._lib.fgt_sort(p.handle, x.data_ptr(), M, y.data_ptr(),
                          alpha.data_ptr() if alpha is not None else None, N,
                          _lib.FGT_SORT_EXACT if exact else 0, perm.data_ptr(), z.data_ptr(), res,
                          ws.data_ptr(), need, stream), "fgt_sort")
    return perm.long() & 0xFFFFFFFF, z, (res[0], res[1])


def sort_resolution(p: Plan) -> tuple[float, float]:
    """(key width, FP64 code tolerance) that the plan's sort uses (host query, no device work)."""
    res = (ctypes.c_double * 2)()
    check(p._lib.fgt_sort(p.handle, None, 0, None, None, 0, 0, None, None, res, None, 0, None),
          "fgt_sort")
    return res[0], res[1]


def eval_sorted(alpha: torch.Tensor, p: Plan, ws: torch.Tensor, M: int,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """u for new strengths on the points whose sort `ws` holds (from eval or backward).

    The radix sort depends on the coordinates only, so a sequence of
    transforms with fixed x, y and changing alpha pays for it once.
    """
    if not isinstance(alpha, torch.Tensor) or not alpha.is_cuda:
        raise ValueError("alpha must be a CUDA (HIP) tensor")
    dev = alpha.device
    alpha = _vec(alpha, "alpha", p.dtype, dev)
    N = alpha.shape[0]
    if out is None:
        out = torch.empty(int(M), dtype=p.dtype, device=dev)
    else:
        out = _vec(out, "out", p.dtype, dev)
        if out.shape[0] != M:
            raise ValueError("out must have length M")
    need = _check_ws(p, ws, M, N, dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    check(p._lib.fgt_eval_sorted(p.handle, int(M), N, alpha.data_ptr(), out.data_ptr(),
                                 ws.data_ptr(), need, stream), "fgt_eval_sorted")
    return out


def backward(x: torch.Tensor, y: torch.Tensor, alpha: torch.Tensor, g: torch.Tensor, p: Plan,
             ws: torch.Tensor | None = None, sorted: bool = False, dalpha: bool = True,
             dx: bool = True, dy: bool = True, ddelta: bool = True):
    """Gradients of L = sum_i g_i u_i: (dL/dalpha, dL/dx, dL/dy, dL/ddelta), None where not asked.

    With sorted=True, `ws` must hold the state left by the last eval or
    eval_sorted with this plan and these points (its sort and its strengths,
    which stand for `alpha`).  dL/ddelta is a 0-dim tensor.
    """
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise ValueError("x must be a CUDA (HIP) tensor")
    dev = x.device
    x = _vec(x, "x", p.dtype, dev)
    y = _vec(y, "y", p.dtype, dev)
    alpha = _vec(alpha, "alpha", p.dtype, dev)
    g = _vec(g, "g", p.dtype, dev)
    M, N = x.shape[0], y.shape[0]
    if alpha.shape[0] != N or g.shape[0] != M:
        raise ValueError("alpha must have length N and g length M")
    if ws is None:
        if sorted:
            raise ValueError("sorted=True needs the workspace that holds the sort")
        ws = workspace(p, M, N, dev)
    need = _check_ws(p, ws, M, N, dev)
    o_da = torch.empty(N, dtype=p.dtype, device=dev) if dalpha else None
    o_dx = torch.empty(M, dtype=p.dtype, device=dev) if dx else None
    o_dy = torch.empty(N, dtype=p.dtype, device=dev) if dy else None
    o_dd = torch.empty((), dtype=p.dtype, device=dev) if ddelta else None
    ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = p._lib.fgt_backward(p.handle, x.data_ptr(), M, y.data_ptr(), alpha.data_ptr(), N,
                             g.data_ptr(), ptr(o_da), ptr(o_dx), ptr(o_dy), ptr(o_dd),
                             _lib.FGT_SORTED if sorted else 0, ws.data_ptr(), need, stream)
    check(rc, "fgt_backward")
    return o_da, o_dx, o_dy, o_dd


class _WorkspaceCache:
    """Plans and workspaces of GaussTransform, kept across calls (LRU, a few shapes).

    Key: (delta, digits, dtype, M, N, device).  Each entry counts the forwards
    that wrote its workspace, so a backward can tell whether the workspace
    still holds its own forward's sort (then it reuses it) or was taken by a
    later forward of the same shape (then it sorts again).
    """

    def __init__(self, capacity: int = 4):
        import collections
        self.capacity = capacity
        self.entries = collections.OrderedDict()

    def get(self, delta: float, digits: int, dtype, M: int, N: int, device):
        key = (float(delta), int(digits), dtype, int(M), int(N), str(device))
        ent = self.entries.get(key)
        if ent is None:
            p = Plan(delta, digits, dtype)
            ent = {"plan": p, "ws": workspace(p, M, N, device), "generation": 0}
            self.entries[key] = ent
            while len(self.entries) > self.capacity:
                self.entries.popitem(last=False)
        else:
            self.entries.move_to_end(key)
        return ent

    def clear(self):
        self.entries.clear()


_gt_cache = _WorkspaceCache()


class GaussTransform(torch.autograd.Function):
    """u = FGT(x, y, alpha; delta) with gradients in x, y, alpha and delta.

    The forward keeps its workspace (the sort of the points) for the backward,
    which runs the adjoint scans on the same sorted order.  Plans and
    workspaces are cached across calls by shape, so a training loop allocates
    them once; if another forward of the same shape ran in between, the
    backward sorts the points again instead of using the workspace.
    """

    @staticmethod
    def forward(ctx, x, y, alpha, delta, digits):
        d = float(delta.detach().item()) if isinstance(delta, torch.Tensor) else float(delta)
        ent = _gt_cache.get(d, int(digits), x.dtype, x.shape[0], y.shape[0], x.device)
        u = eval(x, y, alpha, ent["plan"], ws=ent["ws"])
        ent["generation"] += 1
        ctx.save_for_backward(x, y, alpha)
        ctx.entry, ctx.generation = ent, ent["generation"]
        ctx.delta_is_tensor = isinstance(delta, torch.Tensor)
        ctx.delta_dtype = delta.dtype if ctx.delta_is_tensor else None
        return u

    @staticmethod
    def backward(ctx, gu):
        x, y, alpha = ctx.saved_tensors
        nx, ny, na, nd = ctx.needs_input_grad[:4]
        if not (nx or ny or na or nd):
            return None, None, None, None, None
        ent = ctx.entry
        own = ent["generation"] == ctx.generation
        da, dx, dy, dd = backward(x, y, alpha, gu.to(x.dtype).contiguous(), ent["plan"], ent["ws"],
                                  sorted=own, dalpha=na, dx=nx, dy=ny, ddelta=nd)
        if not own:
            ent["generation"] += 1      # this backward sorted again: the workspace is its now
        if dd is not None and ctx.delta_is_tensor:
            dd = dd.to(ctx.delta_dtype)
        return dx, dy, da, dd, None


def gauss_transform(x: torch.Tensor, y: torch.Tensor, alpha: torch.Tensor, delta,
                    digits: int = 6) -> torch.Tensor:
    """Differentiable u_i = sum_j exp(-(x_i - y_j)^2 / (4 delta)) alpha_j (SOE at `digits`).

    delta may be a float or a 0-dim tensor (then dL/ddelta is returned too).
    """
    return GaussTransform.apply(x, y, alpha, delta, digits)


class BatchPlan:
    """B independent transforms in CSR layout (host offsets), one delta each, R columns.

    Transform b: targets x[x_off[b]:x_off[b+1]], sources y[y_off[b]:y_off[b+1]],
    strengths alpha[y_off[b]:y_off[b+1], :R]; FP64 only.
    """

    def __init__(self, delta, digits: int, x_off, y_off, R: int = 1,
                 dtype: torch.dtype = torch.float64):
        if dtype not in _DTYPES:
            raise ValueError(f"dtype must be float64 or float32, got {dtype}")
        lib = _lib.load()
        self._delta = np.ascontiguousarray(np.asarray(delta, dtype=np.float64))
        self._xo = np.ascontiguousarray(np.asarray(x_off, dtype=np.int64))
        self._yo = np.ascontiguousarray(np.asarray(y_off, dtype=np.int64))
        B = self._delta.shape[0]
        if self._xo.shape != (B + 1,) or self._yo.shape != (B + 1,):
            raise ValueError("x_off and y_off must have B + 1 entries")
        h = ctypes.c_void_p()
        i64p = ctypes.POINTER(ctypes.c_int64)
        rc = lib.fgt_batch_plan(B, self._delta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                int(digits), _DTYPES[dtype], self._xo.ctypes.data_as(i64p),
                                self._yo.ctypes.data_as(i64p), int(R), ctypes.byref(h))
        if rc == _lib.FGT_EINVAL:
            raise ValueError(f"fgt_batch_plan: {_lib.strerror(rc)}")
        check(rc, "fgt_batch_plan")
        self._h, self._lib = h, lib
        self.B, self.R, self.digits, self.dtype = B, int(R), int(digits), dtype
        self.M, self.N = int(self._xo[-1]), int(self._yo[-1])
        n, e, tp = ctypes.c_int(), ctypes.c_double(), ctypes.c_int64()
        check(lib.fgt_batch_info(h, ctypes.byref(n), ctypes.byref(e), ctypes.byref(tp)),
              "fgt_batch_info")
        self.n_modes, self.err_bound, self.total_points = n.value, e.value, tp.value

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def workspace_size(self) -> int:
        return int(self._lib.fgt_batch_workspace_size(self._h))

    @property
    def config(self) -> tuple[int, int]:
        """(points per lane in the scan, target bucket size of the sort)."""
        c, b = ctypes.c_int(), ctypes.c_int()
        check(self._lib.fgt_batch_config(self._h, ctypes.byref(c), ctypes.byref(b)), "fgt_batch_config")
        return c.value, b.value

    def set_config(self, chunk: int, bucket_points: int) -> None:
        check(self._lib.fgt_batch_set_config(self._h, int(chunk), int(bucket_points)),
              "fgt_batch_set_config")

    def tune(self, x: torch.Tensor, y: torch.Tensor, alpha: torch.Tensor,
             ws: torch.Tensor | None = None, cache: str | None = None) -> tuple[int, int]:
        """Time the kernel choices on this data (or take them from the JSON cache); returns config."""
        u = torch.empty((self.M, self.R), dtype=self.dtype, device=x.device)
        if alpha.dim() == 1:
            alpha = alpha.reshape(-1, 1)
        alpha = alpha.contiguous()
        if ws is None:
            ws = batch_workspace(self, x.device)
        stream = torch.cuda.current_stream(x.device).cuda_stream
        rc = self._lib.fgt_batch_tune(self._h, x.contiguous().data_ptr(), y.contiguous().data_ptr(),
                                      alpha.data_ptr(), u.data_ptr(), ws.data_ptr(),
                                      self.workspace_size(), stream,
                                      cache.encode() if cache else None)
        check(rc, "fgt_batch_tune")
        return self.config

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.fgt_batch_destroy(h)
            self._h = None


def batch_plan(delta, digits: int, x_off, y_off, R: int = 1) -> BatchPlan:
    return BatchPlan(delta, digits, x_off, y_off, R)


def eval_batch(x: torch.Tensor, y: torch.Tensor, alpha: torch.Tensor, bp: BatchPlan,
               out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """u[sum M, R] for every transform of the batch plan, on the current stream."""
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise ValueError("x must be a CUDA (HIP) tensor")
    dev = x.device
    x = _vec(x, "x", bp.dtype, dev)
    y = _vec(y, "y", bp.dtype, dev)
    if x.shape[0] != bp.M or y.shape[0] != bp.N:
        raise ValueError(f"x and y must have {bp.M} and {bp.N} entries")
    if alpha.dim() == 1 and bp.R == 1:
        alpha = alpha.reshape(-1, 1)
    if (alpha.dim() != 2 or alpha.shape != (bp.N, bp.R) or alpha.dtype != bp.dtype
            or alpha.device != dev):
        raise ValueError(f"alpha must be a {bp.dtype} tensor of shape ({bp.N}, {bp.R}) on {dev}")
    alpha = alpha.contiguous()
    if out is None:
        out = torch.empty((bp.M, bp.R), dtype=bp.dtype, device=dev)
    elif out.shape != (bp.M, bp.R) or not out.is_contiguous() or out.dtype != bp.dtype:
        raise ValueError("out must be a contiguous tensor of shape (M, R)")
    need = bp.workspace_size()
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    elif ws.numel() * ws.element_size() < need or not ws.is_contiguous() or ws.device != dev:
        raise ValueError(f"workspace must be a contiguous {dev} tensor of >= {need} bytes")
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = bp._lib.fgt_batch_eval(bp.handle, x.data_ptr(), y.data_ptr(), alpha.data_ptr(),
                                out.data_ptr(), ws.data_ptr(), need, stream)
    check(rc, "fgt_batch_eval")
    return out


def batch_sorted(bp: BatchPlan, ws: torch.Tensor):
    """The sort step of the last eval_batch on `ws` (fgt_batch_sorted): (codes, z, resolution).

    codes[p] (int64) is source row j (< SN) or SN + target row i at sorted
    position p, transforms one after another; z[p] the coordinate as given;
    resolution the sort resolution in scaled units (coordinate / sqrt(delta)).
    """
    need = bp.workspace_size()
    if ws.numel() * ws.element_size() < need or not ws.is_contiguous() or not ws.is_cuda:
        raise ValueError(f"workspace must be a contiguous device tensor of >= {need} bytes")
    dev = ws.device
    P = bp.M + bp.N
    codes = torch.empty(P, dtype=torch.int32, device=dev)
    z = torch.empty(P, dtype=torch.float64, device=dev)
    res = ctypes.c_double()
    stream = torch.cuda.current_stream(dev).cuda_stream
    check(bp._lib.fgt_batch_sorted(bp.handle, ws.data_ptr(), need, codes.data_ptr(), z.data_ptr(),
                                   ctypes.byref(res), stream), "fgt_batch_sorted")
    return codes.long() & 0xFFFFFFFF, z, res.value


def batch_workspace(bp: BatchPlan, device) -> torch.Tensor:
    return torch.empty(max(bp.workspace_size(), 1), dtype=torch.uint8, device=device)


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
        if not name:
            raise RuntimeError("fgt_profile_end: a call marked more phases than the profiler records")
        if ms[i] > 0:
            out[name] = ms[i]
    return out, n_calls.value
