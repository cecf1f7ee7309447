"""ctypes loader for libfgt.so (the C ABI declared in include/fgt.h).

Marshalling only: every step of the transform runs in the library's HIP
kernels.  A missing library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfgt.so")

FGT_OK, FGT_EINVAL, FGT_EUNSUPPORTED, FGT_ENONFINITE, FGT_EDEVICE, FGT_EUNSORTED = 0, 1, 2, 3, 4, 5
FGT_ENOSPACE = 6
FGT_NOALLOC_BYTES = 64 << 20
FGT_F64, FGT_F32 = 0, 1
FGT_MAX_MODES = 8
FGT_SORTED = 1
FGT_PRESORTED = 2
FGT_SORT_EXACT = 4

_lib = None


class FGTError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (status {code})")


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1909_09825_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    c_i64, c_int, c_dbl, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    dp, ip = ctypes.POINTER(c_dbl), ctypes.POINTER(c_int)
    lib.fgt_plan.argtypes = [c_dbl, c_int, c_int, ctypes.POINTER(vp)]
    lib.fgt_plan.restype = c_int
    lib.fgt_max_digits.argtypes = [c_int]
    lib.fgt_max_digits.restype = c_int
    lib.fgt_plan_info.argtypes = [vp, ip, dp, dp, dp, dp, dp]
    lib.fgt_plan_info.restype = c_int
    lib.fgt_plan_destroy.argtypes = [vp]
    lib.fgt_plan_destroy.restype = None
    lib.fgt_workspace_size.argtypes = [vp, c_i64, c_i64]
    lib.fgt_workspace_size.restype = ctypes.c_size_t
    lib.fgt_eval.argtypes = [vp, vp, c_i64, vp, vp, c_i64, vp, vp, ctypes.c_size_t, vp]
    lib.fgt_eval.restype = c_int
    lib.fgt_eval_noalloc.argtypes = [vp, vp, c_i64, vp, vp, c_i64, vp, vp]
    lib.fgt_eval_noalloc.restype = c_int
    lib.fgt_sort.argtypes = [vp, vp, c_i64, vp, vp, c_i64, c_int, vp, vp, dp, vp, ctypes.c_size_t, vp]
    lib.fgt_sort.restype = c_int
    lib.fgt_eval_sorted.argtypes = [vp, c_i64, c_i64, vp, vp, vp, ctypes.c_size_t, vp]
    lib.fgt_eval_sorted.restype = c_int
    lib.fgt_eval_self.argtypes = [vp, vp, c_i64, vp, vp, c_int, vp, ctypes.c_size_t, vp]
    lib.fgt_eval_self.restype = c_int
    lib.fgt_backward.argtypes = [vp, vp, c_i64, vp, vp, c_i64, vp, vp, vp, vp, vp, c_int, vp,
                                 ctypes.c_size_t, vp]
    lib.fgt_backward.restype = c_int
    i64p = ctypes.POINTER(c_i64)
    lib.fgt_batch_plan.argtypes = [c_i64, dp, c_int, c_int, i64p, i64p, c_int, ctypes.POINTER(vp)]
    lib.fgt_batch_plan.restype = c_int
    lib.fgt_batch_workspace_size.argtypes = [vp]
    lib.fgt_batch_workspace_size.restype = ctypes.c_size_t
    lib.fgt_batch_info.argtypes = [vp, ip, dp, i64p]
    lib.fgt_batch_info.restype = c_int
    lib.fgt_batch_eval.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.fgt_batch_eval.restype = c_int
    lib.fgt_batch_sorted.argtypes = [vp, vp, ctypes.c_size_t, vp, vp, dp, vp]
    lib.fgt_batch_sorted.restype = c_int
    lib.fgt_batch_tune.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp, ctypes.c_char_p]
    lib.fgt_batch_tune.restype = c_int
    lib.fgt_batch_config.argtypes = [vp, ip, ip]
    lib.fgt_batch_config.restype = c_int
    lib.fgt_batch_set_config.argtypes = [vp, c_int, c_int]
    lib.fgt_batch_set_config.restype = c_int
    lib.fgt_batch_destroy.argtypes = [vp]
    lib.fgt_batch_destroy.restype = None
    lib.fgt_eval_batched_workspace_size.argtypes = [c_i64, i64p, i64p, c_int, c_int]
    lib.fgt_eval_batched_workspace_size.restype = ctypes.c_size_t
    lib.fgt_eval_batched.argtypes = [c_i64, dp, c_int, c_int, i64p, i64p, vp, vp, vp, c_int, vp, vp,
                                     ctypes.c_size_t, vp]
    lib.fgt_eval_batched.restype = c_int
    lib.fgt_last_device_status.argtypes = [vp, vp]
    lib.fgt_last_device_status.restype = c_int
    lib.fgt_strerror.argtypes = [c_int]
    lib.fgt_strerror.restype = ctypes.c_char_p
    lib.fgt_profile_begin.argtypes = []
    lib.fgt_profile_begin.restype = c_int
    lib.fgt_profile_end.argtypes = [dp, c_int, ip, ip]
    lib.fgt_profile_end.restype = c_int
    lib.fgt_profile_phase_name.argtypes = [c_int]
    lib.fgt_profile_phase_name.restype = ctypes.c_char_p
    lib.fgt_version.argtypes = []
    lib.fgt_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code: int) -> str:
    try:
        return load().fgt_strerror(int(code)).decode()
    except RuntimeError:
        return f"status {code}"


def check(code: int, where: str) -> None:
    if code != FGT_OK:
        raise FGTError(code, where)
