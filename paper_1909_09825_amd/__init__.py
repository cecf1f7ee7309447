"""One-dimensional fast Gauss transform for AMD MI355X (gfx950).

u_i = sum_j exp(-(x_i - y_j)^2 / (4 delta)) alpha_j through sum-of-exponentials
approximations of the Gaussian (S. Jiang, arXiv 1909.09825): a device radix
sort of targets and sources, then forward and backward complex recurrences
per mode as parallel scans, all in hand-written HIP kernels behind the C ABI
of include/fgt.h.
"""
from ._lib import (FGT_EDEVICE, FGT_EINVAL, FGT_ENONFINITE, FGT_ENOSPACE, FGT_NOALLOC_BYTES, FGT_EUNSORTED, FGT_EUNSUPPORTED,
                   FGT_F32, FGT_F64, FGT_OK, FGT_PRESORTED, FGT_SORT_EXACT, FGT_SORTED, FGTError, LIB_PATH)
from .api import (BatchPlan, GaussTransform, Plan, backward, batch_plan, batch_sorted,
                  batch_workspace, eval, eval_batch, eval_noalloc, eval_self, eval_sorted,
                  gauss_transform, last_device_status, max_digits, plan, profile_begin,
                  profile_end, sort, sort_resolution, workspace)

__all__ = ["Plan", "plan", "eval", "eval_noalloc", "sort", "sort_resolution", "FGT_SORT_EXACT", "FGT_ENOSPACE", "FGT_NOALLOC_BYTES", "eval_self", "eval_sorted", "backward", "GaussTransform", "gauss_transform",
           "BatchPlan", "batch_plan", "eval_batch", "batch_sorted", "batch_workspace",
           "workspace", "last_device_status", "max_digits", "FGTError",
           "FGT_OK", "FGT_EINVAL", "FGT_EUNSUPPORTED", "FGT_ENONFINITE", "FGT_EDEVICE",
           "FGT_F64", "FGT_F32", "FGT_SORTED", "FGT_PRESORTED", "FGT_EUNSORTED", "LIB_PATH", "profile_begin", "profile_end"]
