"""Phase events of fgt_profile_begin / fgt_profile_end, which bench.py turns into
per-kernel times and roofline fractions.

A multi-kernel fgt_eval records one phase per kernel group: the sort's setup,
one per radix pass (8 for FP64 keys, 4 for FP32, passes that move nothing
included), the tile reduce, the carries and the final scan.  A small problem
(M + N <= 4096) records its one launch as the single phase "setup".  A call
that marked more phases than the profiler holds makes profile_end raise.
"""
import numpy as np
import pytest
import torch

import paper_1909_09825_amd as fgt
from fgt_testlib import say, to_dev

pytestmark = pytest.mark.gpu

F64_PHASES = {"setup", *(f"radix{i}" for i in range(8)), "tiles_reduce", "carry", "tiles_final"}
F32_PHASES = {"setup", *(f"radix{i}" for i in range(4)), "tiles_reduce", "carry", "tiles_final"}


def profiled(M, N, dtype, calls=4):
    g = np.random.default_rng(M + 7 * N)
    x, y, a = g.random(M), g.random(N), g.standard_normal(N)
    say(f"[gpu] profiled fgt_eval M={M} N={N} {dtype}")
    p = fgt.plan(1e-4, 6, dtype)
    X, Y, A = to_dev(x, dtype), to_dev(y, dtype), to_dev(a, dtype)
    ws = fgt.workspace(p, M, N, X.device)
    u = torch.empty(M, dtype=dtype, device="cuda")
    fgt.eval(X, Y, A, p, out=u, ws=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fgt.profile_begin()
    e0.record()
    for _ in range(calls):
        fgt.eval(X, Y, A, p, out=u, ws=ws)
    e1.record()
    phases, n = fgt.profile_end()
    torch.cuda.synchronize()
    assert fgt.last_device_status(ws) == fgt.FGT_OK
    assert n == calls
    return phases, e0.elapsed_time(e1)


@pytest.mark.parametrize("dtype,names", [(torch.float64, F64_PHASES), (torch.float32, F32_PHASES)])
def test_phases_of_the_multi_kernel_path(dtype, names):
    phases, wall = profiled(1 << 19, 1 << 19, dtype)
    assert set(phases) == names
    assert all(v > 0 for v in phases.values())
    total = sum(phases.values())
    say(f"   phases {total:.3f} ms of {wall:.3f} ms")
    # the phases tile each call: their sum is the calls' time less the gaps between calls
    assert 0.5 * wall <= total <= 1.05 * wall


def test_small_problem_is_one_phase():
    phases, wall = profiled(1000, 1000, torch.float64)
    assert set(phases) == {"setup"}
    assert phases["setup"] <= 1.05 * wall
