"""The library's FP64 sort-key code (Codec<double>, make_codec), checked on the CPU.

`codec_check.hip` includes the library's internal header and runs the key code
as host code over many kinds of range: ranges away from 0 (offset grid),
through 0 with values below the grid step, [0,1) data as in the benchmark,
huge, subnormal, overflowing and non-finite ranges.  It checks that grid keys
stay below 2^63, that key order never contradicts coordinate order, that grid
points decode exactly and others move by less than the grid step g, the
(key difference + 1) g gap bound the sort's resolution rule relies on, and
that IEEE keys are used (and decode exactly) where the grid step would exceed
the tolerance or the range is degenerate.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not found")
def test_fp64_key_code_on_host(tmp_path):
    exe = str(tmp_path / "codec_check")
    cmd = [HIPCC, "-O2", "-std=c++17", "--cuda-host-only", "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "codec_check.hip"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0 and "all cases passed" in r.stdout, r.stdout[-3000:]
