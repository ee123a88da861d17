"""Host check of the invariant-divisor division used by the KSG staging
(FastDiv, box_local_fast in csrc/common.h): compiled as host code with hipcc
and compared with plain integer division, exhaustively for small divisors
and numerators, at the edges, and on random values up to 2^31 - 1."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fastdiv_matches_integer_division(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = os.path.join(str(tmp_path), "fastdiv_check")
    src = os.path.join(ROOT, "tests", "native", "fastdiv_check.cpp")
    subprocess.run([hipcc if os.path.exists(hipcc) else "hipcc", "-O2", "-std=c++17", "-x", "c++",
                    "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "paper_2309_03308_amd", "csrc"),
                    src, "-o", exe], check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
