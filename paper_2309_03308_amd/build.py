"""Build libcorr.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled with FP contraction off (KSG counts and
the FP64 statistics must be bit-reproducible) and without packed-FP32
instruction selection.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcorr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["api.hip", "standardize.hip", "pairs.hip", "ksg.hip", "gemm.hip", "gemm_smallk.hip", "bos.hip", "mlp.hip", "aggregate.hip", "sampling.hip", "peaks.hip"]

# The contraction kernels only see finite standardised values (|r| <= 1), so
# they run with IEEE mode off: max/min need no NaN quieting of MFMA results.
EXTRA = {"gemm.hip": ["-mno-amdgpu-ieee", "-fno-honor-nans"],
         "gemm_smallk.hip": ["-mno-amdgpu-ieee", "-fno-honor-nans"],
         "ksg.hip": ["-mno-amdgpu-ieee", "-fno-honor-nans"]}

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _up_to_date(src: str, obj: str) -> bool:
    """The object is newer than its source and every header it may include."""
    if not os.path.exists(obj):
        return False
    deps = [os.path.join(CSRC, src), os.path.join(CSRC, "common.h")]
    deps += [os.path.join(HERE, "..", "include", h) for h in os.listdir(os.path.join(HERE, "..", "include"))]
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(d) < t for d in deps)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if incremental and _up_to_date(src, obj):
        return obj
    cmd = [HIPCC, *CFLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int = 8, verbose: bool = True, incremental: bool = False) -> str:
    """Compile every source (or, with incremental, only those whose object is
    older than the source or a header) and link libcorr.so."""
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(jobs, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, incremental), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
