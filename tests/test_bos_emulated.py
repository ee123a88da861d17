"""Batched BOS kernels (Sec. 3.1) run under a host emulation of HIP and
checked against the FP64 oracle: every pair's history must be reproduced
batch by batch by the oracle replaying it (same initial design, candidates,
believer picks, rounding and dedupe), and every objective value must match
the oracle's Pearson / KSG at those cells.

The kernels' source is compiled for the host by g++ with the primitives of
tests/emu/hip/hip_runtime.h (AddressSanitizer on, LDS allocated at exactly
the size the library requests), so indexing, barriers and termination are
exercised without a GPU.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth
from oracle import bos_ref as B
from test_oracle_bos import replay_iterations

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
EMU = os.path.join(HERE, "emu")


@pytest.fixture(scope="module")
def emu_bin(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("bos_emu")
    src = os.path.join(d, "bos_emu.cpp")
    with open(src, "w") as fh:
        subprocess.run(["python3", os.path.join(EMU, "transform.py"),
                        os.path.join(ROOT, "paper_2309_03308_amd", "csrc", "bos.hip")], stdout=fh, check=True)
    exe = os.path.join(d, "bos_emu")
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-I" + EMU, "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2309_03308_amd", "csrc"),
           "-include", "hip/hip_runtime.h", "-x", "c++", src, "-x", "c++", os.path.join(EMU, "emu_main.cpp"),
           "-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe, d


def _run(emu_bin, e, pairs, measure, seed, mode="graph"):
    exe, d = emu_bin
    inp = os.path.join(d, f"in_{measure}_{seed}_{mode}.bin")
    out = os.path.join(d, f"out_{measure}_{seed}_{mode}.txt")
    hdr = np.array([e.M, e.nx, e.ny, e.nz, len(e.regions), len(pairs), 0 if measure == "pearson" else 1, seed],
                   np.int32)
    regs = np.array([r.as_tuple() for r in e.regions], np.int32)
    with open(inp, "wb") as fh:
        for a in (hdr, np.ascontiguousarray(e.data, np.float32), regs, np.asarray(pairs, np.int32)):
            fh.write(a.tobytes())
    r = subprocess.run([exe, inp, out, mode], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "ERROR: AddressSanitizer" not in r.stderr
    hist, lines, i = {}, open(out).read().split("\n"), 0
    while i < len(lines) and lines[i]:
        t = lines[i].split()
        p, value, n = int(t[1]), float(t[3]), int(t[5])
        rows = np.array([list(map(float, lines[i + 1 + k].split())) for k in range(n)])
        hist[p] = (rows[:, :6].astype(np.int64), rows[:, 6], value)
        i += 1 + n
    return hist, r.stderr


@pytest.mark.parametrize("measure,npairs,seed,mode", [("pearson", 6, 3, "graph"), ("pearson", 5, 3, "plain"),
                                                    ("ksg", 2, 4, "graph")])
def test_emulated_bos_matches_oracle(emu_bin, measure, npairs, seed, mode):
    e = synth.make_context(4, 2, (12, 12, 6), M=100, seed=21, n_groups=3, blob_r=2.0, min_region_gap=2)
    pairs = synth.region_pair_list(len(e.regions))[:npairs]
    hist, log = _run(emu_bin, e, pairs, measure, seed, mode)
    assert "active=0" in log
    cfg = B.BosConfig(seed=seed)
    for p, (ia, ib) in enumerate(pairs):
        cells, vals, best = hist[p]
        ra, rb = e.regions[ia], e.regions[ib]
        assert cells.shape[0] <= cfg.n_total and len({tuple(c) for c in cells}) == cells.shape[0]
        pa, pb = B.cells_to_points(cells, ra, rb, e.nx, e.ny)
        pp = np.stack([pa, pb], 1).astype(np.int32)
        if measure == "pearson":
            ref = np.abs(oracle.pearson_pairs(e.data, pp))
        else:
            ref, _ = oracle.ksg_pairs(e.data, pp, 10, want_counts=False)
        assert np.max(np.abs(vals - ref)) <= 1e-5
        assert best == pytest.approx(float(vals.max()), abs=1e-7)
        m, t = replay_iterations(cfg, p, (ra.dx, ra.dy, ra.dz, rb.dx, rb.dy, rb.dz), cells, vals)
        assert m == t, (p, m, t)
