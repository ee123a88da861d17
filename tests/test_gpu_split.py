"""Exhaustive region maxima over 2^31 or more point pairs (Sec. 3: the maximum
over every pA in A and pB in B). The result key carries a 31-bit pair index,
so such a call runs as consecutive pieces of region A. Two 64x64x40 bricks of
a 128x64x40 M = 100 field (2.7e10 point pairs):
  - a planted pair (one point of B a noisy copy of one point of A) is found,
    its value the oracle's FP64 Pearson at that pair;
  - on an unplanted field the value equals the maximum over an independent
    partition of A into slabs (each below 2^31 pairs; the same kernels give
    the same per-pair values), and the argmax is that of the first slab
    attaining it;
  - n_evaluated counts every pair.
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

NX, NY, NZ, M = 128, 64, 40, 100
RA, RB = (0, 0, 0, 64, 64, 40), (64, 0, 0, 64, 64, 40)


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _gid(x, y, z):
    return x + NX * (y + NY * z)


@pytest.fixture(scope="module")
def env():
    import torch
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as pc
    rng = np.random.default_rng(31)
    data = rng.standard_normal((M, NX * NY * NZ), dtype=np.float32)
    planted = data.copy()
    p, q = _gid(10, 20, 30), _gid(64 + 50, 5, 7)
    planted[:, q] = 0.9 * planted[:, p] + 0.1 * rng.standard_normal(M, dtype=np.float32)
    ctx = pc.Context(0)
    yield dict(torch=torch, pc=pc, ctx=ctx, data=data, planted=planted, p=p, q=q)
    ctx.close()


def _field(env, arr):
    return env["pc"].Field(env["torch"].from_numpy(arr).cuda(), NX, NY, NZ)


def test_planted_pair_found_over_2e10_pairs(env):
    pc, ctx = env["pc"], env["ctx"]
    f = _field(env, env["planted"])
    got = ctx.corr_region_max(f, pc.region(*RA), pc.region(*RB), "pearson", "f16x3")
    _say(f"  2.7e10 pairs: {got}")
    assert got["n_evaluated"] == (64 * 64 * 40) ** 2
    assert (got["pa"], got["pb"]) == (env["p"], env["q"])
    ref = oracle.pearson_pairs(env["planted"], np.array([[env["p"], env["q"]]], np.int32))[0]
    assert abs(got["value"] - abs(ref)) <= 1e-5 and got["signed_value"] * ref > 0


def test_split_equals_independent_partition(env):
    pc, ctx = env["pc"], env["ctx"]
    f = _field(env, env["data"])
    rb = pc.region(*RB)
    got = ctx.corr_region_max(f, pc.region(*RA), rb, "pearson", "f16x3")
    # slabs of 5 z-layers: 20 480 x 163 840 = 3.4e9 pairs is too many, so 2 layers each
    parts = [ctx.corr_region_max(f, pc.region(0, 0, z, 64, 64, 2), rb, "pearson", "f16x3") for z in range(0, 40, 2)]
    best = max(r["value"] for r in parts)
    first = next(r for r in parts if r["value"] == best)
    assert got["value"] == best
    assert (got["pa"], got["pb"], got["signed_value"]) == (first["pa"], first["pb"], first["signed_value"])
    assert got["n_evaluated"] == sum(r["n_evaluated"] for r in parts)
    ref = oracle.pearson_pairs(env["data"], np.array([[got["pa"], got["pb"]]], np.int32))[0]
    assert abs(got["value"] - abs(ref)) <= 1e-5
    _say(f"  unplanted: max |r| {got['value']:.5f} over {got['n_evaluated']} pairs")
