"""The long-K contraction (M > 128: K staged through LDS in chunk groups, the
next chunks' loads held in registers, K zero-padded to a whole group) against
the oracle's exhaustive region maximum, at its edges: the smallest member
count it takes (129), an uneven one, the largest the library accepts (2048);
bricks whose point counts are not multiples of the 128-row tiles; and a brick
overlapping itself, where a point paired with itself is left out.

Bars: value within the precision's tolerance, n_evaluated exact, argmax
equal where the oracle's top-2 gap exceeds twice the tolerance.
"""
import sys

import numpy as np
import pytest

import oracle
from argmax_checks import check_pearson_argmax
import synth

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f16": 2e-3, "bf16": 7.9e-3, "f16x3": 1e-5, "bf16x3": 3e-5}


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as pc
    ctx = pc.Context(0)
    yield dict(torch=torch, pc=pc, ctx=ctx)
    ctx.close()


def _field(M, dims, seed, dtype=np.float32):
    rng = np.random.default_rng(seed)
    P = dims[0] * dims[1] * dims[2]
    common = rng.standard_normal((M, 4))
    mix = rng.standard_normal((4, P)) * (rng.uniform(size=P) < 0.3)
    d = rng.standard_normal((M, P)) + common @ mix + rng.uniform(-3, 3, P)
    return np.ascontiguousarray(d.astype(dtype))


def _check(env, data, dims, ra, rb, prec, same=True):
    pc, ctx, torch = env["pc"], env["ctx"], env["torch"]
    f = pc.Field(torch.from_numpy(data).cuda(), *dims)
    got = ctx.corr_region_max(f, pc.region(*ra), pc.region(*rb), "pearson", prec)
    ia = synth.Region(*ra).global_indices(dims[0], dims[1])
    ib = synth.Region(*rb).global_indices(dims[0], dims[1])
    ref = oracle.pearson_region_max_matmul(data, ia, ib)
    _say(f"  M={data.shape[0]} {prec} {ra}x{rb}: gpu {got['value']:.6f} oracle {ref['value']:.6f}")
    assert abs(got["value"] - ref["value"]) <= TOL[prec]
    assert got["n_evaluated"] == ref["n_evaluated"]
    check_pearson_argmax(got, ref, data, ia, ib, TOL[prec])


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16", "f16x3", "bf16x3"])
@pytest.mark.parametrize("M", [129, 300])
def test_long_k_ragged_bricks(env, M, prec):
    dims = (23, 17, 6)
    data = _field(M, dims, seed=M)
    # 7*9*5 = 315 and 11*6*4 = 264 points: ragged against 128-row tiles
    _check(env, data, dims, (0, 0, 0, 7, 9, 5), (9, 8, 1, 11, 6, 4), prec)


@pytest.mark.parametrize("prec", ["f32", "f16x3"])
def test_long_k_brick_overlapping_itself(env, prec):
    dims = (20, 14, 5)
    data = _field(200, dims, seed=3)
    _check(env, data, dims, (2, 1, 0, 10, 9, 4), (6, 4, 1, 10, 9, 4), prec)


@pytest.mark.parametrize("prec", ["f16", "f32"])
def test_long_k_largest_member_count(env, prec):
    dims = (12, 10, 4)
    data = _field(2048, dims, seed=7, dtype=np.float16)
    _check(env, data.astype(np.float32) if prec == "f32" else data, dims, (0, 0, 0, 6, 10, 4), (6, 0, 0, 6, 10, 4), prec)


def test_long_k_single_points(env):
    dims = (8, 8, 2)
    data = _field(500, dims, seed=11)
    _check(env, data, dims, (3, 4, 1, 1, 1, 1), (5, 2, 0, 1, 1, 1), "f32")
