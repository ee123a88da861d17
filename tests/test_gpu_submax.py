"""Sub-brick maxima on the GPU (corr_region_submax: one refinement level of a
brick pair) against the oracle's exhaustive maxima over the oracle's
sub-bricks.

Bars as for region maxima: value within the precision's tolerance (FP32 and
split modes 1e-5, FP16 2e-3), n_evaluated exact (a point paired with itself
excluded within one field), argmax equal where the oracle's top-2 gap exceeds
twice the tolerance.
"""
import sys

import numpy as np
import pytest

import oracle
from argmax_checks import check_pearson_argmax
import synth
from oracle import aggregate_ref as AG

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


def _check(e_data, nx, ny, got, ra, sa, rb, sb, prec, data_b=None):
    subs_a, subs_b = AG.split_region(ra, sa), AG.split_region(rb, sb)
    assert len(got) == len(subs_a) and all(len(row) == len(subs_b) for row in got)
    for i, ba in enumerate(subs_a):
        for j, bb in enumerate(subs_b):
            ia = synth.Region(*ba).global_indices(nx, ny)
            ib = synth.Region(*bb).global_indices(nx, ny)
            ref = oracle.pearson_region_max_matmul(e_data, ia, ib, data_b=data_b,
                                                   same_field=None if data_b is None else False)
            g = got[i][j]
            assert abs(g["value"] - ref["value"]) <= TOL[prec], (prec, i, j, g, ref)
            assert g["n_evaluated"] == ref["n_evaluated"], (i, j, g["n_evaluated"], ref["n_evaluated"])
            check_pearson_argmax(g, ref, e_data, ia, ib, TOL[prec], data_b=data_b,
                                 same_field=data_b is None)


@pytest.mark.parametrize("prec", ["f32", "f16", "f16x3"])
def test_submax_two_bricks(env, prec):
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    e = synth.make_cfg1()
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    ra, rb = (r.as_tuple() for r in e.regions)
    got = ctx.corr_region_submax(f, pc.region(*ra), pc.region(*rb), (2, 2, 2), (2, 2, 2), prec)
    _check(e.data, e.nx, e.ny, got, ra, (2, 2, 2), rb, (2, 2, 2), prec)


def test_submax_brick_with_itself_and_uneven_splits(env):
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    e = synth.make_context(2, 2, (13, 9, 5), M=100, seed=8, n_groups=1, blob_r=2.0, min_region_gap=1)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    r0, r1 = e.regions[0].as_tuple(), e.regions[3].as_tuple()
    for ra, sa, rb, sb in ((r0, (2, 2, 1), r0, (2, 2, 1)), (r0, (3, 2, 2), r1, (1, 3, 5)),
                           ((2, 1, 0, 20, 12, 5), (3, 1, 2), (5, 0, 1, 15, 16, 4), (2, 2, 1))):  # overlapping bricks
        got = ctx.corr_region_submax(f, pc.region(*ra), pc.region(*rb), sa, sb, "f32")
        _check(e.data, e.nx, e.ny, got, ra, sa, rb, sb, "f32")


def test_submax_two_variables(env):
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    U, V, regs = synth.make_two_variables(nx=24, ny=16, nz=8, M=100, seed=7)
    fu = pc.Field(torch.from_numpy(U.data).cuda(), U.nx, U.ny, U.nz)
    fv = pc.Field(torch.from_numpy(V.data).cuda(), V.nx, V.ny, V.nz)
    ra, rb = regs[0].as_tuple(), regs[0].as_tuple()  # the same brick, different variables: nothing excluded
    got = ctx.corr_region_submax(fu, pc.region(*ra), pc.region(*rb), (2, 1, 2), (2, 2, 1), "f16x3", B=fv)
    _check(U.data, U.nx, U.ny, got, ra, (2, 1, 2), rb, (2, 2, 1), "f16x3", data_b=V.data)


def test_submax_large_members(env):
    # M = 1000 (FP16 storage) takes the generic contraction
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    rng = np.random.default_rng(3)
    nx, ny, nz, M = 16, 12, 6, 1000
    data = (rng.standard_normal((M, nx * ny * nz)) + 0.3 * rng.standard_normal((1, nx * ny * nz))).astype(np.float16)
    f = pc.Field(torch.from_numpy(data).cuda(), nx, ny, nz)
    ra, rb = (0, 0, 0, 8, 12, 6), (8, 0, 0, 8, 12, 6)
    got = ctx.corr_region_submax(f, pc.region(*ra), pc.region(*rb), (2, 1, 2), (1, 2, 2), "f16x3")
    _check(data.astype(np.float32), nx, ny, got, ra, (2, 1, 2), rb, (1, 2, 2), "f16x3")


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_submax_wide_tiles(env, prec):
    # sub-bricks of 4160 and 7040 points at M = 300: 17 x 28 tiles of 256 x 256
    # per sub-pair, so the wide-tile kernel runs on each block of the padded
    # sub-brick layout (ragged: its last tile rows are clamped and masked)
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    rng = np.random.default_rng(12)
    nx, ny, nz, M = 48, 32, 10, 300
    data = (rng.standard_normal((M, nx * ny * nz)) + 0.3 * rng.standard_normal((1, nx * ny * nz))).astype(np.float32)
    f = pc.Field(torch.from_numpy(data).cuda(), nx, ny, nz)
    ra, rb = (0, 0, 0, 26, 32, 10), (26, 0, 0, 22, 32, 10)
    _say(f"  submax wide tiles {prec}")
    got = ctx.corr_region_submax(f, pc.region(*ra), pc.region(*rb), (2, 1, 1), (1, 1, 1), prec)
    _check(data, nx, ny, got, ra, (2, 1, 1), rb, (1, 1, 1), prec)


def test_submax_focus_bricks_match_region_max(env):
    # the focus workload's 32x32x20 bricks split 2x2x2: all 64 sub-pairs equal
    # corr_region_max on the sub-boxes; four of them against the oracle
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    e = synth.make_cfg2()
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    ra, rb = (r.as_tuple() for r in e.regions)
    got = ctx.corr_region_submax(f, pc.region(*ra), pc.region(*rb), (2, 2, 2), (2, 2, 2), "f16x3")
    subs_a, subs_b = AG.split_region(ra, (2, 2, 2)), AG.split_region(rb, (2, 2, 2))
    for i, ba in enumerate(subs_a):
        for j, bb in enumerate(subs_b):
            one = ctx.corr_region_max(f, pc.region(*ba), pc.region(*bb), "pearson", "f16x3")
            assert abs(one["value"] - got[i][j]["value"]) <= 1e-6 and one["n_evaluated"] == got[i][j]["n_evaluated"]
    for i, j in ((0, 0), (3, 5), (7, 7), (6, 1)):
        ia = synth.Region(*subs_a[i]).global_indices(e.nx, e.ny)
        ib = synth.Region(*subs_b[j]).global_indices(e.nx, e.ny)
        ref = oracle.pearson_region_max_matmul(e.data, ia, ib)
        assert abs(got[i][j]["value"] - ref["value"]) <= 1e-5
    _say("  64 sub-brick pairs of the focus bricks checked")


def test_submax_bad_arguments(env):
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    f = pc.Field(torch.zeros((3, 8 * 8 * 8), device="cuda"), 8, 8, 8)
    r = pc.region(0, 0, 0, 4, 4, 4)
    for sa in ((0, 1, 1), (5, 1, 1), (1, -1, 1)):
        with pytest.raises(pc.CorrError) as ei:
            ctx.corr_region_submax(f, r, r, sa, (1, 1, 1), "f32")
        assert ei.value.status == 1
    with pytest.raises(pc.CorrError) as ei:
        ctx.corr_region_submax(f, r, pc.region(6, 0, 0, 4, 4, 4), (1, 1, 1), (1, 1, 1), "f32")
    assert ei.value.status == 1
