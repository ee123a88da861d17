"""Brick-pair samplers and sampled maxima on the GPU (corr_sample_pairs,
corr_sampled_max; Sec. 3.1) against the oracle, and the Sec. 5 strategy
dispatch for small bricks.

Bars: sample point pairs bit-exact (FP64 decisions taken the same way on
both sides); sampled maxima within the measure's tolerance (Pearson FP32
1e-5, KSG MI 1e-5), argmax equal where the oracle's top-2 gap exceeds twice
that, n_evaluated equal (samples of a point with itself skipped in one field).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import sampling_ref as SR

pytestmark = pytest.mark.gpu

SAMPLERS = {"uniform": SR.UNIFORM, "halton": SR.HALTON, "plastic": SR.PLASTIC}


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as pc
    ctx = pc.Context(0)
    e = synth.make_context(4, 3, (16, 16, 8), M=100, seed=5, n_groups=3, blob_r=3.0, min_region_gap=2)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    rp = synth.region_pair_list(len(e.regions))
    yield dict(torch=torch, pc=pc, ctx=ctx, e=e, f=f, rp=rp)
    ctx.close()


def _oracle_points(e, rp, sampler, seed, n, regions=None):
    regs = e.regions if regions is None else regions
    return np.stack([SR.sample_points(SAMPLERS[sampler], seed, p, regs[a], regs[b], e.nx, e.ny, n)
                     for p, (a, b) in enumerate(rp)])


@pytest.mark.parametrize("sampler", list(SAMPLERS))
def test_sample_pairs_bit_exact(env, sampler):
    ctx, e, f, rp = env["ctx"], env["e"], env["f"], env["rp"][:24]
    for seed in (0, 12345):
        got = ctx.corr_sample_pairs(f, [r.as_tuple() for r in e.regions], rp, sampler, 150, seed).cpu().numpy()
        ref = _oracle_points(e, rp, sampler, seed, 150)
        assert np.array_equal(got, ref), (sampler, seed, int((got != ref).sum()))


@pytest.mark.parametrize("sampler", list(SAMPLERS))
def test_sampled_max_pearson(env, sampler):
    ctx, e, f, rp = env["ctx"], env["e"], env["f"], env["rp"]
    n = 200
    res = ctx.corr_sampled_max(f, [r.as_tuple() for r in e.regions], rp, "pearson", "f32", 10, sampler, n, 7)
    pts = _oracle_points(e, rp, sampler, 7, n)
    for p in range(len(rp)):
        r = oracle.pearson_pairs(e.data, pts[p])
        ref = SR.sampled_max(r, pts[p], use_abs=True, same_field=True)
        got = res[p]
        assert abs(got["value"] - ref[0]) <= 1e-5 and got["n_evaluated"] == ref[4]
        top = np.sort(np.abs(r))[-2:]
        if top[1] - top[0] > 2e-5:
            assert (got["pa"], got["pb"]) == (ref[2], ref[3]) and abs(got["signed_value"] - ref[1]) <= 1e-5


def test_sampled_max_ksg_and_self_pairs(env):
    ctx, e, f = env["ctx"], env["e"], env["f"]
    regions = list(e.regions) + [synth.Region(0, 0, 0, 2, 2, 1)]  # 4 cells: many samples pair a point with itself
    regs = [r.as_tuple() for r in regions]
    rp = np.array([[0, 5], [3, 3], [7, 2], [12, 12]], np.int32)
    n = 300
    res = ctx.corr_sampled_max(f, regs, rp, "ksg", "f32", 10, "halton", n, 3)
    pts = _oracle_points(e, rp, "halton", 3, n, regions)
    for p in range(len(rp)):
        mi, _ = oracle.ksg_pairs(e.data, pts[p], 10, want_counts=False)
        ref = SR.sampled_max(mi, pts[p], use_abs=False, same_field=True)
        got = res[p]
        assert abs(got["value"] - ref[0]) <= 1e-5 and got["n_evaluated"] == ref[4], (p, got, ref)
        keep = pts[p][:, 0] != pts[p][:, 1]
        top = np.sort(mi[keep])[-2:]
        if top[1] - top[0] > 2e-5:
            assert (got["pa"], got["pb"]) == (ref[2], ref[3])
    assert res[3]["n_evaluated"] < n  # the tiny brick's self samples were skipped


def test_sampled_max_two_variables(env):
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    U, V, regs = synth.make_two_variables(nx=24, ny=16, nz=8, M=100, seed=7)
    fu = pc.Field(torch.from_numpy(U.data).cuda(), U.nx, U.ny, U.nz)
    fv = pc.Field(torch.from_numpy(V.data).cuda(), V.nx, V.ny, V.nz)
    rp = np.array([[0, 1], [0, 0], [1, 1]], np.int32)
    n = 500
    res = ctx.corr_sampled_max(fu, [r.as_tuple() for r in regs], rp, "pearson", "f32", 10, "plastic", n, 1, B=fv)
    for p, (a, b) in enumerate(rp):
        pts = SR.sample_points(SR.PLASTIC, 1, p, regs[a], regs[b], U.nx, U.ny, n)
        r = oracle.pearson_pairs(U.data, pts, data_b=V.data)
        ref = SR.sampled_max(r, pts, use_abs=True, same_field=False)
        assert abs(res[p]["value"] - ref[0]) <= 1e-5 and res[p]["n_evaluated"] == n


def test_sampling_bad_arguments(env):
    pc, ctx, e, f = env["pc"], env["ctx"], env["e"], env["f"]
    regs = [r.as_tuple() for r in e.regions]
    with pytest.raises(KeyError):
        ctx.corr_sample_pairs(f, regs, [(0, 1)], "sobol", 10)
    for rp, n in (([(0, 99)], 10), ([(0, 1)], -1)):
        with pytest.raises(pc.CorrError) as ei:
            ctx.corr_sampled_max(f, regs, rp, "pearson", "f32", 10, "uniform", n, 0)
        assert ei.value.status == 1
    import ctypes
    ra, nr, rpa = ctx._region_arrays(regs, [(0, 1)])
    st = ctx.L.corr_sample_pairs(ctx.h, ctypes.byref(f.c), ctypes.byref(f.c), ctypes.cast(ra, ctypes.c_void_p), nr,
                                 rpa.ctypes.data_as(ctypes.c_void_p), 1, 7, 10, 0, None, None)
    assert st == 2
    with pytest.raises(pc.CorrError) as ei:
        ctx.corr_sampled_max(f, regs, [(0, 1)], "ksg", "f32", 100, "uniform", 10, 0)
    assert ei.value.status == 1
    assert ctx.corr_sampled_max(f, regs, np.zeros((0, 2), np.int32)) == []
    empty = ctx.corr_sampled_max(f, regs, [(0, 1)], "pearson", "f32", 10, "uniform", 0, 0)[0]
    assert empty["n_evaluated"] == 0 and empty["pa"] == -1


def test_context_scale_samples(env):
    # all 3828 brick pairs (32x32x20) of the 352x256x20 context field, 100
    # samples each: sampled pairs of 16 pairs bit-exact, every sampled maximum
    # at most the exhaustive one
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    e = synth.make_cfg3()
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    regs = [r.as_tuple() for r in e.regions]
    rp = synth.region_pair_list(len(regs))
    rng = np.random.default_rng(4)
    sel = rng.choice(len(rp), 16, replace=False)
    for sampler in SAMPLERS:
        got = ctx.corr_sample_pairs(f, regs, rp, sampler, 100, 9).cpu().numpy()
        for p in sel:
            a, b = rp[p]
            ref = SR.sample_points(SAMPLERS[sampler], 9, int(p), e.regions[a], e.regions[b], e.nx, e.ny, 100)
            assert np.array_equal(got[p], ref), (sampler, p)
        res = ctx.corr_sampled_max(f, regs, rp, "pearson", "f32", 10, sampler, 100, 9)
        for p in sel:
            a, b = rp[p]
            ex = ctx.corr_region_max(f, pc.region(*regs[a]), pc.region(*regs[b]), "pearson", "f32")
            assert res[p]["value"] <= ex["value"] + 1e-5
        _say(f"  {sampler}: 3828 x 100 samples checked")


def test_brick_max_dispatch(env):
    pc, ctx, e, f = env["pc"], env["ctx"], env["e"], env["f"]
    ra = pc.region(0, 0, 0, 8, 8, 4)
    rb = pc.region(20, 10, 2, 8, 6, 4)
    st, r = pc.brick_max(ctx, f, ra, rb, "pearson", "f32")
    assert st == "exhaustive"
    assert r == ctx.corr_region_max(f, ra, rb, "pearson", "f32")
    st, r = pc.brick_max(ctx, f, ra, rb, "pearson", "f32", pairs_per_s=10.0, n_samples=64, seed=4)
    assert st == "random"
    assert r == ctx.corr_sampled_max(f, [ra, rb], [(0, 1)], "pearson", "f32", 10, "uniform", 64, 4)[0]
