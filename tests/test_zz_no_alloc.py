"""corr_region_max_noalloc (fixed per-GPU scratch, no device allocation)
against corr_region_max on the same inputs, through the C ABI.

Both run the same kernels on the same standardised data, so every output
must be identical: value, signed value, argmax and n_evaluated. Each case
makes two no-allocation calls in a row, the second on smaller regions, so a
stale first call's scratch contents would show. A call that needs more than
the fixed scratch is refused on the host with CORR_EINVAL.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as pc
    e = synth.make_cfg2()
    ctx = pc.Context(0)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    rng = np.random.default_rng(5)
    big = rng.standard_normal((300, 6 * 5 * 4 * 8), dtype=np.float32)  # M = 300: the chunked contraction
    f300 = pc.Field(torch.from_numpy(big).cuda(), 12, 10, 8)
    yield dict(torch=torch, pc=pc, e=e, ctx=ctx, f=f, f300=f300)
    ctx.close()


def _same(a, b):
    assert a["value"] == b["value"] and a["signed_value"] == b["signed_value"], (a, b)
    assert (a["pa"], a["pb"], a["n_evaluated"]) == (b["pa"], b["pb"], b["n_evaluated"]), (a, b)


def _regions(env, shrink):
    pc, e = env["pc"], env["e"]
    ra, rb = e.regions
    if not shrink:
        return pc.region(*ra.as_tuple()), pc.region(*rb.as_tuple())
    # a smaller, ragged pair inside the same bricks
    return pc.region(ra.x0 + 3, ra.y0 + 1, ra.z0 + 2, 17, 23, 9), pc.region(rb.x0 + 5, rb.y0, rb.z0 + 1, 21, 13, 11)


@pytest.mark.parametrize("prec", ["f16", "f32", "f16x3", "bf16"])
def test_exhaustive_pearson_two_calls(env, prec):
    ctx, f = env["ctx"], env["f"]
    for shrink in (False, True):
        ra, rb = _regions(env, shrink)
        _say(f"  noalloc exhaustive pearson {prec}, {'smaller' if shrink else 'focus'} regions")
        got = ctx.corr_region_max_noalloc(f, ra, rb, "pearson", prec)
        ref = ctx.corr_region_max(f, ra, rb, "pearson", prec)
        _same(got, ref)


def test_exhaustive_pearson_same_brick_self_pairs(env):
    ctx, f = env["ctx"], env["f"]
    ra, _ = _regions(env, False)
    small, _ = _regions(env, True)
    for r in (ra, small):  # a brick with itself: the self-pair list lives in the scratch too
        _same(ctx.corr_region_max_noalloc(f, r, r, "pearson", "f16"), ctx.corr_region_max(f, r, r, "pearson", "f16"))


def test_sampled_pearson_and_ksg_two_calls(env):
    torch, ctx, f, e = env["torch"], env["ctx"], env["f"], env["e"]
    for shrink, n in ((False, 200_000), (True, 5_000)):
        ra, rb = _regions(env, shrink)
        rA = synth.Region(ra.x0, ra.y0, ra.z0, ra.dx, ra.dy, ra.dz)
        rB = synth.Region(rb.x0, rb.y0, rb.z0, rb.dx, rb.dy, rb.dz)
        pairs = synth.region_pairs_uniform(11 + n, n, rA, rB, e.nx, e.ny)
        dp = torch.from_numpy(pairs).cuda()
        _say(f"  noalloc sampled pearson / ksg, {n} pairs")
        _same(ctx.corr_region_max_noalloc(f, ra, rb, "pearson", "f32", samples=dp),
              ctx.corr_region_max(f, ra, rb, "pearson", "f32", samples=dp))
        _same(ctx.corr_region_max_noalloc(f, ra, rb, "ksg", k=10, samples=dp),
              ctx.corr_region_max(f, ra, rb, "ksg", k=10, samples=dp))


def test_long_k_contraction_two_calls(env):
    pc, ctx, f = env["pc"], env["ctx"], env["f300"]
    for box in ((0, 0, 0, 12, 10, 4, 0, 0, 4, 12, 10, 4), (1, 2, 0, 5, 7, 3, 3, 0, 5, 9, 4, 2)):
        ra, rb = pc.region(*box[:6]), pc.region(*box[6:])
        for prec in ("f16", "f32"):
            _same(ctx.corr_region_max_noalloc(f, ra, rb, "pearson", prec), ctx.corr_region_max(f, ra, rb, "pearson", prec))


def test_wide_tile_contraction_two_calls(env):
    # M = 1000, two 16^3 bricks: 256 tiles of 256 x 256 (the wide-tile
    # kernel); then a smaller ragged pair that takes the 128 x 128 kernel
    pc, ctx, torch = env["pc"], env["ctx"], env["torch"]
    rng = np.random.default_rng(9)
    data = rng.standard_normal((1000, 32 * 16 * 16), dtype=np.float32)
    f = pc.Field(torch.from_numpy(data).cuda(), 32, 16, 16)
    for box in ((0, 0, 0, 16, 16, 16, 16, 0, 0, 16, 16, 16), (1, 0, 2, 15, 16, 13, 16, 3, 0, 14, 11, 16)):
        ra, rb = pc.region(*box[:6]), pc.region(*box[6:])
        for prec in ("f16", "bf16"):
            _say(f"  noalloc wide-tile contraction {prec}, {box}")
            _same(ctx.corr_region_max_noalloc(f, ra, rb, "pearson", prec), ctx.corr_region_max(f, ra, rb, "pearson", prec))


def test_too_large_is_refused(env):
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    # KSG at M = 1000 over two 5000-point boxes: z rows, sorted rows and
    # statistics need about 82 MB, more than the fixed scratch
    data = np.random.default_rng(9).standard_normal((1000, 25 * 20 * 20), dtype=np.float32)
    f = pc.Field(torch.from_numpy(data).cuda(), 25, 20, 20)
    ra, rb = pc.region(0, 0, 0, 25, 20, 10), pc.region(0, 0, 10, 25, 20, 10)
    pairs = torch.from_numpy(np.array([[0, 5000], [2, 5003]], np.int32)).cuda()
    with pytest.raises(pc.CorrError, match="scratch"):
        ctx.corr_region_max_noalloc(f, ra, rb, "ksg", k=10, samples=pairs)
    # the same call fits with smaller boxes, and the context stays usable
    ra, rb = pc.region(0, 0, 0, 25, 20, 4), pc.region(0, 0, 10, 25, 20, 4)
    _same(ctx.corr_region_max_noalloc(f, ra, rb, "ksg", k=10, samples=pairs),
          ctx.corr_region_max(f, ra, rb, "ksg", k=10, samples=pairs))
    del f
