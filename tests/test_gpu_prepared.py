"""Prepared fields (corr_prepare): pair-list calls on a field standardised
once give exactly the results of the calls that standardise on every call
(same kernels, same rows), and those match the FP64 oracle (Sec. 3.2).
"""
import sys

import numpy as np
import pytest

import oracle
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
    e = synth.make_cfg2()
    ctx = pc.Context(0)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    u, v, _ = synth.make_two_variables()
    fu = pc.Field(torch.from_numpy(u.data).cuda(), u.nx, u.ny, u.nz)
    fv = pc.Field(torch.from_numpy(v.data.astype(np.float16)).cuda(), v.nx, v.ny, v.nz)
    yield dict(torch=torch, pc=pc, e=e, ctx=ctx, f=f, u=u, v=v, fu=fu, fv=fv)
    ctx.close()


@pytest.mark.parametrize("prec", ["f32", "f16", "f16x3", "bf16", "bf16x3"])
def test_pearson_prepared_equals_per_call(env, prec):
    torch, ctx, f, e = env["torch"], env["ctx"], env["f"], env["e"]
    pairs = synth.random_pairs(301, 300_000, e.P)
    dp = torch.from_numpy(pairs).cuda()
    p = ctx.corr_prepare(f, "pearson", prec)
    got = ctx.corr_pearson_pairs_prepared(p, dp).cpu().numpy()
    ref = ctx.corr_pearson_pairs(f, dp, prec).cpu().numpy()
    assert np.array_equal(got, ref)
    sel = np.random.default_rng(3).choice(pairs.shape[0], 20_000, replace=False)
    err = np.max(np.abs(got[sel] - oracle.pearson_pairs(e.data, pairs[sel])))
    _say(f"  prepared pearson {prec}: max |err| vs oracle {err:.2e}")
    assert err <= TOL[prec]
    p.close()


def test_ksg_prepared_equals_per_call_with_counts(env):
    torch, ctx, f, e = env["torch"], env["ctx"], env["f"], env["e"]
    pairs = synth.random_pairs(302, 50_000, e.P)
    dp = torch.from_numpy(pairs).cuda()
    p = ctx.corr_prepare(f, "ksg")
    mi, cnt = ctx.corr_ksg_mi_pairs_prepared(p, dp, k=10, counts=True)
    mi0, cnt0 = ctx.corr_ksg_mi_pairs(f, dp, k=10, counts=True)
    assert torch.equal(mi, mi0) and torch.equal(cnt, cnt0)
    mi_ref, cnt_ref = oracle.ksg_pairs(e.data, pairs[:300], 10)
    assert np.array_equal(cnt[:300].cpu().numpy(), cnt_ref)
    assert np.max(np.abs(mi[:300].cpu().numpy() - mi_ref)) <= 1e-5
    p.close()


def test_two_prepared_variables(env):
    """A != B, B stored FP16: both measures, against the per-call form and the oracle."""
    torch, ctx, u, v, fu, fv = env["torch"], env["ctx"], env["u"], env["v"], env["fu"], env["fv"]
    rng = np.random.default_rng(4)
    pairs = np.stack([rng.integers(0, u.P, 20_000), rng.integers(0, v.P, 20_000)], 1).astype(np.int32)
    dp = torch.from_numpy(pairs).cuda()
    pu, pv = ctx.corr_prepare(fu, "pearson", "f32"), ctx.corr_prepare(fv, "pearson", "f32")
    r = ctx.corr_pearson_pairs_prepared(pu, dp, B=pv)
    assert torch.equal(r, ctx.corr_pearson_pairs(fu, dp, "f32", B=fv))
    ku, kv = ctx.corr_prepare(fu, "ksg"), ctx.corr_prepare(fv, "ksg")
    mi, cnt = ctx.corr_ksg_mi_pairs_prepared(ku, dp, k=10, B=kv, counts=True)
    mi0, cnt0 = ctx.corr_ksg_mi_pairs(fu, dp, k=10, B=fv, counts=True)
    assert torch.equal(mi, mi0) and torch.equal(cnt, cnt0)
    v16 = v.data.astype(np.float16)
    assert np.max(np.abs(r.cpu().numpy()[:5000] - oracle.pearson_pairs(u.data, pairs[:5000], data_b=v16))) <= 1e-5
    _, cref = oracle.ksg_pairs(u.data, pairs[:200], 10, data_b=v16)
    assert np.array_equal(cnt[:200].cpu().numpy(), cref)
    for h in (pu, pv, ku, kv):
        h.close()


def test_prepared_errors(env):
    torch, pc, ctx, f = env["torch"], env["pc"], env["ctx"], env["f"]
    dp = torch.zeros((4, 2), dtype=torch.int32, device="cuda")
    pk = ctx.corr_prepare(f, "ksg")
    pp = ctx.corr_prepare(f, "pearson", "f16")
    pq = ctx.corr_prepare(f, "pearson", "f32")
    with pytest.raises(pc.CorrError):  # a KSG preparation is not a Pearson one
        ctx.corr_pearson_pairs_prepared(pk, dp)
    with pytest.raises(pc.CorrError):  # nor the other way round
        ctx.corr_ksg_mi_pairs_prepared(pp, dp)
    with pytest.raises(pc.CorrError):  # precisions must agree
        ctx.corr_pearson_pairs_prepared(pp, dp, B=pq)
    with pytest.raises(pc.CorrError):  # k out of range
        ctx.corr_ksg_mi_pairs_prepared(pk, dp, k=100)
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    assert ctx.corr_pearson_pairs_prepared(pp, empty).numel() == 0
    for h in (pk, pp, pq):
        h.close()
