"""One reference point against every grid point (the shape of the paper's
performance table, Sec. 5.2): a 250x352x20 field at M = 100, the pair list
(ref, p) for all 1.76e6 points p, through the pair-list calls the bench
times. Pearson is checked against the FP64 oracle on 20 000 sampled outputs,
KSG counts bit-exactly on 200 of them and MI on 2000; the reference point
with itself gives r = 1 and, without ties, MI = psi(M) - psi(k) exactly.
"""
import sys

import numpy as np
import pytest

import oracle
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
    _say("generating the 250x352x20 M=100 field")
    e = synth.make_field("onetoall-250x352x20-M100", 5, 100, 250, 352, 20, [], [])
    P = e.nx * e.ny * e.nz
    ref = (e.nx // 2) + e.nx * ((e.ny // 2) + e.ny * (e.nz // 2))
    pairs = np.stack([np.full(P, ref, np.int32), np.arange(P, dtype=np.int32)], 1)
    ctx = pc.Context(0)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    yield dict(torch=torch, pc=pc, e=e, ctx=ctx, f=f, pairs=pairs, dpairs=torch.from_numpy(pairs).cuda(), ref=ref)
    ctx.close()


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f16", 2e-3), ("f16x3", 1e-5)])
def test_onetoall_pearson(env, prec, tol):
    ctx, f, e, pairs = env["ctx"], env["f"], env["e"], env["pairs"]
    r = ctx.corr_pearson_pairs(f, env["dpairs"], prec).cpu().numpy()
    sel = np.random.default_rng(11).choice(pairs.shape[0], 20_000, replace=False)
    err = np.max(np.abs(r[sel] - oracle.pearson_pairs(e.data, pairs[sel])))
    _say(f"  one-to-all pearson {prec}: max |err| on 20000 samples {err:.2e}")
    assert err <= tol
    assert abs(r[env["ref"]] - 1.0) <= tol
    assert np.all(np.abs(r) <= 1.0)


def test_onetoall_pearson_prepared_equals(env):
    ctx, f = env["ctx"], env["f"]
    p = ctx.corr_prepare(f, "pearson", "f16")
    a = ctx.corr_pearson_pairs_prepared(p, env["dpairs"])
    b = ctx.corr_pearson_pairs(f, env["dpairs"], "f16")
    assert env["torch"].equal(a, b)
    p.close()


def test_onetoall_ksg(env):
    torch, ctx, f, e, pairs = env["torch"], env["ctx"], env["f"], env["e"], env["pairs"]
    mi = ctx.corr_ksg_mi_pairs(f, env["dpairs"], k=10).cpu().numpy()
    sel = np.random.default_rng(12).choice(pairs.shape[0], 2000, replace=False)
    mi_ref, cnt_ref = oracle.ksg_pairs(e.data, pairs[sel], 10)
    assert np.max(np.abs(mi[sel] - mi_ref)) <= 1e-5
    sub = torch.from_numpy(np.ascontiguousarray(pairs[sel[:200]])).cuda()
    _, cnt = ctx.corr_ksg_mi_pairs(f, sub, k=10, counts=True)
    assert np.array_equal(cnt.cpu().numpy(), cnt_ref[:200])
    # the reference with itself: where no two members tie, n_x = n_y = k - 1
    # for every sample, so MI = psi(M) - psi(k)
    self_pair = np.array([[env["ref"], env["ref"]]], np.int32)
    mi_self, cnt_self = oracle.ksg_pairs(e.data, self_pair, 10)
    assert abs(mi[env["ref"]] - mi_self[0]) <= 1e-5
    if np.all(cnt_self == 9):
        assert abs(mi[env["ref"]] - (oracle.digamma_int(100) - oracle.digamma_int(10))) <= 1e-5
