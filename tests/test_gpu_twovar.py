"""Correlation between two variables of one ensemble (field A from one
variable, field B from another): pairs, KSG counts and region maxima against
the FP64 oracle, with mixed storage types. A point is never "the same" across
two fields, so no self pair is excluded even when the regions coincide.
"""
import sys

import numpy as np
import pytest

import oracle
from argmax_checks import check_pearson_argmax
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
    U, V, regs = synth.make_two_variables(nx=24, ny=16, nz=8, M=100, seed=7, rho=0.8)
    ctx = pc.Context(0)
    fu = pc.Field(torch.from_numpy(U.data).cuda(), U.nx, U.ny, U.nz)
    Vh = np.ascontiguousarray(V.data.astype(np.float16))  # V is stored as FP16; its FP16 values are the input
    fv = pc.Field(torch.from_numpy(Vh).cuda(), V.nx, V.ny, V.nz)
    yield dict(torch=torch, pc=pc, ctx=ctx, U=U, V=V, Vh=Vh, fu=fu, fv=fv, regs=regs)
    ctx.close()


def test_pairs_across_variables(env):
    torch, ctx = env["torch"], env["ctx"]
    U, Vh = env["U"], env["Vh"]
    P = U.nx * U.ny * U.nz
    pairs = synth.random_pairs(31, 20000, P, distinct=False)
    pd = torch.from_numpy(pairs).cuda()
    ref = oracle.pearson_pairs(U.data, pairs, data_b=Vh)
    for prec, tol in (("f32", 1e-5), ("f16x3", 1e-5), ("f16", 2e-3)):
        r = ctx.corr_pearson_pairs(env["fu"], pd, prec, B=env["fv"]).cpu().numpy()
        _say(f"  two-variable pairs {prec}: max err {np.abs(r - ref).max():.2e}")
        assert np.abs(r - ref).max() <= tol
    mi, cnt = ctx.corr_ksg_mi_pairs(env["fu"], pd, k=10, B=env["fv"], counts=True)
    mi_ref, cnt_ref = oracle.ksg_pairs(U.data, pairs, 10, data_b=Vh)
    assert np.array_equal(cnt.cpu().numpy(), cnt_ref)
    assert np.abs(mi.cpu().numpy() - mi_ref).max() <= 1e-5


@pytest.mark.parametrize("which", [(0, 1), (0, 0)])
def test_region_max_across_variables(env, which):
    pc, ctx, U, Vh = env["pc"], env["ctx"], env["U"], env["Vh"]
    ra, rb = env["regs"][which[0]], env["regs"][which[1]]
    ia, ib = ra.global_indices(U.nx, U.ny), rb.global_indices(U.nx, U.ny)
    ref = oracle.pearson_region_max_matmul(U.data, ia, ib, data_b=Vh, same_field=False)
    got = ctx.corr_region_max(env["fu"], pc.region(*ra.as_tuple()), pc.region(*rb.as_tuple()), "pearson", "f16x3",
                              B=env["fv"])
    _say(f"  region max {which}: gpu {got['value']:.6f} oracle {ref['value']:.6f}")
    assert abs(got["value"] - ref["value"]) <= 1e-5
    assert got["n_evaluated"] == ia.size * ib.size  # nothing excluded across fields
    check_pearson_argmax(got, ref, U.data, ia, ib, 1e-5, data_b=Vh, same_field=False)
    if which == (0, 1):
        assert ref["value"] > 0.6  # the planted cross-variable blob


def test_sampled_ksg_region_max_across_variables(env):
    torch, pc, ctx, U, Vh = env["torch"], env["pc"], env["ctx"], env["U"], env["Vh"]
    ra, rb = env["regs"]
    s = synth.region_pairs_uniform(5, 4000, ra, rb, U.nx, U.ny)
    ia, ib = ra.global_indices(U.nx, U.ny), rb.global_indices(U.nx, U.ny)
    la, lb = np.searchsorted(ia, s[:, 0]), np.searchsorted(ib, s[:, 1])
    mi, _ = oracle.ksg_pairs(U.data, s, 10, data_b=Vh, want_counts=False)
    ref = oracle.region_max_from_values(mi, la, lb, s[:, 0], s[:, 1], use_abs=False)
    got = ctx.corr_region_max(env["fu"], pc.region(*ra.as_tuple()), pc.region(*rb.as_tuple()), "ksg", k=10,
                              B=env["fv"], samples=torch.from_numpy(s).cuda())
    assert abs(got["value"] - ref["value"]) <= 1e-5 and got["n_evaluated"] == s.shape[0]
    top = np.sort(mi)[-2:]
    if top[1] - top[0] > 2e-5:
        assert (got["pa"], got["pb"]) == (ref["pa"], ref["pb"])
