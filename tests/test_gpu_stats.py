"""Per-point statistics for long member rows (M >= 256) on the GPU against
the oracle: the means and inverse standard deviations that feed KSG must be
bit-identical (both sides add the members in member order in FP64), over
ragged point counts and member counts that leave partial sweeps, for both
kernels (all members of 16 points staged in LDS for up to 32768 points and
64 KiB of members, one thread per point otherwise) and both storage types.
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
    ctx = pc.Context(0)
    yield dict(torch=torch, pc=pc, ctx=ctx)
    ctx.close()


def _field_data(M, dims, dtype, seed):
    rng = np.random.default_rng(seed)
    P = dims[0] * dims[1] * dims[2]
    # a common member signal, per-point offsets and scales, and a few constant points
    d = (rng.standard_normal((M, 1)) * 0.7 + rng.standard_normal((M, P))) * rng.uniform(0.2, 3.0, P) \
        + rng.uniform(-5, 5, P)
    d[:, ::97] = 1.5
    return np.ascontiguousarray(d.astype(dtype))


@pytest.mark.parametrize("M,dims,dtype", [
    (300, (37, 5, 3), np.float32),      # 555 points staged in LDS
    (256, (17, 1, 1), np.float16),      # fewer points than one workgroup
    (1000, (16, 16, 16), np.float16),   # a 16^3 focus brick
    (1000, (41, 31, 27), np.float16),   # 34317 points: one thread per point
    (257, (40, 40, 21), np.float32),    # 33600 points: one thread per point
    (257, (40, 40, 20), np.float32),    # 32000 points staged in LDS
    (1024, (9, 7, 5), np.float32),      # 64 KiB of members per 16 points
    (1025, (9, 7, 5), np.float32),      # above 64 KiB: one thread per point
    (2048, (5, 4, 3), np.float16),      # 64 KiB of FP16 members
])
def test_stats_bitwise_long_rows(env, M, dims, dtype):
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    data = _field_data(M, dims, dtype, seed=M)
    _say(f"  stats M={M} dims={dims} {np.dtype(dtype).name}")
    f = pc.Field(torch.from_numpy(data).cuda(), *dims)
    mu, inv, sig = ctx.corr_standardize(f)
    _, s2, mu32, inv32 = oracle.stats(data)
    assert np.array_equal(mu.cpu().numpy(), mu32)
    assert np.array_equal(inv.cpu().numpy(), inv32)
    assert np.allclose(sig.cpu().numpy(), np.sqrt(s2 / M), rtol=1e-6)
    assert np.all(inv32[::97] == 0.0)


def test_ksg_counts_long_rows_region(env):
    # KSG pairs inside one brick of a 300-member field: counts bit-exact
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    dims = (24, 20, 9)
    data = _field_data(300, dims, np.float32, seed=5)
    data[:, ::97] += np.random.default_rng(2).standard_normal((300, 1)).astype(np.float32)  # no constant points
    f = pc.Field(torch.from_numpy(data).cuda(), *dims)
    pairs = synth.random_pairs(11, 300, dims[0] * dims[1] * dims[2])
    mi, cnt = ctx.corr_ksg_mi_pairs(f, torch.from_numpy(pairs).cuda(), k=10, counts=True)
    mi_ref, cnt_ref = oracle.ksg_pairs(data, pairs, 10)
    assert np.array_equal(cnt.cpu().numpy(), cnt_ref)
    assert np.max(np.abs(mi.cpu().numpy() - mi_ref)) <= 1e-5


@pytest.mark.parametrize("prec", ["f32", "f16x3"])
def test_region_max_fp32_statistics_at_256(env, prec):
    # M = 256 is the largest member count with FP32 accumulation for Pearson
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    dims = (20, 12, 8)
    data = _field_data(256, dims, np.float32, seed=9)
    data[:, ::97] += np.random.default_rng(1).standard_normal((256, 1)).astype(np.float32)  # no constant points
    f = pc.Field(torch.from_numpy(data).cuda(), *dims)
    ra, rb = pc.region(0, 0, 0, 10, 12, 8), pc.region(10, 0, 0, 10, 12, 8)
    got = ctx.corr_region_max(f, ra, rb, "pearson", prec)
    ia = synth.Region(0, 0, 0, 10, 12, 8).global_indices(*dims[:2])
    ib = synth.Region(10, 0, 0, 10, 12, 8).global_indices(*dims[:2])
    ref = oracle.pearson_region_max_matmul(data, ia, ib)
    assert abs(got["value"] - ref["value"]) <= 1e-5
    assert got["n_evaluated"] == ia.size * ib.size
