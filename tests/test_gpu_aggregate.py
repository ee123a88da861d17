"""Mean-tree levels on the GPU (corr_block_means) against the oracle.

Bars: FP32 output within one FP32 ulp of the FP64 mean (both sides sum in
FP64 and round once; only the summation order differs), FP16 output within
one FP16 ulp. Cases: ragged grids that span several 64-column segments and
end in partial blocks on every axis, f in {1, 2, 4, 8, 64}, FP16 input,
padded member strides (both kernels: the vector one for f = 2, 4 over
aligned rows whole in x, the lane-group one otherwise), error handling; at the 180-member 640 x 704 x 64 shape
the benchmark times, sampled blocks (edges included) are checked one by one.
The composed path -- brick maxima estimated on a level -- is compared with
the oracle's maxima on the oracle's own level.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import aggregate_ref as AG

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


def _ulps(got, ref, dt):
    # distance in units of the output type's spacing at the reference (plus
    # 1e-12 absolute for means that cancel to almost nothing)
    sp = np.spacing(np.abs(ref.astype(dt))).astype(np.float64) + 1e-12
    return np.abs(got.astype(np.float64) - ref) / sp


# nx a multiple of f with aligned rows takes the vector kernel (f = 2, 4);
# the odd member stride P + 7 and the ragged nx take the lane-group kernel
@pytest.mark.parametrize("dims", [(37, 13, 5), (130, 7, 9), (64, 64, 4), (36, 5, 3), (1, 3, 2)])
@pytest.mark.parametrize("f", [1, 2, 4, 8, 64])
@pytest.mark.parametrize("io", ["f32-f32", "f32-f16", "f16-f32", "f16-f16"])
@pytest.mark.parametrize("pad", [0, 7])
def test_block_means_parity(env, dims, f, io, pad):
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    nx, ny, nz = dims
    din, dout = io.split("-")
    rng = np.random.default_rng(hash((dims, f)) & 0xffff)
    M, P = 5, nx * ny * nz
    data = (rng.standard_normal((M, P)) * 3 + 1).astype(np.float32 if din == "f32" else np.float16)
    padded = np.zeros((M, P + pad), data.dtype)  # member stride P + pad
    padded[:, :P] = data
    A = pc.Field(torch.from_numpy(padded).cuda(), nx, ny, nz)
    lvl = ctx.corr_block_means(A, f, dout)
    got = lvl.data.cpu().numpy()
    ref = AG.block_means(data.astype(np.float32), nx, ny, nz, f)
    assert (lvl.nx, lvl.ny, lvl.nz) == AG.level_dims(nx, ny, nz, f)
    assert got.shape == ref.shape
    u = _ulps(got, ref, np.float32 if dout == "f32" else np.float16)
    assert u.max() <= 1.0, (u.max(), np.unravel_index(np.argmax(u), u.shape))


def test_output_stride_and_member_range(env):
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    nx, ny, nz, f = 70, 9, 6, 4
    rng = np.random.default_rng(5)
    data = rng.standard_normal((19, nx * ny * nz)).astype(np.float32)
    A = pc.Field(torch.from_numpy(data).cuda(), nx, ny, nz)
    NX, NY, NZ = AG.level_dims(nx, ny, nz, f)
    out = torch.full((19, NX * NY * NZ + 5), 7.0, device="cuda")
    lvl = ctx.corr_block_means(A, f, "f32", out=out)
    o = out.cpu().numpy()
    assert np.all(o[:, NX * NY * NZ:] == 7.0)  # the padding is not written
    assert _ulps(o[:, :NX * NY * NZ], AG.block_means(data, nx, ny, nz, f), np.float32).max() <= 1.0
    assert lvl.M == 19


def test_block_means_bad_arguments(env):
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    A = pc.Field(torch.zeros((3, 8 * 8 * 8), device="cuda"), 8, 8, 8)
    for f in (0, 3, 128, -2):
        with pytest.raises(pc.CorrError) as ei:
            ctx.corr_block_means(A, f)
        assert ei.value.status == 1
    L, h = ctx.L, ctx.h
    import ctypes
    out = torch.empty((3, 64), device="cuda")
    assert L.corr_block_means(h, ctypes.byref(A.c), 2, 7, ctypes.c_void_p(out.data_ptr()), 0, None) == 2
    assert L.corr_block_means(h, ctypes.byref(A.c), 2, 0, None, 0, None) == 1
    assert L.corr_block_means(h, ctypes.byref(A.c), 2, 0, ctypes.c_void_p(out.data_ptr()), 63, None) == 1


def test_block_means_full_shape_sampled(env):
    # 180 members on 640 x 704 x 64 (20.8 GB FP32), the shape the benchmark times
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    M, nx, ny, nz = 180, 640, 704, 64
    _say("mean tree full shape: generating 180 x 640 x 704 x 64 on the device")
    X = synth.smooth_field_torch(M, nx, ny, nz, seed=11)
    A = pc.Field(X, nx, ny, nz)
    rng = np.random.default_rng(12)
    vol = X.view(M, nz, ny, nx)
    for f in (2, 4):
        _say(f"  f = {f}")
        lvl = ctx.corr_block_means(A, f, "f32")
        NX, NY, NZ = lvl.nx, lvl.ny, lvl.nz
        L = lvl.data.view(M, NZ, NY, NX)
        picks = [(M - 1, NX - 1, NY - 1, NZ - 1), (0, 0, 0, 0)]
        picks += [tuple(int(v) for v in (rng.integers(M), rng.integers(NX), rng.integers(NY), rng.integers(NZ)))
                  for _ in range(200)]
        for m, bx, by, bz in picks:
            blk = vol[m, f * bz:f * bz + f, f * by:f * by + f, f * bx:f * bx + f].cpu().numpy()
            ref = AG.block_means(blk.reshape(1, -1), blk.shape[2], blk.shape[1], blk.shape[0], f)[0, 0]
            got = float(L[m, bz, by, bx])
            assert abs(got - ref) <= np.spacing(np.float32(abs(ref))), (f, m, bx, by, bz, got, ref)
        del lvl, L
    del A, X, vol
    torch.cuda.empty_cache()


def test_maxima_on_levels(env):
    # brick maxima estimated on the levels (Sec. 5): the library's level and
    # maximum against the oracle's level and exhaustive maximum
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    e = synth.make_context(3, 2, (32, 32, 20), M=100, seed=21, n_groups=2, min_region_gap=2)
    A = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    pairs = synth.region_pair_list(len(e.regions))
    for f in (2, 4):
        lvl = ctx.corr_block_means(A, f, "f32")
        ref_lvl = AG.block_means(e.data, e.nx, e.ny, e.nz, f).astype(np.float32)
        NX, NY = lvl.nx, lvl.ny
        for a, b in pairs:
            ra = pc.region_at_level(pc.region(*e.regions[a].as_tuple()), f)
            rb = pc.region_at_level(pc.region(*e.regions[b].as_tuple()), f)
            ia = synth.Region(ra.x0, ra.y0, ra.z0, ra.dx, ra.dy, ra.dz).global_indices(NX, NY)
            ib = synth.Region(rb.x0, rb.y0, rb.z0, rb.dx, rb.dy, rb.dz).global_indices(NX, NY)
            ref = oracle.pearson_region_max_matmul(ref_lvl, ia, ib)
            got = ctx.corr_region_max(lvl, ra, rb, "pearson", "f16x3")
            assert abs(got["value"] - ref["value"]) <= 1e-5, (f, a, b, got, ref)
            assert got["n_evaluated"] == ia.size * ib.size
        _say(f"  f = {f}: {len(pairs)} brick maxima on the level match the oracle")
