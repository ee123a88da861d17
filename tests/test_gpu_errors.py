"""Error paths that need a context: CORR_EUNSUPPORTED for sizes and
precisions the library does not handle, CORR_ENOMEM when a call's
workspaces would pass the context's cap (returned before any work is
enqueued, the context usable afterwards), and calls that switch streams on
one context (ordered by the library, same results). Also the peak probes
(corr_peaks.h): each runs and writes its words, bad arguments give
CORR_EINVAL."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as pc
    from paper_2309_03308_amd import _lib
    e = synth.make_cfg1()
    ctx = pc.Context(0)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    ra, rb = [pc.region(*r.as_tuple()) for r in e.regions]
    yield dict(torch=torch, pc=pc, lib=_lib, e=e, ctx=ctx, f=f, ra=ra, rb=rb)
    ctx.close()


def _status(fn, pc):
    with pytest.raises(pc.CorrError) as ei:
        fn()
    return ei.value.status


def test_unsupported(env):
    torch, pc, lib, ctx, f, ra, rb = (env[k] for k in ("torch", "pc", "lib", "ctx", "f", "ra", "rb"))
    pairs = torch.zeros((8, 2), dtype=torch.int32, device="cuda")
    assert _status(lambda: ctx.corr_ksg_mi_pairs(f, pairs, k=40), pc) == lib.CORR_EUNSUPPORTED  # k > 31
    assert _status(lambda: ctx.corr_region_max(f, ra, rb, "ksg", k=33), pc) == lib.CORR_EUNSUPPORTED
    # a precision code outside the enumeration, through the raw ABI
    out = lib.corr_max()
    st = ctx.L.corr_region_max(ctx.h, lib.ctypes.byref(f.c), lib.ctypes.byref(ra), lib.ctypes.byref(f.c),
                               lib.ctypes.byref(rb), 0, 99, 10, None, 0, lib.ctypes.byref(out), None)
    assert st == lib.CORR_EUNSUPPORTED
    # KSG at more members than the LDS layout holds
    big = pc.Field(torch.zeros((2100, 8), dtype=torch.float32, device="cuda"), 2, 2, 2)
    assert _status(lambda: ctx.corr_ksg_mi_pairs(big, pairs[:2] * 0, k=10), pc) == lib.CORR_EUNSUPPORTED
    assert _status(lambda: ctx.corr_prepare(big, "ksg"), pc) == lib.CORR_EUNSUPPORTED


def test_workspace_limit_gives_enomem_and_recovers(env):
    pc, lib, e, ra, rb = env["pc"], env["lib"], env["e"], env["ra"], env["rb"]
    torch = env["torch"]
    ctx = pc.Context(0)  # a fresh context: no workspace held yet
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    ctx.set_workspace_limit(4096)
    assert _status(lambda: ctx.corr_region_max(f, ra, rb, "pearson", "f32"), pc) == lib.CORR_ENOMEM
    assert b"workspace limit" in ctx.L.corr_last_error()
    ctx.set_workspace_limit(0)
    got = ctx.corr_region_max(f, ra, rb, "pearson", "f32")
    ref = env["ctx"].corr_region_max(env["f"], ra, rb, "pearson", "f32")
    assert got == ref
    # a cap above what is held already lets the same call through again
    ctx.set_workspace_limit(64 << 20)
    assert ctx.corr_region_max(f, ra, rb, "pearson", "f32") == ref
    ctx.close()


def test_stream_switch_is_ordered(env):
    torch, ctx, f, ra, rb = env["torch"], env["ctx"], env["f"], env["ra"], env["rb"]
    ref = ctx.corr_region_max(f, ra, rb, "pearson", "f16x3")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    pairs = torch.from_numpy(synth.region_pairs_uniform(3, 5000, env["e"].regions[0], env["e"].regions[1],
                                                        env["e"].nx, env["e"].ny)).cuda()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        r1 = ctx.corr_pearson_pairs(f, pairs, "f32")
    with torch.cuda.stream(s2):
        mi2 = ctx.corr_ksg_mi_pairs(f, pairs, k=10)
        got = ctx.corr_region_max(f, ra, rb, "pearson", "f16x3")
    torch.cuda.synchronize()
    assert got == ref
    r0 = ctx.corr_pearson_pairs(f, pairs, "f32")
    mi0 = ctx.corr_ksg_mi_pairs(f, pairs, k=10)
    torch.cuda.synchronize()
    assert torch.equal(r1, r0) and torch.equal(mi2, mi0)
    assert np.all(np.isfinite(r1.cpu().numpy()))


def test_peak_probes(env):
    torch, pc, lib = env["torch"], env["pc"], env["lib"]
    nb = 64
    o32 = torch.full((nb * 256,), float("nan"), dtype=torch.float32, device="cuda")
    o64 = torch.full((nb * 256,), float("nan"), dtype=torch.float64, device="cuda")
    oi = torch.zeros(nb * 256, dtype=torch.int32, device="cuda")
    pc.corr_peak_mfma_f16(nb, 10, o32)
    torch.cuda.synchronize()
    assert torch.isfinite(o32).all()
    o32.fill_(float("nan"))
    pc.corr_peak_valu_f32(nb, 10, o32)
    pc.corr_peak_valu_f64(nb, 10, o64)
    pc.corr_peak_valu_med3(nb, 10, o32)
    torch.cuda.synchronize()
    assert torch.isfinite(o32).all() and torch.isfinite(o64).all()
    pc.corr_peak_lds(nb, 4, oi)
    buf = torch.arange(1 << 20, dtype=torch.int32, device="cuda")
    pc.corr_peak_hbm_read(buf, nb, oi)
    torch.cuda.synchronize()
    assert _status(lambda: pc.corr_peak_lds(0, 4, oi), pc) == lib.CORR_EINVAL
    pc.corr_peak_mfma_f16(nb, 10, o32, random_operands=False)
    assert _status(lambda: pc.corr_peak_mfma_f16(nb, 0, o32), pc) == lib.CORR_EINVAL
    assert _status(lambda: pc.corr_peak_hbm_read(buf[1:5], nb, oi), pc) == lib.CORR_EINVAL  # misaligned
    with pytest.raises(ValueError):  # fewer than n_blocks * 256 words: refused by the binding
        pc.corr_peak_valu_f32(nb + 1, 10, o32)
