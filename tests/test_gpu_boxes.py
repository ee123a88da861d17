"""corr_box_pairs_max: exhaustive maxima of many small box pairs in one call
(Sec. 3, the brick-pair indicator) against the FP64 oracle, against
corr_region_max on the same boxes, and with the self pairs of one field
excluded."""
import numpy as np
import pytest

import oracle
import synth
from argmax_checks import check_pearson_argmax

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as pc
    e = synth.make_cfg2()
    ctx = pc.Context(0)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    yield dict(torch=torch, pc=pc, e=e, ctx=ctx, f=f)
    ctx.close()


def _boxes(e, n, seed, max_side=6):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        d = rng.integers(1, max_side + 1, 3)
        o = [rng.integers(0, g - dd + 1) for g, dd in zip((e.nx, e.ny, e.nz), d)]
        out.append((int(o[0]), int(o[1]), int(o[2]), int(d[0]), int(d[1]), int(d[2])))
    return out


def test_box_maxima_match_oracle_and_region_max(env):
    pc, ctx, f, e = env["pc"], env["ctx"], env["f"], env["e"]
    ba, bb = _boxes(e, 300, 1), _boxes(e, 300, 2)
    # some overlapping pairs (same box, shifted box) for the self-pair rule
    ba[:10] = bb[:10]
    ba[10:20] = [(x + 1 if x + dx < e.nx else x, y, z, dx, dy, dz) for (x, y, z, dx, dy, dz) in bb[10:20]]
    p = ctx.corr_prepare(f, "pearson", "f32")
    got = ctx.corr_box_pairs_max(p, ba, bb)
    for t in range(300):
        ra, rb = synth.Region(*ba[t]), synth.Region(*bb[t])
        ia, ib = ra.global_indices(e.nx, e.ny), rb.global_indices(e.nx, e.ny)
        if t < 60:  # oracle on a subset (FP64 definition)
            ref = oracle.pearson_region_max_matmul(e.data, ia, ib)
            assert abs(got[t]["value"] - ref["value"]) <= 1e-5, (t, got[t], ref)
            assert got[t]["n_evaluated"] == ref["n_evaluated"]
            if ref["n_evaluated"]:
                check_pearson_argmax(got[t], ref, e.data, ia, ib, 1e-5)
        rm = ctx.corr_region_max(f, pc.region(*ba[t]), pc.region(*bb[t]), "pearson", "f32")
        assert abs(got[t]["value"] - rm["value"]) <= 1e-5 and got[t]["n_evaluated"] == rm["n_evaluated"], t
    p.close()


def test_box_maxima_edges(env):
    torch, pc, ctx, f, e = env["torch"], env["pc"], env["ctx"], env["f"], env["e"]
    p = ctx.corr_prepare(f, "pearson", "f32")
    one = (3, 4, 5, 1, 1, 1)
    # a single point with itself: nothing evaluated
    r = ctx.corr_box_pairs_max(p, [one], [one])
    assert r[0]["n_evaluated"] == 0 and r[0]["pa"] == -1
    # the largest box (4096 points) against a single point
    big = (0, 0, 0, 16, 16, 16)
    r = ctx.corr_box_pairs_max(p, [big], [(40, 20, 10, 1, 1, 1)])
    ia = synth.Region(*big).global_indices(e.nx, e.ny)
    ref = oracle.pearson_region_max_matmul(e.data, ia, np.array([40 + e.nx * (20 + e.ny * 10)], np.int32))
    assert abs(r[0]["value"] - ref["value"]) <= 1e-5 and r[0]["n_evaluated"] == 4096
    with pytest.raises(pc.CorrError):  # more than 4096 points
        ctx.corr_box_pairs_max(p, [(0, 0, 0, 17, 16, 16)], [one])
    with pytest.raises(pc.CorrError):  # outside the grid
        ctx.corr_box_pairs_max(p, [(78, 0, 0, 5, 1, 1)], [one])
    q = ctx.corr_prepare(f, "pearson", "f16")
    with pytest.raises(pc.CorrError):  # FP32 rows only
        ctx.corr_box_pairs_max(q, [one], [one])
    assert ctx.corr_box_pairs_max(p, [], []) == []
    p.close()
    q.close()
