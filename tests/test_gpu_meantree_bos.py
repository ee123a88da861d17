"""Batched BOS on mean-tree levels (Sec. 3.3: where the data is aggregated,
BOS runs on the level; Sec. 5 compares f = 2 and f = 4 with the initial data).

The level is built on the GPU (corr_block_means) and BOS runs on it through
the same entry points as on the initial data. Checks: every value in a pair's
history is the oracle's Pearson (or KSG) on the oracle's own level (FP64 block
means rounded once to FP32, as the level is stored), the oracle replays the
GPU's batches on the level's cell grid, and no estimate exceeds the
exhaustive maximum on the level.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import aggregate_ref as AG
from oracle import bos_ref as B
from test_oracle_bos import replay_iterations

pytestmark = pytest.mark.gpu

TIMEOUT_S = 60.0


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    _say("meantree bos fixture: importing torch")
    import torch
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as pc
    e = synth.make_context(4, 2, (12, 12, 6), M=100, seed=21, n_groups=3, blob_r=2.0, min_region_gap=2)
    ctx = pc.Context(0)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    pairs = synth.region_pair_list(len(e.regions))
    yield dict(torch=torch, pc=pc, e=e, ctx=ctx, f=f, pairs=pairs)
    ctx.close()


class _Reg:
    def __init__(self, t):
        self.x0, self.y0, self.z0, self.dx, self.dy, self.dz = t


def _oracle_cfg(c):
    return B.BosConfig(n_init=c.n_init, n_total=c.n_total, n_uniform=c.n_uniform, n_local=c.n_local, kappa=c.kappa,
                       lengthscale=c.lengthscale, local_sd=c.local_sd, jitter=c.jitter, seed=c.seed)


@pytest.mark.parametrize("fct,measure", [(2, "pearson"), (4, "pearson"), (2, "ksg")])
def test_bos_on_level_matches_oracle(env, fct, measure):
    pc, ctx, e, f, pairs = (env[k] for k in ("pc", "ctx", "e", "f", "pairs"))
    lvl = ctx.corr_block_means(f, fct, "f32")
    nxl, nyl, nzl = AG.level_dims(e.nx, e.ny, e.nz, fct)
    assert (lvl.nx, lvl.ny, lvl.nz) == (nxl, nyl, nzl)
    ref_level = AG.block_means(e.data, e.nx, e.ny, e.nz, fct).astype(np.float32)
    # both sides sum a block's FP32 values in FP64 (exactly, at these magnitudes)
    # and round the mean once, so the stored level is the oracle's bit for bit;
    # the KSG counts below rely on that
    assert np.array_equal(lvl.data[:, :lvl.P].cpu().numpy(), ref_level)
    regs_o = [_Reg(AG.region_at_level(r.as_tuple(), fct)) for r in e.regions]
    regs = [pc.region_at_level(pc.region(*r.as_tuple()), fct) for r in e.regions]
    for ro, rg in zip(regs_o, regs):
        assert (ro.x0, ro.y0, ro.z0, ro.dx, ro.dy, ro.dz) == (rg.x0, rg.y0, rg.z0, rg.dx, rg.dy, rg.dz)
    sel = pairs if measure == "pearson" else pairs[:6]
    cfg = pc.bos_defaults(seed=4, measure=measure, k=10)
    bos = pc.Bos(ctx, lvl, regs, sel, cfg)
    bos.bos_set_launch("graph", TIMEOUT_S)
    bos.bos_run()
    res = bos.bos_results()
    ocfg = _oracle_cfg(bos.cfg)
    full = 0
    for p, (ia, ib) in enumerate(sel):
        cells, vals = bos.bos_history(p)
        ra, rb = regs_o[ia], regs_o[ib]
        pa, pb = B.cells_to_points(cells.astype(np.int64), ra, rb, nxl, nyl)
        pp = np.stack([pa, pb], 1).astype(np.int32)
        if measure == "pearson":
            ref = np.abs(oracle.pearson_pairs(ref_level, pp))
        else:
            ref, _ = oracle.ksg_pairs(ref_level, pp, 10, want_counts=False)
        assert np.max(np.abs(vals - ref)) <= 1e-5, p
        assert len({tuple(c) for c in cells}) == cells.shape[0] <= cfg.n_total
        assert res[p]["value"] == pytest.approx(float(vals.max()), abs=1e-7)
        dims = (ra.dx, ra.dy, ra.dz, rb.dx, rb.dy, rb.dz)
        m, t = replay_iterations(ocfg, p, dims, cells.astype(np.int64), vals)
        full += int(m == t)
        if measure == "pearson":
            ex = ctx.corr_region_max(lvl, regs[ia], regs[ib], "pearson", "f32")
            assert res[p]["value"] <= ex["value"] + 1e-5
    _say(f"  f={fct} {measure}: {len(sel)} pairs on the {nxl}x{nyl}x{nzl} level, "
         f"batches reproduced exactly for {full}/{len(sel)}")
    assert full >= 0.9 * len(sel)
    bos.close()
