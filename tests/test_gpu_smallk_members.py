"""Small-K contraction (M <= 128) at member counts that pad to each K (64,
112, 128) and at the edges of those, in every precision and every tile
configuration (forced through the tuning table; a configuration a
precision cannot use falls back to the default): the exhaustive region
maximum (Sec. 3) against the oracle's FP64 maximum -- value within the
precision's tolerance, the planted pair as argmax, n_evaluated exact -- and
every configuration giving the same result bit for bit (the MFMA K order
does not depend on the tile shape or the B-fragment lookahead)."""
import json
import os
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

NX, NY, NZ = 40, 20, 8
RA, RB = (0, 0, 0, 20, 20, 8), (20, 0, 0, 20, 20, 8)
TOL = {"f32": 1e-5, "f16": 2e-3, "bf16": 7.9e-3, "f16x3": 1e-5, "bf16x3": 3e-5}
N_CFG = 12


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _gid(x, y, z):
    return x + NX * (y + NY * z)


@pytest.fixture(scope="module")
def env():
    import torch
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as pc
    ctx = pc.Context(0)
    yield dict(torch=torch, pc=pc, ctx=ctx)
    ctx.close()


def _force(ctx, path, K, prec_code, cfg):
    with open(path, "w") as fh:
        fh.write(json.dumps(dict(arch="gfx950", kind=0, K=K, prec=prec_code, na=3200, nb=3200, cfg=cfg, ms=0.0)) + "\n")
    ctx.corr_tune_load(path)


@pytest.mark.parametrize("M,K", [(17, 64), (64, 64), (65, 112), (113, 128), (128, 128)])
def test_every_tile_and_precision(env, tmp_path, M, K):
    torch, pc, ctx = env["torch"], env["pc"], env["ctx"]
    rng = np.random.default_rng(M)
    data = rng.standard_normal((M, NX * NY * NZ)).astype(np.float32)
    p, q = _gid(3, 17, 5), _gid(20 + 11, 2, 6)
    data[:, q] = 0.95 * data[:, p] + 0.05 * rng.standard_normal(M).astype(np.float32)
    f = pc.Field(torch.from_numpy(data).cuda(), NX, NY, NZ)
    ra, rb = pc.region(*RA), pc.region(*RB)
    ia = np.array([_gid(x, y, z) for z in range(8) for y in range(20) for x in range(20)], np.int64)
    ib = np.array([_gid(20 + x, y, z) for z in range(8) for y in range(20) for x in range(20)], np.int64)
    ref = oracle.pearson_region_max_matmul(data, ia, ib)
    assert (ref["pa"], ref["pb"]) == (p, q)
    path = os.path.join(str(tmp_path), "tune.jsonl")
    for prec in ("f32", "f16", "bf16", "f16x3", "bf16x3"):
        outs = []
        for cfg in range(N_CFG):
            _force(ctx, path, K, pc.PREC[prec], cfg)
            got = ctx.corr_region_max(f, ra, rb, "pearson", prec)
            outs.append((got["value"], got["signed_value"], got["pa"], got["pb"], got["n_evaluated"]))
        assert all(o == outs[0] for o in outs), (prec, outs)
        v, sv, pa, pb, n = outs[0]
        assert n == 3200 * 3200
        assert (pa, pb) == (p, q), prec
        assert abs(v - ref["value"]) <= TOL[prec] and sv > 0, (prec, v, ref["value"])
        _say(f"  M={M} K={K} {prec}: {v:.6f} (oracle {ref['value']:.6f}), {N_CFG} tile configurations identical")
