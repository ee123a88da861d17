"""GPU batched BOS against the FP64 oracle (Sec. 3.1).

Step parity: the oracle replays every pair's GPU history batch by batch and
must reproduce the cells the GPU chose (same candidates, believer picks,
rounding and dedupe). Objective values match the oracle's Pearson / KSG.
Direct launches and the captured-graph launches give bit-identical
histories. Every library wait is bounded (bos_set_launch), so a kernel that
did not finish would fail the test instead of blocking it.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import bos_ref as B
from test_oracle_bos import replay_iterations

pytestmark = pytest.mark.gpu

# every wait of the library for the GPU gives up after this many seconds
TIMEOUT_S = 60.0


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    _say("bos fixture: importing torch")
    import torch
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as pc
    e = synth.make_context(4, 2, (12, 12, 6), M=100, seed=21, n_groups=3, blob_r=2.0, min_region_gap=2)
    _say("bos fixture: creating context")
    ctx = pc.Context(0)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    regions = [pc.region(*r.as_tuple()) for r in e.regions]
    pairs = synth.region_pair_list(len(e.regions))
    yield dict(torch=torch, pc=pc, e=e, ctx=ctx, f=f, regions=regions, pairs=pairs)
    ctx.close()


def _dims(e, pair):
    ra, rb = e.regions[pair[0]], e.regions[pair[1]]
    return (ra.dx, ra.dy, ra.dz, rb.dx, rb.dy, rb.dz)


def _oracle_cfg(c):
    return B.BosConfig(n_init=c.n_init, n_total=c.n_total, n_uniform=c.n_uniform, n_local=c.n_local, kappa=c.kappa,
                       lengthscale=c.lengthscale, local_sd=c.local_sd, jitter=c.jitter, seed=c.seed)


def _check_history(env, bos, measure, pairs_to_check):
    e, cfg = env["e"], _oracle_cfg(bos.cfg)
    res = bos.bos_results()
    full = 0
    for p in pairs_to_check:
        cells, vals = bos.bos_history(p)
        ra, rb = e.regions[env["pairs"][p][0]], e.regions[env["pairs"][p][1]]
        pa, pb = B.cells_to_points(cells.astype(np.int64), ra, rb, e.nx, e.ny)
        pp = np.stack([pa, pb], 1).astype(np.int32)
        if measure == "pearson":
            ref = np.abs(oracle.pearson_pairs(e.data, pp))
            tol = 1e-5
        else:
            ref, _ = oracle.ksg_pairs(e.data, pp, 10, want_counts=False)
            tol = 1e-5
        assert np.max(np.abs(vals - ref)) <= tol, p
        assert cells.shape[0] <= 100 and len({tuple(c) for c in cells}) == cells.shape[0]
        assert res[p]["n_evaluated"] == cells.shape[0]
        assert res[p]["value"] == pytest.approx(float(vals.max()), abs=1e-7)
        m, t = replay_iterations(cfg, p, _dims(e, env["pairs"][p]), cells.astype(np.int64), vals)
        full += int(m == t)
    return full, res


def _bos(env, cfg, pairs=None, mode="graph"):
    pc = env["pc"]
    b = pc.Bos(env["ctx"], env["f"], env["regions"], env["pairs"] if pairs is None else pairs, cfg)
    b.bos_set_launch(mode, TIMEOUT_S)
    return b


def _histories(bos, n):
    return [bos.bos_history(p) for p in range(n)]


def test_bos_pearson_plain_launch_matches_oracle_replay(env):
    pc = env["pc"]
    _say(f"  pearson BOS (direct launches) over {len(env['pairs'])} pairs: create")
    bos = _bos(env, pc.bos_defaults(seed=3), mode="plain")
    steps = 0
    for _ in range(64):
        active = bos.bos_sample_step()
        steps += 1
        _say(f"  step {steps}: {active} pairs active")
        if active == 0:
            break
    assert active == 0 and steps <= 12
    full, res = _check_history(env, bos, "pearson", range(len(env["pairs"])))
    _say(f"  batches reproduced exactly for {full}/{len(env['pairs'])} pairs")
    assert full >= 0.9 * len(env["pairs"])
    env["plain_hist"] = _histories(bos, len(env["pairs"]))
    bos.close()


def test_bos_pearson_matches_oracle_replay(env):
    pc, ctx, f = env["pc"], env["ctx"], env["f"]
    _say(f"  pearson BOS (graph) over {len(env['pairs'])} pairs: create")
    bos = _bos(env, pc.bos_defaults(seed=3))
    steps = 0
    for _ in range(64):  # at most 1 + 80 / 8 iterations are ever active
        active = bos.bos_sample_step()
        steps += 1
        _say(f"  step {steps}: {active} pairs active")
        if active == 0:
            break
    assert active == 0 and steps <= 12
    full, res = _check_history(env, bos, "pearson", range(len(env["pairs"])))
    _say(f"  batches reproduced exactly for {full}/{len(env['pairs'])} pairs")
    assert full >= 0.9 * len(env["pairs"])
    if "plain_hist" in env:  # the captured graph replays exactly the direct launches
        for (c0, v0), (c1, v1) in zip(env["plain_hist"], _histories(bos, len(env["pairs"]))):
            assert np.array_equal(c0, c1) and np.array_equal(v0, v1)
    # never above the exhaustive maximum
    for p, (ia, ib) in enumerate(env["pairs"]):
        ex = ctx.corr_region_max(f, env["regions"][ia], env["regions"][ib], "pearson", "f32")
        assert res[p]["value"] <= ex["value"] + 1e-5
    bos.close()


def test_bos_ksg_matches_oracle_replay(env):
    pc, ctx, f = env["pc"], env["ctx"], env["f"]
    sub = env["pairs"][:6]
    _say("  ksg BOS over 6 pairs")
    bos = _bos(env, pc.bos_defaults(measure="ksg", k=10, seed=4), pairs=sub)
    bos.bos_run()
    env2 = dict(env, pairs=sub)
    full, _ = _check_history(env2, bos, "ksg", range(len(sub)))
    assert full >= 5
    bos.close()


def test_bos_determinism_save_load(env, tmp_path):
    pc, ctx, f = env["pc"], env["ctx"], env["f"]
    cfg = pc.bos_defaults(seed=9)
    _say("  BOS save / load")
    a = _bos(env, cfg)
    a.bos_run()
    ra = a.bos_results()
    b = _bos(env, cfg)
    b.bos_sample_step()
    b.bos_sample_step()
    path = os.path.join(str(tmp_path), "bos.state")
    b.bos_save(path)
    b.bos_run()
    assert b.bos_results() == ra
    c = _bos(env, cfg, mode="plain")
    c.bos_load(path)
    c.bos_run()
    assert c.bos_results() == ra
    for p in range(len(env["pairs"])):
        ha, hc = a.bos_history(p), c.bos_history(p)
        assert np.array_equal(ha[0], hc[0]) and np.array_equal(ha[1], hc[1])
    for s in (a, b, c):
        s.close()


def test_bos_prior_cell_is_evaluated_first(env):
    pc, ctx, f, e = env["pc"], env["ctx"], env["f"], env["e"]
    pairs = env["pairs"]
    prior = np.zeros((len(pairs), 6), np.float32)
    truth = []
    for p, (ia, ib) in enumerate(pairs):
        ex = ctx.corr_region_max(f, env["regions"][ia], env["regions"][ib], "pearson", "f32")
        ra, rb = e.regions[ia], e.regions[ib]
        ca = ((ex["pa"] % e.nx) - ra.x0, (ex["pa"] // e.nx % e.ny) - ra.y0, (ex["pa"] // (e.nx * e.ny)) - ra.z0)
        cb = ((ex["pb"] % e.nx) - rb.x0, (ex["pb"] // e.nx % e.ny) - rb.y0, (ex["pb"] // (e.nx * e.ny)) - rb.z0)
        prior[p] = ca + cb
        truth.append(ex["value"])
    _say("  BOS with a prior cell")
    bos = _bos(env, pc.bos_defaults(seed=5, n_total=28))
    bos.bos_set_prior(prior)
    bos.bos_run()
    res = bos.bos_results()
    for p in range(len(pairs)):
        cells, _ = bos.bos_history(p)
        assert tuple(cells[0]) == tuple(int(v) for v in prior[p])
        assert abs(res[p]["value"] - truth[p]) <= 2e-5
    bos.close()


def test_bos_error_paths(env):
    pc, ctx, f = env["pc"], env["ctx"], env["f"]
    with pytest.raises(pc.CorrError):
        pc.Bos(ctx, f, env["regions"], [[0, 99]], pc.bos_defaults())
    with pytest.raises(pc.CorrError):
        pc.Bos(ctx, f, env["regions"], env["pairs"], pc.bos_defaults(n_total=101))
    with pytest.raises(pc.CorrError):
        pc.Bos(ctx, f, env["regions"], env["pairs"], pc.bos_defaults(n_uniform=10, n_local=10))
    b = _bos(env, pc.bos_defaults(n_total=28))
    with pytest.raises(pc.CorrError):
        b.bos_set_launch("plain", 0.0)
    b.bos_sample_step()
    with pytest.raises(pc.CorrError):  # the prior must come before sampling
        b.bos_set_prior(np.zeros((len(env["pairs"]), 6), np.float32))
    b.bos_run()
    assert b.bos_sample_step() == 0  # done: further steps do nothing
    b.close()


def test_bos_schedule_matches_oracle(env):
    pc = env["pc"]
    cfg = pc.bos_defaults(seed=7)
    b = _bos(env, cfg)
    sched = b.bos_schedule()
    ocfg = _oracle_cfg(cfg)
    for p in range(len(env["pairs"])):
        assert [int(v) for v in sched[p]] == B.schedule(ocfg, p)
        assert sum(sched[p]) == cfg.n_total - cfg.n_init and all(8 <= v <= 64 and v % 8 == 0 for v in sched[p])
    b.close()
