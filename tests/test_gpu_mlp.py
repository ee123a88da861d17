"""GPU learned-proposal kernels (include/mlp.h) against the FP64 oracle.

Forward, gradients and the AdamW update are compared with oracle/mlp_ref.py
on the same BF16-rounded weights; the region summaries with the oracle's
eigen-decomposition and projections.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import mlp_ref as R

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


def _batch(seed, B, n_in, n_out):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, n_in)).astype(np.float32)
    t = rng.standard_normal((B, n_out)).astype(np.float32)
    return x, t


@pytest.mark.parametrize("shape", [(42, 256, 8, 256), (7, 33, 3, 5), (42, 256, 8, 1)])
def test_forward_and_grad_match_oracle(env, shape):
    torch, pc = env["torch"], env["pc"]
    n_in, H, n_out, B = shape
    _say(f"mlp forward/grad shape={shape}")
    net = pc.PropMlp(env["ctx"], n_in, H, n_out, seed=5)
    p = net.get_params().astype(np.float64)
    x, t = _batch(1, B, n_in, n_out)
    w = np.linspace(0.5, 2.0, n_out).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    y = net.forward(xd).cpu().numpy()
    y_ref, _ = R.forward(p, x, n_in, H, n_out, bf16=True)
    np.testing.assert_allclose(y, y_ref, rtol=1e-4, atol=1e-5)
    loss = net.train_step(xd, td, lr=1e-3, wd=1e-2, loss_w=w)
    L_ref, g_ref = R.loss_and_grad(p, x, t, w, n_in, H, n_out, bf16=True)
    g = net.get_grads().astype(np.float64)
    assert loss == pytest.approx(L_ref, rel=1e-5)
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    _say(f"  grad rel Frobenius error {rel:.2e}")
    assert rel < 1e-4
    # AdamW step (t = 1) from the GPU's own gradient
    p_ref, _, _ = R.adamw(p, g, np.zeros_like(p), np.zeros_like(p), 1, 1e-3, 1e-2)
    np.testing.assert_allclose(net.get_params(), p_ref, rtol=1e-5, atol=1e-7)
    net.close()


def test_training_is_deterministic_and_learns(env):
    torch, pc = env["torch"], env["pc"]
    rng = np.random.default_rng(2)
    n_in, n_out, B = 42, 8, 256
    A = rng.standard_normal((n_in, n_out)) / np.sqrt(n_in)
    x = rng.standard_normal((B, n_in)).astype(np.float32)
    t = np.tanh(x @ A).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    runs = []
    for _ in range(2):
        net = pc.PropMlp(env["ctx"], n_in, 256, n_out, seed=3)
        losses = [net.train_step(xd, td, lr=2e-3, wd=1e-4) for _ in range(200)]
        runs.append((losses, net.get_params()))
        net.close()
    _say(f"  loss {runs[0][0][0]:.4f} -> {runs[0][0][-1]:.5f}")
    assert runs[0][0] == runs[1][0]
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    assert runs[0][0][-1] < 0.05 * runs[0][0][0]


def test_multi_step_adamw_matches_oracle(env):
    torch, pc = env["torch"], env["pc"]
    n_in, H, n_out, B = 10, 24, 4, 16
    net = pc.PropMlp(env["ctx"], n_in, H, n_out, seed=9)
    p = net.get_params().astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    for it in range(5):
        x, t = _batch(100 + it, B, n_in, n_out)
        net.train_step(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), lr=1e-2, wd=1e-3)
        _, g_ref = R.loss_and_grad(p, x, t, None, n_in, H, n_out, bf16=True)
        g = net.get_grads().astype(np.float64)
        assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) < 1e-4
        p, m, v = R.adamw(p, g, m, v, it + 1, 1e-2, 1e-3)
        # continue the oracle from the GPU's parameters so rounding does not accumulate
        q = net.get_params().astype(np.float64)
        np.testing.assert_allclose(q, p, rtol=1e-5, atol=1e-6)
        p = q
    net.close()


def test_bad_arguments(env):
    pc = env["pc"]
    with pytest.raises(pc.CorrError):
        pc.PropMlp(env["ctx"], 42, 2048, 8)
    with pytest.raises(pc.CorrError):
        pc.PropMlp(env["ctx"], 42, 256, 65)


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_region_features_match_oracle(env, dtype):
    torch, pc = env["torch"], env["pc"]
    e = synth.make_context(3, 2, (12, 12, 6), M=100, seed=31, n_groups=3, blob_r=2.0, min_region_gap=2)
    _say(f"region features dtype={dtype} grid={e.nx}x{e.ny}x{e.nz}")
    data = e.data if dtype == "f32" else e.data.astype(np.float16)
    f = pc.Field(torch.from_numpy(np.ascontiguousarray(data)).cuda(), e.nx, e.ny, e.nz)
    regs = [pc.region(*r.as_tuple()) for r in e.regions]
    feats, ev = pc.corr_region_features(env["ctx"], f, regs, n_pc=16)
    ref, ev_ref = R.region_features(data.astype(np.float64), e.regions, e.nx, e.ny, e.nz, n_pc=16)
    np.testing.assert_allclose(ev, ev_ref, rtol=1e-4, atol=1e-6)
    got = feats.cpu().numpy()
    # the planted groups give well separated leading components; the rest
    # may rotate within near-degenerate eigenspaces, so compare the top three
    gap = np.abs(np.diff(ev_ref[:4]))
    assert np.all(gap > 1e-2 * ev_ref[0])
    np.testing.assert_allclose(got[:, :3], ref[:, :3], atol=2e-4)
    np.testing.assert_allclose(got[:, 16:], ref[:, 16:], rtol=1e-5, atol=1e-5)
