"""Pins of the learned-proposal oracle (oracle/mlp_ref.py) against facts
that do not come from the oracle itself: central finite differences of its
loss, torch.optim.AdamW, torch's BF16 conversion, an SVD of the member
matrix, and closed-form cases of the region summaries.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp_ref as R


def _params(rng, n_in, H, n_out, scale=0.5):
    n = n_in * H + H + H * H + H + H * n_out + n_out
    return rng.standard_normal(n) * scale


def test_grad_matches_central_differences():
    rng = np.random.default_rng(7)
    n_in, H, n_out, B = 5, 7, 3, 4
    p = _params(rng, n_in, H, n_out)
    x = rng.standard_normal((B, n_in))
    t = rng.standard_normal((B, n_out))
    w = np.array([1.0, 0.5, 2.0])
    _, g = R.loss_and_grad(p, x, t, w, n_in, H, n_out, bf16=False)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = R.loss_and_grad(p + e, x, t, w, n_in, H, n_out, bf16=False)
        lm, _ = R.loss_and_grad(p - e, x, t, w, n_in, H, n_out, bf16=False)
        fd[i] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_loss_is_weighted_mse():
    # y is affine in the last layer: with W3 = 0 the output is b3 for every row
    n_in, H, n_out, B = 3, 4, 2, 5
    p = np.zeros(n_in * H + H + H * H + H + H * n_out + n_out)
    p[-2:] = [1.0, -2.0]
    x = np.ones((B, n_in))
    t = np.zeros((B, n_out))
    L, _ = R.loss_and_grad(p, x, t, [3.0, 1.0], n_in, H, n_out, bf16=False)
    assert L == pytest.approx((3.0 * 1.0 + 1.0 * 4.0) * B / (B * n_out))


def test_adamw_matches_torch():
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) * 10.0 ** rng.uniform(-4, 1) for _ in range(6)]
    lr, wd = 1e-2, 0.1
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([tp], lr=lr, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, 1):
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = R.adamw(p, g, m, v, t, lr, wd)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.standard_normal(10000).astype(np.float32),
                        # exact halfway cases between BF16 neighbours
                        (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
                        np.array([0.0, -0.0, 1.0, -3.5, 65504.0], np.float32)])
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(R.bf16_round(a), ref)


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    np.testing.assert_allclose(R.dsilu(z), (R.silu(z + h) - R.silu(z - h)) / (2 * h), rtol=1e-7, atol=1e-10)


def test_region_features_eigenvalues_match_svd():
    e = synth.make_context(2, 2, (8, 8, 4), M=40, seed=9, n_groups=2, blob_r=2.0, min_region_gap=1)
    regions = e.regions
    f, ev = R.region_features(e.data, regions, e.nx, e.ny, e.nz, n_pc=6)
    x = e.data.astype(np.float64)
    d = x - x.mean(0)
    z = d / np.sqrt((d * d).sum(0))
    s = np.linalg.svd(z, compute_uv=False)
    np.testing.assert_allclose(ev, (s ** 2 / x.shape[1])[:6], rtol=1e-10)
    # unit-norm columns: the eigenvalues of G sum to one
    _, ev_all = R.region_features(e.data, regions[:1], e.nx, e.ny, e.nz, n_pc=40)
    assert ev_all.sum() == pytest.approx(1.0, abs=1e-12)
    assert f.shape == (len(regions), 11)
    assert np.all(f[:, :6] >= 0) and np.all(f[:, :6] <= 1 + 1e-12)


def test_region_features_rank_one_field():
    # every point is an affine image of one member vector: G has rank one,
    # its eigenvector is that vector, and every |projection| is one
    rng = np.random.default_rng(11)
    M, nx, ny, nz = 12, 4, 3, 2
    v = rng.standard_normal(M)
    a = rng.uniform(0.5, 2.0, nx * ny * nz) * rng.choice([-1, 1], nx * ny * nz)
    b = rng.standard_normal(nx * ny * nz)
    data = v[:, None] * a[None, :] + b[None, :]
    regs = [synth.Region(0, 0, 0, 2, 3, 2), synth.Region(2, 0, 0, 2, 2, 1)]
    f, ev = R.region_features(data, regs, nx, ny, nz, n_pc=2)
    assert ev[0] == pytest.approx(1.0, abs=1e-12) and abs(ev[1]) < 1e-12
    np.testing.assert_allclose(f[:, 0], 1.0, atol=1e-12)
    # per-point mean of v*a+b is mean(v)*a+b; sigma is |a| * std(v)
    g0 = regs[0].global_indices(nx, ny)
    assert f[0, 2] == pytest.approx(np.mean(v.mean() * a[g0] + b[g0]), abs=1e-12)
    assert f[0, 3] == pytest.approx(np.mean(np.abs(a[g0]) * v.std()), abs=1e-12)
    # centre of x in [0, 2) on nx = 4 is 0.5 / 4
    assert f[0, 4] == pytest.approx(0.5 / 4) and f[1, 4] == pytest.approx(2.5 / 4)
    assert f[0, 5] == pytest.approx(1.0 / 3) and f[1, 6] == pytest.approx(0.0)
