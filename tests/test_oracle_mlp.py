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


def _brute_self_similarity(data, nx, ny, nz, D):
    P = nx * ny * nz
    out = np.zeros(P)
    for p in range(P):
        x, y, z = p % nx, (p // nx) % ny, p // (nx * ny)
        vals = []
        for dx, dy, dz in ((D, 0, 0), (-D, 0, 0), (0, D, 0), (0, -D, 0), (0, 0, D), (0, 0, -D)):
            X, Y, Z = x + dx, y + dy, z + dz
            if 0 <= X < nx and 0 <= Y < ny and 0 <= Z < nz:
                q = X + nx * (Y + ny * Z)
                a, b = data[:, p], data[:, q]
                if a.std() > 0 and b.std() > 0:
                    vals.append(np.corrcoef(a, b)[0, 1])
                else:
                    vals.append(0.0)
        out[p] = np.mean(vals) if vals else 0.0
    return out


def test_self_similarity_brute_force():
    rng = np.random.default_rng(21)
    nx, ny, nz, M = 7, 5, 3, 9
    data = rng.standard_normal((M, nx * ny * nz))
    data[:, 4] = 2.5  # a constant point
    _, _, z = R.standardize(data)
    for D in (1, 2, 4):
        np.testing.assert_allclose(R.self_similarity(z, nx, ny, nz, D), _brute_self_similarity(data, nx, ny, nz, D),
                                   atol=1e-12)


def test_self_similarity_rank_one_is_one():
    rng = np.random.default_rng(2)
    nx, ny, nz, M = 9, 6, 5, 20
    v = rng.standard_normal(M)
    data = v[:, None] * rng.uniform(0.5, 3.0, nx * ny * nz) + rng.standard_normal(nx * ny * nz)
    _, _, z = R.standardize(data)
    np.testing.assert_allclose(R.self_similarity(z, nx, ny, nz, 2), 1.0, atol=1e-12)


def test_hot_spots_find_planted_blob_and_suppress():
    e = synth.make_context(2, 1, (16, 16, 10), M=100, seed=5, n_groups=1, blob_r=3.0, min_region_gap=1)
    g = e.groups[0]
    _, _, z = R.standardize(e.data)
    sim = R.self_similarity(z, e.nx, e.ny, e.nz, 4)
    for ri, (cx, cy, cz, rad) in zip(g["regions"], g["blobs"]):
        r = e.regions[ri]
        h = R.hot_spots(sim, r, e.nx, e.ny, n_hot=4, r_nms=3)
        x, y, zc = h[0] % e.nx, (h[0] // e.nx) % e.ny, h[0] // (e.nx * e.ny)
        assert (x - cx) ** 2 + (y - cy) ** 2 + (zc - cz) ** 2 <= (rad + 1) ** 2
        co = [(p % e.nx, (p // e.nx) % e.ny, p // (e.nx * e.ny)) for p in h]
        for i in range(4):
            for j in range(i):
                assert max(abs(co[i][k] - co[j][k]) for k in range(3)) > 3
    # a region too small for more than one pick repeats it
    tiny = synth.Region(0, 0, 0, 2, 2, 2)
    h = R.hot_spots(sim, tiny, e.nx, e.ny, n_hot=3, r_nms=3)
    assert h[0] == h[1] == h[2]


def test_proposal_inputs_cross_terms_are_pearson():
    e = synth.make_context(3, 1, (10, 10, 6), M=50, seed=8, n_groups=1, blob_r=2.0, min_region_gap=1)
    pairs = synth.region_pair_list(len(e.regions))
    X, hots = R.proposal_inputs(e.data, e.nx, e.ny, e.nz, e.regions, pairs, n_hot=3, D=3, r_nms=2)
    F = 4 * 3 + 5
    assert X.shape == (len(pairs), 2 * F + 9)
    x = e.data.astype(np.float64)
    for row, (a, b) in zip(X, pairs):
        c = [abs(np.corrcoef(x[:, hots[a][i]], x[:, hots[b][j]])[0, 1]) for i in range(3) for j in range(3)]
        np.testing.assert_allclose(row[2 * F:], c, atol=1e-12)
        ia = e.regions[a].global_indices(e.nx, e.ny)
        assert row[F - 5] == pytest.approx(x[:, ia].mean(), abs=1e-12)
        assert row[F - 4] == pytest.approx(x[:, ia].std(0).mean(), abs=1e-12)
        assert row[F - 3] == pytest.approx((e.regions[a].x0 + 4.5) / e.nx)
    # pick strengths are the similarity map at the picks; positions are local
    _, _, z = R.standardize(e.data)
    sim = R.self_similarity(z, e.nx, e.ny, e.nz, 3)
    r0 = e.regions[pairs[0][0]]
    for i in range(3):
        p = hots[pairs[0][0]][i]
        assert X[0, 4 * i] == pytest.approx(sim[p], abs=1e-15)
        assert X[0, 4 * i + 1] == pytest.approx((p % e.nx - r0.x0) / (r0.dx - 1))
