"""Pins for the BOS oracle (Sec. 3.1): library routines and closed forms,
not the oracle's formulas retyped."""
import math

import numpy as np
import pytest

from oracle import bos_ref as B


def test_philox_matches_numpy():
    # numpy's Philox bit generator is Philox4x64-10; its first block uses
    # counter + 1 (it increments before generating)
    for key, ctr in [((7, 0x636F7272), (0, 0, 0, 0)), ((123456789, 42), (5, 1, 99, 3)),
                     ((2**63 + 11, 2**64 - 1), (2**64 - 2, 2**64 - 1, 17, 2**40))]:
        bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
        got = [int(v) for v in bg.random_raw(4)]
        c = list(ctr)
        c[0] = (c[0] + 1) & B.MASK64
        if c[0] == 0:
            c[1] = (c[1] + 1) & B.MASK64
        assert B.philox4x64(c, key) == got


def test_vectorised_philox_matches_scalar():
    rng = np.random.default_rng(3)
    c = rng.integers(0, 2**63, (50, 4), dtype=np.int64).astype(np.uint64) * np.uint64(2) + np.uint64(1)
    w = B.philox4x64_np(c[:, 0], c[:, 1], c[:, 2], c[:, 3], 2**64 - 5, 77)
    for i in range(50):
        assert [int(w[q][i]) for q in range(4)] == B.philox4x64([int(v) for v in c[i]], (2**64 - 5, 77))


def test_matern_matches_sklearn():
    from sklearn.gaussian_process.kernels import Matern
    rng = np.random.default_rng(0)
    X1, X2 = rng.uniform(0, 20, (7, 6)), rng.uniform(0, 20, (5, 6))
    ref = Matern(length_scale=3.0, nu=2.5)(X1, X2)
    assert np.allclose(B.matern52(X1, X2, 3.0), ref, rtol=1e-12, atol=1e-14)


def test_gp_posterior_matches_sklearn():
    from sklearn.gaussian_process import GaussianProcessRegressor
    from sklearn.gaussian_process.kernels import Matern
    rng = np.random.default_rng(1)
    X = rng.integers(0, 16, (40, 6)).astype(float)
    X = np.unique(X, axis=0)
    y = np.sin(X.sum(1) / 7.0) + 0.1 * rng.standard_normal(X.shape[0])
    yt = B.standardize_y(y)
    Xc = rng.uniform(0, 15, (200, 6))
    mu, var = B.gp_posterior(X, yt, Xc, 3.0, 1e-6)
    gp = GaussianProcessRegressor(kernel=Matern(length_scale=3.0, nu=2.5), alpha=1e-6, optimizer=None,
                                  normalize_y=False).fit(X, yt)
    m2, s2 = gp.predict(Xc, return_std=True)
    assert np.allclose(mu, m2, rtol=0, atol=1e-8)
    assert np.allclose(np.sqrt(var), s2, rtol=0, atol=1e-6)


def test_believer_keeps_means_and_matches_refit():
    from sklearn.gaussian_process import GaussianProcessRegressor
    from sklearn.gaussian_process.kernels import Matern
    rng = np.random.default_rng(2)
    X = np.unique(rng.integers(0, 12, (25, 6)).astype(float), axis=0)
    yt = B.standardize_y(rng.standard_normal(X.shape[0]))
    th = rng.uniform(0, 11, (64, 6))
    cfg = B.BosConfig()
    picks, mu0 = B.believer_picks(cfg, X, yt, th, 3)
    assert len(set(picks)) == 3
    # refit with the believer values: means at all candidates unchanged
    Xe = np.vstack([X, th[picks]])
    ye = np.concatenate([yt, mu0[picks]])
    gp = GaussianProcessRegressor(kernel=Matern(length_scale=3.0, nu=2.5), alpha=1e-6, optimizer=None).fit(Xe, ye)
    assert np.allclose(gp.predict(th), mu0, atol=1e-6)
    # the first pick is the plain UCB argmax
    mu, var = B.gp_posterior(X, yt, th, 3.0, 1e-6)
    assert picks[0] == int(np.argmax(mu + 0.5 * np.sqrt(var)))


def test_schedule_is_a_composition_of_80():
    for pair in range(200):
        s = B.schedule(B.BosConfig(seed=5), pair)
        assert sum(s) == 80 and all(8 <= b <= 64 and b % 8 == 0 for b in s)
    lens = {len(B.schedule(B.BosConfig(seed=5), p)) for p in range(200)}
    assert len(lens) > 3  # uneven across pairs


def test_rounding_is_bernoulli_of_the_fraction():
    cfg = B.BosConfig(seed=9)
    dims = (32, 32, 20, 32, 32, 20)
    th = np.array([3.0, 7.25, 0.5, 30.9, 12.0, 18.75])
    ups = np.zeros(6)
    n = 4000
    for s in range(n):
        c = B.round_cell(cfg, 0, s, th, dims)
        ups += (c > np.floor(th))
    frac = th - np.floor(th)
    assert np.all(np.abs(ups / n - frac) < 4 * np.sqrt(frac * (1 - frac) / n) + 1e-12)
    assert (B.round_cell(cfg, 0, 0, np.array([31.0, 31, 19, 0, 0, 0]), dims) == [31, 31, 19, 0, 0, 0]).all()


def test_bos_finds_analytic_maximum_of_6d_normal():
    # a 6-variate normal PDF in place of a correlation (its grid maximum is
    # found by brute force): mean normalised error of BOS at 100 samples,
    # against 100 uniform random samples of the same objective
    rng = np.random.default_rng(4)
    dims = (8, 8, 8, 8, 8, 8)
    grid = np.stack(np.meshgrid(*[np.arange(8)] * 6, indexing="ij"), -1).reshape(-1, 6).astype(float)
    errs, rnd = [], []
    for t in range(6):
        mean = rng.uniform(1, 6, 6)
        A = rng.standard_normal((6, 6))
        cov = A @ A.T / 6 + 6.0 * np.eye(6)
        P = np.linalg.inv(cov)

        def f(c):
            d = np.asarray(c, float) - mean
            return np.exp(-0.5 * np.einsum("ni,ij,nj->n", d, P, d))

        true_max = f(grid).max()
        res = B.run_pair(B.BosConfig(seed=100 + t), t, dims, f)
        assert res["n_evaluated"] <= 100
        errs.append((true_max - res["value"]) / true_max)
        rnd.append((true_max - f(rng.integers(0, 8, (100, 6))).max()) / true_max)
    assert np.mean(errs) <= 0.05, errs
    assert np.mean(errs) <= np.mean(rnd) / 4, (errs, rnd)


def replay_iterations(cfg, pair, dims, cells, vals):
    """Replay a pair's recorded history batch by batch with the oracle.

    Returns (matched, total): how many batches the oracle reproduces exactly
    from the history that precedes them (stops at the first mismatch)."""
    X0 = B.initial_unique_cells(cfg, pair, dims)
    if not np.array_equal(X0, cells[: X0.shape[0]]):
        return 0, len(B.schedule(cfg, pair)) + 1
    n, slot = X0.shape[0], cfg.n_init
    sched = B.schedule(cfg, pair)
    matched = 1
    for it in range(len(sched)):
        new, b = B.iteration_cells(cfg, pair, it, dims, cells[:n], np.asarray(vals[:n], np.float64), slot)
        k = new.shape[0]
        if not np.array_equal(new, cells[n:n + k]):
            return matched, len(sched) + 1
        matched += 1
        n += k
        slot += b
    assert n == cells.shape[0]
    return matched, len(sched) + 1


def test_replay_reproduces_an_oracle_run():
    rng = np.random.default_rng(8)
    dims = (6, 5, 4, 6, 5, 4)
    w = rng.standard_normal(6)

    def f(c):
        return np.cos(np.asarray(c, float) @ w / 3.0)

    cfg = B.BosConfig(seed=17)
    for pair in range(3):
        res = B.run_pair(cfg, pair, dims, f)
        m, t = replay_iterations(cfg, pair, dims, res["cells"], res["values"])
        assert m == t


def _numpy_word0(seed, pair, stream, index, axis):
    """Word 0 of the Philox4x64-10 block at counter (pair, stream, index, axis)
    under key (seed, 0x636f7272), from numpy's generator (it adds one to the
    counter before its first block, so it starts one below)."""
    ctr = (pair | (stream << 64) | (index << 128) | (axis << 192)) - 1  # 256-bit counter, word 0 lowest
    if ctr < 0:
        ctr += 1 << 256
    words = [(ctr >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    bg = np.random.Philox(key=np.array([seed, B.KEY_HI], np.uint64), counter=np.array(words, np.uint64))
    return int(bg.random_raw(1)[0])


def test_initial_design_is_floor_of_u_times_d_from_numpy_philox():
    # Sec. 3.1 initial design: every coordinate floor(u * d) with u the top
    # 53 bits of Philox word 0 (numpy's generator as the reference stream)
    cfg = B.BosConfig(seed=31)
    dims = (32, 32, 20, 7, 1, 13)
    for pair in (0, 1, 17, 3827):
        got = B.initial_cells(cfg, pair, dims)
        for s in range(cfg.n_init):
            for a in range(6):
                u = (_numpy_word0(cfg.seed, pair, B.S_INIT, s, a) >> 11) / 2.0 ** 53
                assert got[s, a] == min(int(np.floor(u * dims[a])), dims[a] - 1)
    assert (B.initial_cells(cfg, 5, dims)[:, 4] == 0).all()  # a one-cell axis


def test_uniform_candidates_are_uniform_on_zero_to_d_minus_one():
    from scipy import stats
    cfg = B.BosConfig(seed=12, n_uniform=1024, n_local=0)
    dims = (32, 9, 20, 32, 2, 20)
    th = np.vstack([B.candidates(cfg, 4, it, dims, np.zeros(6)) for it in range(4)])
    for a in range(6):
        up = dims[a] - 1
        assert th[:, a].min() >= 0.0 and th[:, a].max() <= up
        # Kolmogorov-Smirnov against U(0, d - 1): scaling by d instead of
        # d - 1 moves the CDF by up to 1/d and fails at these sample sizes
        p = stats.kstest(th[:, a], stats.uniform(loc=0.0, scale=up).cdf).pvalue
        assert p > 1e-3, (a, p)
    # the exact draw: word 0 of stream 2 at index it * n_uniform + c
    u = (_numpy_word0(cfg.seed, 4, B.S_UNIF, 2 * 1024 + 5, 3) >> 11) / 2.0 ** 53
    assert th[2 * 1024 + 5, 3] == u * (dims[3] - 1)


def test_local_candidates_are_normal_around_the_incumbent_before_clipping():
    from scipy import stats
    sd = 1.7
    cfg = B.BosConfig(seed=14, n_uniform=0, n_local=1024, local_sd=sd)
    dims = (200, 200, 200, 200, 200, 200)
    best = np.array([100.0, 50.0, 150.0, 99.0, 120.0, 60.0])  # far from the faces: no clipping
    th = np.vstack([B.candidates(cfg, 9, it, dims, best) for it in range(3)])
    for a in range(6):
        p = stats.kstest(th[:, a], stats.norm(loc=best[a], scale=sd).cdf).pvalue
        assert p > 1e-3, (a, p)
    # clipping to the box at a face
    th = B.candidates(B.BosConfig(seed=14, n_uniform=0, n_local=256, local_sd=sd), 9, 0, (8,) * 6, np.zeros(6))
    assert th.min() == 0.0 and (th == 0.0).mean() > 0.3 and th.max() <= 7.0


def test_duplicate_cells_are_dropped_but_use_their_slots():
    # a 2-cell domain: after the initial design every rounded pick is a
    # repeat; none is evaluated again, and every batch still advances the
    # rounding stream by its full size
    cfg = B.BosConfig(seed=23)
    dims = (1, 1, 1, 1, 1, 2)
    calls = []

    def f(c):
        calls.append(np.asarray(c).copy())
        return np.asarray(c, float)[:, 5] + 0.5

    res = B.run_pair(cfg, 0, dims, f)
    assert res["n_evaluated"] == 2 and sum(len(c) for c in calls) == 2
    assert {tuple(c) for c in res["cells"]} == {(0, 0, 0, 0, 0, 0), (0, 0, 0, 0, 0, 1)}
    # rounding of batch 1 draws from slot n_init + b_0
    sched = B.schedule(cfg, 0)
    X = res["cells"]
    slot = cfg.n_init + sched[0]
    theta = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.4])
    cell = B.round_cell(cfg, 0, slot, theta, dims)
    u = (_numpy_word0(cfg.seed, 0, B.S_ROUND, slot, 5) >> 11) / 2.0 ** 53
    assert cell[5] == (1 if u < 0.4 else 0)
    new, b = B.iteration_cells(cfg, 0, 1, dims, X, res["values"], slot)
    assert b == sched[1] and new.shape[0] == 0
