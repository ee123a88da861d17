"""Oracle for batched Bayesian optimal sampling of region-pair maxima
(Sec. 3.1) -- TEST INFRASTRUCTURE ONLY, FP64 NumPy, one pair at a time.

What it computes, step by step (the same algorithm the GPU library runs):

* domain: theta in [0, d_a - 1] for the 6 axes (x, y, z of a cell in region
  A, then x, y, z of a cell in region B), in cell units (Sec. 3.1: a sample
  position is a point of a 6-D space);
* initial design: n_init cells, coordinate floor(u * d_a);
* batch schedule: 80 acquired samples split into batches of 8 * p,
  p = 1 + floor(u * min(8, units left)) (uneven per-pair batches of 8..64);
* Gaussian-process surrogate with a Matern-5/2 covariance (Sec. 3.1),
  length scale l on every axis, unit signal variance, jitter on the
  diagonal, observations standardised per pair (std floored at 1e-6);
* acquisition: upper confidence bound mu + kappa * sigma, kappa = 0.5,
  maximised over a seeded candidate set (n_uniform uniform points plus
  n_local Gaussian perturbations, sd = local_sd cells, of the best cell so
  far, clipped to the box) -- this replaces the paper's randomized DIRECT-L
  optimiser;
* a batch of b picks by Kriging believer: each pick joins the GP with its
  own posterior mean as value, which leaves every mean unchanged and only
  shrinks the variances; a candidate is picked at most once per batch;
  ties go to the lowest candidate index;
* probabilistic reparameterisation (Sec. 3.1): P = floor(theta) + Ber(theta -
  floor(theta)), clamped to the box;
* a rounded cell already observed (or picked earlier in the batch) is not
  evaluated again and still uses its slot;
* objective |r| (Pearson) or MI (KSG) of the two cells; the pair's running
  maximum keeps the earliest of equal values.

Random numbers: Philox4x64-10 (Salmon et al. 2011), counter = (pair,
stream, index, axis), key = (seed, 0x636f7272); u = (w >> 11) * 2^-53;
normals by Box-Muller from words 0 and 1. Streams: 0 initial design,
1 schedule, 2 uniform candidates, 3 local candidates, 4 rounding.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

MASK64 = (1 << 64) - 1
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
KEY_HI = 0x636F7272

S_INIT, S_SCHED, S_UNIF, S_LOCAL, S_ROUND = 0, 1, 2, 3, 4


def philox4x64(ctr, key, rounds=10):
    """Philox4x64 block function on Python ints: ctr = 4 words, key = 2 words."""
    c = [int(v) & MASK64 for v in ctr]
    k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
    for r in range(rounds):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * c[0]
        p1 = PHILOX_M1 * c[2]
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def _mulhilo(a, b):
    """64 x 64 -> (hi, lo) on numpy uint64 arrays."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a0, a1 = a & m32, a >> s32
    b0, b1 = b & m32, b >> s32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> s32) + (p01 & m32) + (p10 & m32)
    hi = p11 + (p01 >> s32) + (p10 >> s32) + (mid >> s32)
    return hi, a * b


def philox4x64_np(c0, c1, c2, c3, k0, k1, rounds=10):
    """Philox4x64 on numpy uint64 arrays (same function as philox4x64)."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0, k1 = np.uint64(int(k0) & MASK64), np.uint64(int(k1) & MASK64)
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r:
                k0 = np.uint64((int(k0) + PHILOX_W0) & MASK64)
                k1 = np.uint64((int(k1) + PHILOX_W1) & MASK64)
            hi0, lo0 = _mulhilo(np.uint64(PHILOX_M0), c0)
            hi1, lo1 = _mulhilo(np.uint64(PHILOX_M1), c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def u01_np(w):
    return (w >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def u01(w):
    return (int(w) >> 11) * (1.0 / 9007199254740992.0)


def draw(seed, pair, stream, index, axis):
    return philox4x64((pair, stream, index, axis), (seed, KEY_HI))


def gauss(seed, pair, stream, index, axis):
    w = draw(seed, pair, stream, index, axis)
    u1, u2 = u01(w[0]), u01(w[1])
    return math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)


@dataclasses.dataclass
class BosConfig:
    n_init: int = 20
    n_total: int = 100
    n_uniform: int = 384
    n_local: int = 128
    kappa: float = 0.5
    lengthscale: float = 3.0
    local_sd: float = 1.0
    jitter: float = 1e-6
    seed: int = 1


def schedule(cfg: BosConfig, pair: int):
    units = (cfg.n_total - cfg.n_init) // 8
    out, i = [], 0
    while units > 0:
        m = min(8, units)
        p = 1 + int(u01(draw(cfg.seed, pair, S_SCHED, i, 0)[0]) * m)
        out.append(8 * p)
        units -= p
        i += 1
    return out


def initial_cells(cfg: BosConfig, pair: int, dims):
    cells = np.zeros((cfg.n_init, 6), np.int64)
    for s in range(cfg.n_init):
        for a in range(6):
            c = int(u01(draw(cfg.seed, pair, S_INIT, s, a)[0]) * dims[a])
            cells[s, a] = min(c, dims[a] - 1)
    return cells


def matern52(X1, X2, ls):
    d = (X1[:, None, :] - X2[None, :, :]) / ls
    rho = np.sqrt((d * d).sum(-1))
    s5 = math.sqrt(5.0) * rho
    return (1.0 + s5 + 5.0 * rho * rho / 3.0) * np.exp(-s5)


def standardize_y(y):
    m = y.mean()
    s = max(y.std(), 1e-6)
    return (y - m) / s


def gp_posterior(X, yt, Xc, ls, jitter):
    """Posterior mean and variance at Xc given standardised observations (Cholesky solve)."""
    K = matern52(X, X, ls) + jitter * np.eye(X.shape[0])
    L = np.linalg.cholesky(K)
    alpha = np.linalg.solve(L.T, np.linalg.solve(L, yt))
    Kc = matern52(Xc, X, ls)
    mu = Kc @ alpha
    W = np.linalg.solve(L, Kc.T)
    var = np.maximum(0.0, 1.0 - (W * W).sum(0))
    return mu, var


def candidates(cfg: BosConfig, pair: int, it: int, dims, best_cell):
    up = np.array(dims, np.float64) - 1.0
    C = cfg.n_uniform + cfg.n_local
    th = np.zeros((C, 6))
    key = (cfg.seed, KEY_HI)
    ax = np.arange(6, dtype=np.uint64)[None, :]
    if cfg.n_uniform:
        idx = (it * cfg.n_uniform + np.arange(cfg.n_uniform, dtype=np.uint64))[:, None]
        w = philox4x64_np(np.uint64(pair), np.uint64(S_UNIF), idx, ax, *key)
        th[: cfg.n_uniform] = u01_np(w[0]) * up[None, :]
    if cfg.n_local:
        idx = (it * cfg.n_local + np.arange(cfg.n_local, dtype=np.uint64))[:, None]
        w = philox4x64_np(np.uint64(pair), np.uint64(S_LOCAL), idx, ax, *key)
        u1, u2 = u01_np(w[0]), u01_np(w[1])
        z = np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * math.pi * u2)
        th[cfg.n_uniform:] = np.clip(np.asarray(best_cell, np.float64)[None, :] + cfg.local_sd * z, 0.0, up[None, :])
    return th


def believer_picks(cfg: BosConfig, X, yt, th, b):
    """Kriging-believer batch: indices of the b picked candidates, in pick order."""
    mu, var = gp_posterior(X, yt, th, cfg.lengthscale, cfg.jitter)
    Xe = X.copy()
    picked = []
    taken = np.zeros(th.shape[0], bool)
    for _ in range(b):
        ucb = mu + cfg.kappa * np.sqrt(var)
        ucb[taken] = -np.inf
        c = int(np.argmax(ucb))  # first index among ties
        picked.append(c)
        taken[c] = True
        Xe = np.vstack([Xe, th[c:c + 1]])
        # variances under the extended training set (means are unchanged)
        K = matern52(Xe, Xe, cfg.lengthscale) + cfg.jitter * np.eye(Xe.shape[0])
        L = np.linalg.cholesky(K)
        W = np.linalg.solve(L, matern52(th, Xe, cfg.lengthscale).T)
        var = np.maximum(0.0, 1.0 - (W * W).sum(0))
    return picked, mu


def round_cell(cfg: BosConfig, pair: int, slot: int, theta, dims):
    cell = np.zeros(6, np.int64)
    for a in range(6):
        f = math.floor(theta[a])
        u = u01(draw(cfg.seed, pair, S_ROUND, slot, a)[0])
        v = f + (1 if u < theta[a] - f else 0)
        cell[a] = min(max(v, 0), dims[a] - 1)
    return cell


def iteration_cells(cfg: BosConfig, pair: int, it: int, dims, X, y, slot):
    """Cells newly evaluated by batch `it` of `pair`, given its observations so far.

    X (n, 6) int cells and y (n,) values are the pair's observations in
    evaluation order; slot = n_init + samples of the earlier batches.
    """
    b = schedule(cfg, pair)[it]
    yt = standardize_y(np.asarray(y, np.float64))
    best = int(np.argmax(y))
    th = candidates(cfg, pair, it, dims, X[best])
    picks, _ = believer_picks(cfg, np.asarray(X, np.float64), yt, th, b)
    seen = {tuple(int(v) for v in c) for c in X}
    new = []
    for m, c in enumerate(picks):
        cell = round_cell(cfg, pair, slot + m, th[c], dims)
        t = tuple(int(v) for v in cell)
        if t not in seen:
            seen.add(t)
            new.append(cell)
    return np.array(new, np.int64).reshape(-1, 6), b


def initial_unique_cells(cfg: BosConfig, pair: int, dims, prior_cell=None):
    init = initial_cells(cfg, pair, dims)
    if prior_cell is not None and prior_cell[0] >= 0:
        init[0] = [min(max(int(np.rint(v)), 0), dims[a] - 1) for a, v in enumerate(prior_cell)]
    X, seen = [], set()
    for c in init:
        t = tuple(int(v) for v in c)
        if t not in seen:
            seen.add(t)
            X.append(c)
    return np.array(X, np.int64)


def run_pair(cfg: BosConfig, pair: int, dims, objective, max_iters=None, prior_cell=None):
    """Full BOS of one region pair. objective(cells (n, 6)) -> values (n,).

    Returns dict(value, cell, n_evaluated, cells, values, iters) where cells /
    values are the evaluated (unique) observations in order.
    """
    X = initial_unique_cells(cfg, pair, dims, prior_cell)
    y = np.asarray(objective(X), np.float64)
    sched = schedule(cfg, pair)
    slot = cfg.n_init
    n_it = len(sched) if max_iters is None else min(max_iters, len(sched))
    for it in range(n_it):
        new, b = iteration_cells(cfg, pair, it, dims, X, y, slot)
        slot += b
        if new.shape[0]:
            X = np.vstack([X, new])
            y = np.concatenate([y, np.asarray(objective(new), np.float64)])
    best = int(np.argmax(y))
    return dict(value=float(y[best]), cell=X[best].copy(), n_evaluated=int(X.shape[0]), cells=X, values=y,
                iters=n_it)


def cells_to_points(cells, ra, rb, nx, ny):
    """Global point indices of the A and B cells of 6-D cells (local coordinates)."""
    pa = (ra.x0 + cells[:, 0]) + nx * ((ra.y0 + cells[:, 1]) + ny * (ra.z0 + cells[:, 2]))
    pb = (rb.x0 + cells[:, 3]) + nx * ((rb.y0 + cells[:, 4]) + ny * (rb.z0 + cells[:, 5]))
    return pa.astype(np.int64), pb.astype(np.int64)
