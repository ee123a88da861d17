"""Oracle for the learned BOS proposal -- TEST INFRASTRUCTURE ONLY (NumPy FP64).

The network (a proposal prior for Sec. 3.1's sampling; the paper names a
network that predicts correlation values as future work, Sec. 7):
  x (n_in) -> z1 = x W1 + b1 -> a1 = silu(z1) -> z2 = a1 W2 + b2 ->
  a2 = silu(z2) -> y = a2 W3 + b3 (n_out), silu(z) = z / (1 + exp(-z)).
Loss: weighted mean squared error
  L = sum_{b,o} w_o (y_bo - t_bo)^2 / (B * n_out).
Update: AdamW (decoupled weight decay), beta1 0.9, beta2 0.999, eps 1e-8:
  m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
  p <- p - lr * ( (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) + wd * p ).
Parameters are kept as FP32 master values; the forward and backward pass use
their BF16 roundings (round to nearest even), as the GPU kernels do.

Proposal inputs of a region pair (built from the ensemble field alone):
  zhat_p      centred, unit-norm member vector of grid point p (0 if constant)
  s(p)        self-similarity: mean of zhat_p . zhat_q over the grid points
              q = p +- D e_x, p +- D e_y, p +- D e_z inside the grid (0 if none)
  hot spots   per region, n_hot picks; pick i is the first point (local
              x-fastest order) maximising s among the region's points whose
              Chebyshev distance to every earlier pick exceeds r_nms (when no
              point qualifies, the previous pick is repeated)
  region row  per pick: s, local (x, y, z) / (extent - 1) (0 for extent 1);
              then the region's mean of the per-point means, mean of the
              per-point standard deviations, and centre / grid extent
  pair row    region row of a, region row of b, then |zhat_{a_i} . zhat_{b_j}|
              for i, j < n_hot (i outer): 2 (4 n_hot + 5) + n_hot^2 values.
Blob-shaped correlated structure keeps s high at range D where spatially
smooth noise has decorrelated, so the picks locate candidate extrema and the
cross terms say which of them pair up across the two regions.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Round FP32 values to BF16 (nearest even), returned as float64."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def unpack(params, n_in, H, n_out):
    """Split a flat parameter vector: W1 [n_in][H], b1, W2 [H][H], b2, W3 [H][n_out], b3."""
    sizes = [n_in * H, H, H * H, H, H * n_out, n_out]
    out, o = [], 0
    for s in sizes:
        out.append(np.asarray(params[o:o + s], np.float64))
        o += s
    W1, b1, W2, b2, W3, b3 = out
    return W1.reshape(n_in, H), b1, W2.reshape(H, H), b2, W3.reshape(H, n_out), b3


def forward(params, x, n_in, H, n_out, bf16=True):
    W1, b1, W2, b2, W3, b3 = unpack(params, n_in, H, n_out)
    if bf16:
        W1, b1, W2, b2, W3, b3 = (bf16_round(v) for v in (W1, b1, W2, b2, W3, b3))
    x = np.asarray(x, np.float64)
    z1 = x @ W1 + b1
    a1 = silu(z1)
    z2 = a1 @ W2 + b2
    a2 = silu(z2)
    y = a2 @ W3 + b3
    return y, (x, z1, a1, z2, a2, W1, W2, W3)


def loss_and_grad(params, x, t, w, n_in, H, n_out, bf16=True):
    """Weighted MSE and its gradient with respect to the (BF16-rounded) parameters."""
    y, (x, z1, a1, z2, a2, W1, W2, W3) = forward(params, x, n_in, H, n_out, bf16)
    B = x.shape[0]
    w = np.ones(n_out) if w is None else np.asarray(w, np.float64)
    diff = y - np.asarray(t, np.float64)
    L = float((w * diff * diff).sum() / (B * n_out))
    dy = 2.0 * w * diff / (B * n_out)
    gW3 = a2.T @ dy
    gb3 = dy.sum(0)
    dz2 = (dy @ W3.T) * dsilu(z2)
    gW2 = a1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * dsilu(z1)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def adamw(p, g, m, v, t, lr, wd, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v


def standardize(data):
    """FP64 mean, population sigma and zhat (M, P) of a member-major field."""
    x = np.asarray(data, np.float64)
    mu = x.mean(0)
    d = x - mu
    q = np.sqrt((d * d).sum(0))
    z = np.where(q > 0, d / np.where(q > 0, q, 1.0), 0.0)
    return mu, np.sqrt((d * d).mean(0)), z


def self_similarity(z, nx, ny, nz, D=1):
    """s(p) of the module docstring, FP64, shape (P,)."""
    M = z.shape[0]
    zz = z.reshape(M, nz, ny, nx)
    acc = np.zeros((nz, ny, nx))
    cnt = np.zeros((nz, ny, nx))
    for axis in (1, 2, 3):
        n = zz.shape[axis]
        if D >= n:
            continue
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[axis] = slice(0, n - D)
        hi[axis] = slice(D, n)
        dots = (zz[tuple(lo)] * zz[tuple(hi)]).sum(0)  # pairs (p, p + D e)
        acc[tuple(lo[1:])] += dots
        cnt[tuple(lo[1:])] += 1
        acc[tuple(hi[1:])] += dots
        cnt[tuple(hi[1:])] += 1
    return np.where(cnt > 0, acc / np.where(cnt > 0, cnt, 1), 0.0).reshape(-1)


def hot_spots(sim, region, nx, ny, n_hot=4, r_nms=3):
    """Global indices of the region's picks (module docstring)."""
    idx = region.global_indices(nx, ny)
    n = idx.size
    loc = np.arange(n)
    lx, ly, lz = loc % region.dx, (loc // region.dx) % region.dy, loc // (region.dx * region.dy)
    ok = np.ones(n, bool)
    picks = []
    for _ in range(n_hot):
        if not ok.any():
            picks.append(picks[-1])
            continue
        v = np.where(ok, sim[idx], -np.inf)
        i = int(np.argmax(v))  # first maximum in local order
        picks.append(int(idx[i]))
        ok &= np.maximum(np.maximum(np.abs(lx - lx[i]), np.abs(ly - ly[i])), np.abs(lz - lz[i])) > r_nms
    return picks


def proposal_inputs(data, nx, ny, nz, regions, region_pairs, n_hot=4, D=1, r_nms=3):
    """Pair rows (n_pairs, 2 (4 n_hot + 5) + n_hot^2) and hot spots (n_regions, n_hot)."""
    mu, sig, z = standardize(data)
    sim = self_similarity(z, nx, ny, nz, D)
    rows, hots = [], []
    for r in regions:
        h = hot_spots(sim, r, nx, ny, n_hot, r_nms)
        hots.append(h)
        f = []
        for p in h:
            x, y, zc = p % nx, (p // nx) % ny, p // (nx * ny)
            f += [sim[p], _unit(x - r.x0, r.dx), _unit(y - r.y0, r.dy), _unit(zc - r.z0, r.dz)]
        idx = r.global_indices(nx, ny)
        f += [mu[idx].mean(), sig[idx].mean(), (r.x0 + (r.dx - 1) / 2) / nx, (r.y0 + (r.dy - 1) / 2) / ny,
              (r.z0 + (r.dz - 1) / 2) / nz]
        rows.append(np.array(f))
    out = []
    for a, b in np.asarray(region_pairs).reshape(-1, 2):
        cross = np.abs(z[:, hots[a]].T @ z[:, hots[b]]).ravel()
        out.append(np.concatenate([rows[a], rows[b], cross]))
    return np.array(out), np.array(hots, dtype=np.int64)


def _unit(i, d):
    return i / (d - 1) if d > 1 else 0.0
