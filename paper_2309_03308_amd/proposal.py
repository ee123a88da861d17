"""Learned BOS proposal: training records, training loop and prior cells.

A region pair's inputs (corr_proposal_inputs: self-similarity picks of both
regions, n_hot each, and the |r| between every pick of one region and every
pick of the other) are mapped by the proposal network (PropMlp) to
2 + n_hot^2 outputs:
  [0] max |r| over the pair, [1] max MI over the pair,
  [2 + i n_hot + j] the maximum |r| within Chebyshev radius `radius` of the
      candidate cell (pick i of region a, pick j of region b).
The candidate with the largest predicted neighbourhood maximum seeds batched
BOS (Sec. 3.1) as its first initial sample (bos_set_prior); plain BOS and
exhaustive search stay the reference for its error. Records come from the
method itself: exhaustive region maxima over the whole pair (corr_region_max)
and over every candidate's neighbourhood box pair (one corr_box_pairs_max call
per field) give the labels; MI labels are optional (weighted out of the loss
when absent).

Every numeric step runs in the library's kernels; this module only moves
rows between calls and converts picks into cell indices.
"""
from __future__ import annotations

import numpy as np

from . import Bos, Context, Field, PropMlp, bos_defaults, corr_proposal_inputs, region


def n_out(n_hot=4):
    return 2 + n_hot * n_hot


def _regs(regions):
    return [region(*r) if isinstance(r, tuple) else r for r in regions]


def _local(p, r, nx, ny):
    return (p % nx - r.x0, (p // nx) % ny - r.y0, p // (nx * ny) - r.z0)


def _nbhd(c, r, radius):
    """Box of local cells within Chebyshev radius of local cell c, clipped to region r."""
    lo = [max(0, c[t] - radius) for t in range(3)]
    hi = [min(d - 1, c[t] + radius) for t, d in enumerate((r.dx, r.dy, r.dz))]
    return region(r.x0 + lo[0], r.y0 + lo[1], r.z0 + lo[2], hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1)


def inputs(ctx: Context, A: Field, regions, region_pairs, n_hot=4, D=1, r_nms=3):
    """Network inputs (device) and the picks (host, n_regions x n_hot global indices)."""
    x, hot = corr_proposal_inputs(ctx, A, _regs(regions), region_pairs, n_hot=n_hot, D=D, r_nms=r_nms)
    return x, hot.cpu().numpy()


def make_records(ctx: Context, A: Field, regions, region_pairs, mi_values=None, prec="f16x3", n_hot=4, D=1, r_nms=3,
                 radius=2):
    """Inputs (device, n_pairs x width), labels (device, n_pairs x n_out) and the picks of a field's pairs."""
    torch = __import__("torch")
    regs = _regs(regions)
    rp = np.asarray(region_pairs, np.int32).reshape(-1, 2)
    x, hot = inputs(ctx, A, regs, rp, n_hot, D, r_nms)
    y = np.zeros((rp.shape[0], n_out(n_hot)), np.float32)
    boxes_a, boxes_b = [], []
    for k, (a, b) in enumerate(rp):
        ra, rb = regs[a], regs[b]
        y[k, 0] = ctx.corr_region_max(A, ra, rb, "pearson", prec)["value"]
        nb_a = [_nbhd(_local(int(hot[a, i]), ra, A.nx, A.ny), ra, radius) for i in range(n_hot)]
        nb_b = [_nbhd(_local(int(hot[b, j]), rb, A.nx, A.ny), rb, radius) for j in range(n_hot)]
        for i in range(n_hot):
            for j in range(n_hot):
                boxes_a.append(nb_a[i])
                boxes_b.append(nb_b[j])
    # every candidate neighbourhood pair of the field in one batched call
    prep = ctx.corr_prepare(A, "pearson", "f32")
    try:
        nbv = ctx.corr_box_pairs_max(prep, boxes_a, boxes_b)
    finally:
        prep.close()
    y[:, 2:] = np.array([r["value"] for r in nbv], np.float32).reshape(rp.shape[0], n_hot * n_hot)
    if mi_values is not None:
        y[:, 1] = np.asarray(mi_values, np.float32)
    return x, torch.from_numpy(y).to(x.device), hot


def loss_weights(n_hot=4, mi=False):
    return [1.0, 1.0 if mi else 0.0] + [1.0] * (n_hot * n_hot)


def train(net: PropMlp, X, Y, epochs=50, batch=256, lr=1e-3, wd=1e-4, loss_w=None, seed=0):
    """Mini-batch AdamW over shuffled records; returns the mean loss of each epoch."""
    torch = __import__("torch")
    rng = np.random.Generator(np.random.PCG64(seed))
    n = X.shape[0]
    hist = []
    for _ in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(X.device)
        tot, cnt = 0.0, 0
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            loss = net.train_step(X.index_select(0, idx), Y.index_select(0, idx), lr=lr, wd=wd, loss_w=loss_w)
            tot += loss * idx.numel()
            cnt += idx.numel()
        hist.append(tot / max(cnt, 1))
    return hist


def prior_cells(net: PropMlp, X, hot, regions, region_pairs, nx, ny, n_hot=4):
    """Predicted outputs (host) and BOS prior cells (host, n_pairs x 6): the best-scoring candidate of each pair."""
    regs = _regs(regions)
    rp = np.asarray(region_pairs, np.int32).reshape(-1, 2)
    pred = net.forward(X).cpu().numpy()
    cells = np.zeros((rp.shape[0], 6), np.float32)
    for k, (a, b) in enumerate(rp):
        c = int(np.argmax(pred[k, 2:2 + n_hot * n_hot]))
        i, j = divmod(c, n_hot)
        cells[k, :3] = _local(int(hot[a, i]), regs[a], nx, ny)
        cells[k, 3:] = _local(int(hot[b, j]), regs[b], nx, ny)
    return pred, cells


def run_bos(ctx: Context, A: Field, regions, region_pairs, prior=None, **cfg):
    """BOS over the pairs (optionally seeded with prior cells); returns (values, evaluations)."""
    regs = _regs(regions)
    bos = Bos(ctx, A, regs, region_pairs, bos_defaults(**cfg))
    try:
        if prior is not None:
            bos.bos_set_prior(prior)
        bos.bos_run()
        res = bos.bos_results()
    finally:
        bos.close()
    return np.array([r["value"] for r in res]), np.array([r["n_evaluated"] for r in res])
