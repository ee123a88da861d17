"""Learned BOS proposal: training records, training loop and prior cells.

A region pair's inputs (corr_proposal_inputs: self-similarity hot spots of
both regions and their cross correlations) are mapped by the proposal network
(PropMlp) to eight outputs:
  [0] max |r| over the pair, [1] max MI over the pair,
  [2:5] location of the maximum in region a, local (x, y, z) / (extent - 1),
  [5:8] the same in region b.
The predicted location seeds batched BOS (Sec. 3.1) as its first initial
sample (bos_set_prior); plain BOS and exhaustive search stay the reference
for its error. Records come from the method itself: exhaustive region maxima
(corr_region_max) give the Pearson labels; MI labels are optional (BOS maxima
when given, else weighted out of the loss).

Every numeric step runs in the library's kernels; this module only moves
rows between calls and converts predicted positions into cell indices.
"""
from __future__ import annotations

import numpy as np

from . import Bos, Context, Field, PropMlp, bos_defaults, corr_proposal_inputs, region

N_OUT = 8


def _regs(regions):
    return [r if not isinstance(r, tuple) else region(*r) for r in regions]


def _dims(r):
    return (r.dx, r.dy, r.dz)


def _local_unit(p, r, nx, ny):
    x, y, z = p % nx, (p // nx) % ny, p // (nx * ny)
    return [(v - o) / (d - 1) if d > 1 else 0.0 for v, o, d in ((x, r.x0, r.dx), (y, r.y0, r.dy), (z, r.z0, r.dz))]


def make_records(ctx: Context, A: Field, regions, region_pairs, mi_values=None, prec="f16x3", n_hot=4, D=4,
                 r_nms=3):
    """Inputs (device, n_pairs x width) and labels (device, n_pairs x 8) of a field's region pairs."""
    torch = __import__("torch")
    regs = _regs(regions)
    rp = np.asarray(region_pairs, np.int32).reshape(-1, 2)
    x, _ = corr_proposal_inputs(ctx, A, regs, rp, n_hot=n_hot, D=D, r_nms=r_nms)
    y = np.zeros((rp.shape[0], N_OUT), np.float32)
    for k, (a, b) in enumerate(rp):
        m = ctx.corr_region_max(A, regs[a], regs[b], "pearson", prec)
        y[k, 0] = m["value"]
        y[k, 2:5] = _local_unit(m["pa"], regs[a], A.nx, A.ny)
        y[k, 5:8] = _local_unit(m["pb"], regs[b], A.nx, A.ny)
    if mi_values is not None:
        y[:, 1] = np.asarray(mi_values, np.float32)
    return x, torch.from_numpy(y).to(x.device)


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


def prior_cells(net: PropMlp, X, regions, region_pairs):
    """Predicted outputs (host, n_pairs x 8) and BOS prior cells (host, n_pairs x 6)."""
    regs = _regs(regions)
    rp = np.asarray(region_pairs, np.int32).reshape(-1, 2)
    pred = net.forward(X).cpu().numpy()
    cells = np.zeros((rp.shape[0], 6), np.float32)
    for k, (a, b) in enumerate(rp):
        da, db = _dims(regs[a]), _dims(regs[b])
        for t in range(3):
            cells[k, t] = np.clip(pred[k, 2 + t], 0.0, 1.0) * (da[t] - 1)
            cells[k, 3 + t] = np.clip(pred[k, 5 + t], 0.0, 1.0) * (db[t] - 1)
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
