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

Region features (n_pc + 5 per region): c_j = max over the region's points of
|u_j . zhat_p| for the top n_pc eigenvectors u_j of the member-space Gram
matrix G = (1/N) sum_p zhat_p zhat_p^T of all N grid points (zhat: centred,
unit-norm member vectors), then the region's mean of the per-point means,
the mean of the per-point standard deviations, and the region centre divided
by the grid extent (x, y, z).
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


def region_features(data, regions, nx, ny, nz, n_pc=16):
    """Features of each region (see the module docstring), FP64."""
    x = np.asarray(data, np.float64)  # (M, P)
    M, P = x.shape
    mu = x.mean(0)
    d = x - mu
    q = np.sqrt((d * d).sum(0))
    z = np.where(q > 0, d / np.where(q > 0, q, 1.0), 0.0)  # (M, P) unit columns
    sig = np.sqrt((d * d).mean(0))
    G = (z @ z.T) / P
    evals, evecs = np.linalg.eigh(G)
    U = evecs[:, ::-1][:, :n_pc]  # top n_pc
    proj = np.abs(U.T @ z)  # (n_pc, P)
    feats = []
    for r in regions:
        idx = r.global_indices(nx, ny)
        c = proj[:, idx].max(1)
        cx = (r.x0 + (r.dx - 1) / 2) / nx
        cy = (r.y0 + (r.dy - 1) / 2) / ny
        cz = (r.z0 + (r.dz - 1) / 2) / nz
        feats.append(np.concatenate([c, [mu[idx].mean(), sig[idx].mean(), cx, cy, cz]]))
    return np.array(feats), evals[::-1][:n_pc]
