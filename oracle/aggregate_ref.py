"""Mean-tree aggregates (Sec. 3.3, sampling from spatial aggregates) --
TEST INFRASTRUCTURE ONLY (see the package docstring).

A mean-tree level with factor f stores, for every ensemble member and every
block of f x f x f grid points, the mean of the member's values over the
block. Blocks tile the grid from the origin; a block on a high face holds the
min(f, n - f X) points that remain on that axis, and its mean is over those.
The level is itself an ensemble field on a ceil(nx/f) x ceil(ny/f) x
ceil(nz/f) grid, on which the correlation maxima of brick pairs are then
estimated (Sec. 5, the comparison of maxima at f = 1, 2 and 4).

Plain FP64 NumPy, one block at a time.
"""
from __future__ import annotations

import numpy as np


def level_dims(nx, ny, nz, f):
    """Grid extent of the level with factor f."""
    return (-(-nx // f), -(-ny // f), -(-nz // f))


def block_means(data, nx, ny, nz, f):
    """FP64 means over f^3 blocks of a member-major (M, nx*ny*nz) field.

    Returns (M, NX*NY*NZ) float64, x-fastest like the input.
    """
    if f < 1:
        raise ValueError("f must be >= 1")
    d = np.asarray(data, dtype=np.float64)
    M = d.shape[0]
    g = d[:, :nx * ny * nz].reshape(M, nz, ny, nx)
    NX, NY, NZ = level_dims(nx, ny, nz, f)
    out = np.empty((M, NZ, NY, NX))
    for Z in range(NZ):
        for Y in range(NY):
            for X in range(NX):
                blk = g[:, f * Z:f * Z + f, f * Y:f * Y + f, f * X:f * X + f]
                out[:, Z, Y, X] = blk.reshape(M, -1).sum(axis=1) / blk[0].size
    return out.reshape(M, -1)


def region_at_level(region, f):
    """(x0, y0, z0, dx, dy, dz) of the level-f blocks that cover a brick."""
    x0, y0, z0, dx, dy, dz = region
    lo = (x0 // f, y0 // f, z0 // f)
    hi = (-(-(x0 + dx) // f), -(-(y0 + dy) // f), -(-(z0 + dz) // f))
    return (lo[0], lo[1], lo[2], hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2])


def mean_deviation(max_initial, max_level):
    """Average deviation of brick-pair maxima estimated on a level from those
    on the initial data: mean of |m_f - m_1| / |m_1| over the pairs (pairs
    with m_1 = 0 are left out), and the mean absolute difference."""
    m1 = np.asarray(max_initial, np.float64)
    mf = np.asarray(max_level, np.float64)
    keep = m1 != 0
    rel = float(np.mean(np.abs(mf[keep] - m1[keep]) / np.abs(m1[keep]))) if keep.any() else 0.0
    return rel, float(np.mean(np.abs(mf - m1)))


def split_region(region, splits):
    """Sub-bricks of a brick (x0, y0, z0, dx, dy, dz) split into splits = (sx, sy, sz)
    parts per axis, as evenly as possible with the first parts one cell
    larger; listed x-fastest. Brick refinement (Sec. 3) halves each axis,
    splits = (2, 2, 2)."""
    x0, y0, z0, dx, dy, dz = region
    axes = []
    for o, d, s in ((x0, dx, splits[0]), (y0, dy, splits[1]), (z0, dz, splits[2])):
        if not (1 <= s <= d):
            raise ValueError("split count outside [1, extent]")
        parts, start = [], o
        for i in range(s):
            n = d // s + (1 if i < d % s else 0)
            parts.append((start, n))
            start += n
        axes.append(parts)
    out = []
    for (z, nz) in axes[2]:
        for (y, ny) in axes[1]:
            for (x, nx) in axes[0]:
                out.append((x, y, z, nx, ny, nz))
    return out
