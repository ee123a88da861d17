"""Seeded smoothed-Gaussian ensemble fields with planted correlated blobs.

The paper's data sets (a weather ensemble on a 250x352x20 grid with 1000
members, a 180-member 640x704x64 ensemble, and a 1000-member synthetic
256x256x32 set, Sec. 5.1) are not available, so every workload here is a
seeded stand-in of the same structure: an ensemble of E (here ``M``) members
on a regular X x Y x Z grid, one scalar variable per point (Sec. 3).

Recipe (all randomness from ``numpy.random.Generator(PCG64(seed))``):

* white noise ``W_m ~ N(0, 1)`` per member and cell;
* ``F_m`` = Gaussian smoothing of ``W_m`` (sigma = 2 cells, periodic
  boundaries, kernel truncated at 4 sigma), divided by the L2 norm of the 3D
  smoothing kernel so every cell has unit variance;
* a planted group ``g`` has one shared member signal ``S_g ~ N(0, 1)`` and an
  amplitude ``a_g = sqrt(rho_g / (1 - rho_g))``; every cell within Euclidean
  distance ``r`` of one of the group's blob centres is replaced by
  ``(F + a_g S_g) / sqrt(1 + a_g^2)``, so two cells in far-apart blobs of the
  same group correlate with population coefficient exactly ``rho_g``
  (the planted-cluster idea of the paper's first synthetic set, Sec. 5.1);
* the large-ensemble workload adds ``0.5 * T`` with ``T ~ Student-t(4)/sqrt(2)``
  i.i.d. per member and cell, then stores the field as FP16
  (round-to-nearest-even); the FP16 values are the input for every consumer.

Layout: ``data[m, p]`` member-major, ``p = x + nx * (y + ny * z)``.
This module computes no correlation of any kind.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.ndimage as ndi

SMOOTH_SIGMA = 2.0
SMOOTH_TRUNCATE = 4.0


@dataclasses.dataclass(frozen=True)
class Region:
    """Half-open box [x0, x0+dx) x [y0, y0+dy) x [z0, z0+dz) of grid cells."""

    x0: int
    y0: int
    z0: int
    dx: int
    dy: int
    dz: int

    @property
    def npts(self) -> int:
        return self.dx * self.dy * self.dz

    def as_tuple(self):
        return (self.x0, self.y0, self.z0, self.dx, self.dy, self.dz)

    def global_indices(self, nx: int, ny: int) -> np.ndarray:
        """Global linear indices of the region's cells in local x-fastest order."""
        z, y, x = np.meshgrid(
            np.arange(self.z0, self.z0 + self.dz),
            np.arange(self.y0, self.y0 + self.dy),
            np.arange(self.x0, self.x0 + self.dx),
            indexing="ij",
        )
        return (x + nx * (y + ny * z)).reshape(-1).astype(np.int32)

    def center(self):
        return (self.x0 + (self.dx - 1) / 2, self.y0 + (self.dy - 1) / 2, self.z0 + (self.dz - 1) / 2)


@dataclasses.dataclass
class Ensemble:
    """A generated ensemble plus the metadata that describes its structure."""

    name: str
    data: np.ndarray  # (M, P) member-major, float32 or float16
    nx: int
    ny: int
    nz: int
    regions: list
    groups: list  # [{"rho": float, "blobs": [(cx, cy, cz, r), ...]}]
    seed: int

    @property
    def M(self) -> int:
        return int(self.data.shape[0])

    @property
    def P(self) -> int:
        return self.nx * self.ny * self.nz


def _kernel_l2_norm(sigma: float, truncate: float) -> float:
    radius = int(truncate * sigma + 0.5)
    t = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-0.5 * (t / sigma) ** 2)
    w /= w.sum()
    return float(np.sqrt(np.sum(w * w)) ** 3)


def smooth_noise(rng: np.random.Generator, M: int, nz: int, ny: int, nx: int,
                 sigma: float = SMOOTH_SIGMA, chunk: int = 64, threads: int = 0) -> np.ndarray:
    """Unit-variance periodic smoothed white noise, shape (M, nz, ny, nx), float32.

    The noise is drawn chunk by chunk in member order (so the result does not
    depend on ``threads``); the smoothing of the chunks runs on a thread pool.
    """
    import concurrent.futures
    import os

    out = np.empty((M, nz, ny, nx), dtype=np.float32)
    norm = np.float32(_kernel_l2_norm(sigma, SMOOTH_TRUNCATE))

    def smooth(m0, w):
        ndi.gaussian_filter(w, sigma=(0.0, sigma, sigma, sigma), mode="wrap",
                            truncate=SMOOTH_TRUNCATE, output=out[m0:m0 + w.shape[0]])
        out[m0:m0 + w.shape[0]] /= norm

    n_threads = threads or min(16, os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(max_workers=n_threads) as ex:
        futs = []
        for m0 in range(0, M, chunk):
            m1 = min(M, m0 + chunk)
            w = rng.standard_normal((m1 - m0, nz, ny, nx), dtype=np.float32)
            futs.append(ex.submit(smooth, m0, w))
            if len(futs) >= 2 * n_threads:
                futs.pop(0).result()
        for f in futs:
            f.result()
    return out


def _plant(field: np.ndarray, rng: np.random.Generator, groups: list) -> None:
    """Overwrite blob cells of each group with the mixed shared signal (in place)."""
    M, nz, ny, nx = field.shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for g in groups:
        rho = g["rho"]
        a = math.sqrt(rho / (1.0 - rho))
        s = rng.standard_normal(M).astype(np.float32)
        for (cx, cy, cz, r) in g["blobs"]:
            mask = (xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2 <= r * r
            f = field[:, mask]
            field[:, mask] = ((f + np.float32(a) * s[:, None]) / np.float32(math.sqrt(1.0 + a * a))).astype(np.float32)


def make_field(name, seed, M, nx, ny, nz, groups, regions, heavy_tail=0.0, offset=0.0,
               store=np.float32) -> Ensemble:
    rng = np.random.Generator(np.random.PCG64(seed))
    f = smooth_noise(rng, M, nz, ny, nx)
    _plant(f, rng, groups)
    if heavy_tail:
        for m0 in range(0, M, 64):
            m1 = min(M, m0 + 64)
            t = rng.standard_t(4.0, size=(m1 - m0, nz, ny, nx)).astype(np.float32)
            f[m0:m1] += np.float32(heavy_tail / math.sqrt(2.0)) * t
    if offset:
        f += np.float32(offset)
    data = np.ascontiguousarray(f.reshape(M, nx * ny * nz)).astype(store)
    return Ensemble(name, data, nx, ny, nz, list(regions), groups, seed)


def _place_centers(rng, region: Region, n, margin, min_sep, taken=()):
    lo = np.array([region.x0 + margin, region.y0 + margin, region.z0 + margin])
    hi = np.array([region.x0 + region.dx - 1 - margin, region.y0 + region.dy - 1 - margin,
                   region.z0 + region.dz - 1 - margin])
    out = []
    for _ in range(100000):
        if len(out) == n:
            break
        c = rng.integers(lo, hi + 1)
        if all(np.linalg.norm(c - np.array(o)) >= min_sep for o in list(out) + list(taken)):
            out.append(tuple(int(v) for v in c))
    if len(out) != n:
        raise RuntimeError("blob placement failed")
    return out


def make_cfg1(copy_variant: bool = False) -> Ensemble:
    """16x8x4 grid, M=100, two 8x8x4 regions, one planted group (rho=0.8, r=1.5)."""
    ra, rb = Region(0, 0, 0, 8, 8, 4), Region(8, 0, 0, 8, 8, 4)
    groups = [{"rho": 0.8, "blobs": [(3.5, 3.5, 1.5, 1.5), (11.5, 3.5, 1.5, 1.5)]}]
    e = make_field("tiny-16x8x4-M100", 1, 100, 16, 8, 4, groups, [ra, rb])
    if copy_variant:
        p = 1 + 16 * (2 + 8 * 1)        # (1, 2, 1) in region A
        q = 13 + 16 * (5 + 8 * 2)       # (13, 5, 2) in region B
        e.data[:, q] = e.data[:, p]
        e.name += "-copy"
        e.copy_pair = (p, q)
    return e


def make_cfg2(seed: int = 2) -> Ensemble:
    """80x32x20 grid, M=100, regions x in [0,32) and [48,80), 3 planted groups (r=4)."""
    ra, rb = Region(0, 0, 0, 32, 32, 20), Region(48, 0, 0, 32, 32, 20)
    rng = np.random.Generator(np.random.PCG64(10_000 + seed))
    ca = _place_centers(rng, ra, 3, 4, 10)
    cb = _place_centers(rng, rb, 3, 4, 10)
    groups = [{"rho": rho, "blobs": [(*ca[g], 4.0), (*cb[g], 4.0)]}
              for g, rho in enumerate((0.5, 0.8, 0.95))]
    return make_field("focus-80x32x20-M100", seed, 100, 80, 32, 20, groups, [ra, rb])


def context_regions(ni: int, nj: int, dims=(32, 32, 20)):
    dx, dy, dz = dims
    return [Region(dx * i, dy * j, 0, dx, dy, dz) for j in range(nj) for i in range(ni)]


def cfg3_regions():
    return context_regions(11, 8)


def make_context(ni: int, nj: int, dims=(32, 32, 20), M: int = 100, seed: int = 3, n_groups: int = 8,
                 blob_r: float = 4.0, min_region_gap: int = 3, name: str = None) -> Ensemble:
    """Grid of ni x nj regions (one region layer), planted groups of 2-3 blobs
    in regions at least `min_region_gap` region steps apart (Chebyshev)."""
    regions = context_regions(ni, nj, dims)
    rng = np.random.Generator(np.random.PCG64(10_000 + seed))
    used = set()
    groups = []
    margin = int(min(blob_r, (min(dims) - 1) // 2))
    for g in range(n_groups):
        nb = int(rng.integers(2, 4))
        chosen = []
        for _ in range(100000):
            if len(chosen) == nb:
                break
            r = int(rng.integers(0, ni * nj))
            ri, rj = r % ni, r // ni
            if r in used or any(max(abs(ri - c % ni), abs(rj - c // ni)) < min_region_gap for c in chosen):
                continue
            chosen.append(r)
        if len(chosen) < 2:
            continue
        used.update(chosen)
        blobs = [(*_place_centers(rng, regions[r], 1, margin, 0)[0], blob_r) for r in chosen]
        groups.append({"rho": (0.5, 0.8, 0.95)[g % 3], "blobs": blobs, "regions": chosen})
    nx, ny, nz = ni * dims[0], nj * dims[1], dims[2]
    return make_field(name or f"context-{nx}x{ny}x{nz}-M{M}", seed, M, nx, ny, nz, groups, regions)


def make_cfg3(M: int = 100, seed: int = 3) -> Ensemble:
    """352x256x20 grid, M members, 88 regions of 32x32x20, 8 planted groups of 2-3 blobs."""
    return make_context(11, 8, (32, 32, 20), M, seed, 8, 4.0, 3, f"context-352x256x20-M{M}")


def make_two_variables(nx=24, ny=16, nz=8, M=100, seed=7, rho=0.8, blob_r=2.5):
    """Two variables U, V of one ensemble on the same grid (independent
    smoothed noise), with one shared member signal planted in a blob of U in
    the left half and a blob of V in the right half, so that U there and V
    there correlate with rho. Returns (U, V, regions) with regions the left
    and right halves."""
    rng = np.random.Generator(np.random.PCG64(20_000 + seed))
    fu = smooth_noise(rng, M, nz, ny, nx)
    fv = smooth_noise(rng, M, nz, ny, nx)
    s = rng.standard_normal(M).astype(np.float32)
    a = math.sqrt(rho / (1.0 - rho))
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for f, cx in ((fu, nx // 4), (fv, 3 * nx // 4)):
        mask = (xx - cx) ** 2 + (yy - ny // 2) ** 2 + (zz - nz // 2) ** 2 <= blob_r * blob_r
        f[:, mask] = ((f[:, mask] + np.float32(a) * s[:, None]) / np.float32(math.sqrt(1.0 + a * a))).astype(
            np.float32)
    regs = [Region(0, 0, 0, nx // 2, ny, nz), Region(nx // 2, 0, 0, nx - nx // 2, ny, nz)]
    U = Ensemble("U", np.ascontiguousarray(fu.reshape(M, -1)), nx, ny, nz, regs, [], seed)
    V = Ensemble("V", np.ascontiguousarray(fv.reshape(M, -1)), nx, ny, nz, regs, [], seed)
    return U, V, regs


def region_pair_list(n_regions: int) -> np.ndarray:
    """All unordered pairs (i < j) of regions, int32 (n, 2)."""
    i, j = np.triu_indices(n_regions, 1)
    return np.ascontiguousarray(np.stack([i, j], 1).astype(np.int32))


def make_cfg4(stress_offset: bool = False, M: int = 1000, seed: int = 4) -> Ensemble:
    """128x128x32 grid, M=1000, Student-t perturbation, FP16 storage, 4 planted groups."""
    ra, rb = Region(0, 0, 0, 16, 16, 16), Region(64, 64, 16, 16, 16, 16)
    rng = np.random.Generator(np.random.PCG64(10_004))
    fa, fb = (8, 8, 8), (72, 72, 24)
    taken = [fa, fb]
    whole = Region(0, 0, 0, 128, 128, 32)
    groups = []
    for g, rho in enumerate((0.5, 0.8, 0.9, 0.95)):
        if rho == 0.9:
            blobs = [(*fa, 4.0), (*fb, 4.0)]
        else:
            cs = _place_centers(rng, whole, 2, 5, 14, taken)
            taken += cs
            blobs = [(*c, 4.0) for c in cs]
        groups.append({"rho": rho, "blobs": blobs})
    name = "large-128x128x32-M%d-fp16%s" % (M, "-offset8" if stress_offset else "")
    return make_field(name, seed, M, 128, 128, 32, groups, [ra, rb], heavy_tail=0.5,
                      offset=8.0 if stress_offset else 0.0, store=np.float16)


def random_pairs(seed: int, n: int, P: int, distinct: bool = True) -> np.ndarray:
    """n uniform (pA, pB) global index pairs over a whole P-point field, int32 (n, 2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.integers(0, P, n, dtype=np.int64)
    b = rng.integers(0, P, n, dtype=np.int64)
    if distinct:
        same = a == b
        while same.any():
            b[same] = rng.integers(0, P, int(same.sum()), dtype=np.int64)
            same = a == b
    return np.ascontiguousarray(np.stack([a, b], 1).astype(np.int32))


def region_pairs_uniform(seed: int, n: int, ra: Region, rb: Region, nx: int, ny: int) -> np.ndarray:
    """n pairs drawn uniformly with replacement from region A x region B, int32 (n, 2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ia, ib = ra.global_indices(nx, ny), rb.global_indices(nx, ny)
    a = ia[rng.integers(0, ia.size, n)]
    b = ib[rng.integers(0, ib.size, n)]
    return np.ascontiguousarray(np.stack([a, b], 1).astype(np.int32))
