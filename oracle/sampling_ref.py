"""Random and quasi-random sampling of brick-pair maxima, and the switch
between BOS, random sampling and exhaustive computation -- TEST
INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.1 samples a brick pair at positions of the 6-D box (x, y, z in brick
A; x, y, z in brick B) and compares uniform pseudo-random sampling with the
Halton and plastic low-discrepancy sequences; Sec. 5 (sampling strategy)
uses BOS for bricks of at least 16x16x16 and otherwise random sampling, down
to the size where computing every point pair takes less than 5 s.

Readings (the paper names the sequences but not their construction):
* a sample is u in [0, 1)^6 mapped to cell c_j = min(floor(u_j d_j), d_j - 1)
  with d = (A.dx, A.dy, A.dz, B.dx, B.dy, B.dz);
* uniform: u_j = U(philox(pair, S_SAMPLE, s, j)), the generator and the
  53-bit conversion of the BOS oracle;
* Halton: u_j = frac(h_{b_j}(s + 1) + c_j) with the first six primes as bases
  and one Cranley-Patterson shift c_j = U(philox(pair, S_SHIFT, 0, j)) per
  pair (so repeated runs with other seeds differ); h_b(n) reverses the base-b
  digits of n behind the radix point, computed as an exact ratio of integers;
* plastic: the d-dimensional generalisation of the plastic-number sequence,
  u_j = frac(c_j + (s + 1) alpha_j) with alpha_j = phi^-j, phi the real root
  above 1 of x^7 = x + 1 (d = 6), the same per-pair shift;
* the maximum of a brick pair over its samples uses the region-maximum rule
  (objective |r| for Pearson, MI for KSG, the earliest of equal values, and
  within one field no point paired with itself);
* strategy: BOS when both bricks hold at least 16^3 points, else the
  exhaustive computation when |A| |B| / rate is at most the time budget
  (5 s), else uniform random sampling.

Plain Python / NumPy, one sample at a time.
"""
from __future__ import annotations

import math

import numpy as np

from .bos_ref import KEY_HI, philox4x64, u01

S_SAMPLE, S_SHIFT = 5, 6
UNIFORM, HALTON, PLASTIC = 0, 1, 2
HALTON_BASES = (2, 3, 5, 7, 11, 13)
PHI6 = 1.1127756842787055  # real root > 1 of x^7 = x + 1, correctly rounded
BOS, RANDOM, EXHAUSTIVE = 0, 1, 2


def radical_inverse(n: int, b: int) -> float:
    """Digits of n (base b) mirrored behind the radix point, as one FP64 ratio."""
    num, den = 0, 1
    while n > 0:
        n, d = divmod(n, b)
        num = num * b + d
        den *= b
    return num / den


def plastic_alphas():
    a, out = 1.0, []
    for _ in range(6):
        a = a / PHI6
        out.append(a)
    return out


def _frac(x: float) -> float:
    return x - math.floor(x)


def shifts(seed: int, pair: int):
    return [u01(philox4x64((pair, S_SHIFT, 0, j), (seed, KEY_HI))[0]) for j in range(6)]


def unit_point(sampler: int, seed: int, pair: int, s: int):
    """The sample's u in [0, 1)^6."""
    if sampler == UNIFORM:
        return [u01(philox4x64((pair, S_SAMPLE, s, j), (seed, KEY_HI))[0]) for j in range(6)]
    c = shifts(seed, pair)
    if sampler == HALTON:
        return [_frac(radical_inverse(s + 1, HALTON_BASES[j]) + c[j]) for j in range(6)]
    if sampler == PLASTIC:
        al = plastic_alphas()
        return [_frac(c[j] + (s + 1) * al[j]) for j in range(6)]
    raise ValueError("unknown sampler")


def sample_cells(sampler: int, seed: int, pair: int, dims, n: int) -> np.ndarray:
    """(n, 6) int64 cells of a brick pair with extents dims = (ax, ay, az, bx, by, bz)."""
    out = np.zeros((n, 6), np.int64)
    for s in range(n):
        u = unit_point(sampler, seed, pair, s)
        for j in range(6):
            out[s, j] = min(int(math.floor(u[j] * dims[j])), dims[j] - 1)
    return out


def sample_points(sampler, seed, pair, ra, rb, nx, ny, n):
    """(n, 2) int32 global point pairs: the samples of bricks ra x rb (Region objects)."""
    dims = (ra.dx, ra.dy, ra.dz, rb.dx, rb.dy, rb.dz)
    c = sample_cells(sampler, seed, pair, dims, n)
    pa = (ra.x0 + c[:, 0]) + nx * ((ra.y0 + c[:, 1]) + ny * (ra.z0 + c[:, 2]))
    pb = (rb.x0 + c[:, 3]) + nx * ((rb.y0 + c[:, 4]) + ny * (rb.z0 + c[:, 5]))
    return np.stack([pa, pb], 1).astype(np.int32)


def sampled_max(values, pairs, use_abs=True, same_field=False):
    """(value, signed value, pA, pB, samples counted) of the earliest maximum
    over the samples; within one field a point paired with itself is no
    sample (the region-maximum rule)."""
    values = np.asarray(values)
    keep = np.ones(len(values), bool)
    if same_field:
        keep = pairs[:, 0] != pairs[:, 1]
    if not keep.any():
        return 0.0, 0.0, -1, -1, 0
    v = np.where(keep, np.abs(values) if use_abs else values, -np.inf)
    i = int(np.argmax(v))  # first of equal maxima
    return float(v[i]), float(values[i]), int(pairs[i, 0]), int(pairs[i, 1]), int(keep.sum())


def choose_strategy(na: int, nb: int, pairs_per_s: float, budget_s: float = 5.0, bos_min: int = 16 ** 3) -> int:
    """BOS, RANDOM or EXHAUSTIVE for bricks of na and nb points."""
    if na >= bos_min and nb >= bos_min:
        return BOS
    if na * nb <= budget_s * pairs_per_s:
        return EXHAUSTIVE
    return RANDOM
