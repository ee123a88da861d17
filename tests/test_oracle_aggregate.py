"""Pins of the mean-tree oracle (Sec. 3.3, sampling from spatial aggregates):
a pure-Python loop over global indices on tiny ragged grids, the closed form
for fields linear in x, y, z (a block's mean is the value at the centre of
the points it holds), conservation of the member total, the tree property
(a coarser level is the count-weighted mean of the finer one), and the
brick-to-level mapping.
"""
import itertools

import numpy as np
import pytest

from oracle import aggregate_ref as AG


def _loop_means(data, nx, ny, nz, f):
    M = data.shape[0]
    NX, NY, NZ = -(-nx // f), -(-ny // f), -(-nz // f)
    out = np.zeros((M, NX * NY * NZ))
    cnt = np.zeros(NX * NY * NZ)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        q = x // f + NX * (y // f + NY * (z // f))
        cnt[q] += 1
        for m in range(M):
            out[m, q] += float(data[m, x + nx * (y + ny * z)])
    return out / cnt


@pytest.mark.parametrize("dims,f", [((5, 3, 2), 2), ((7, 6, 5), 4), ((9, 4, 3), 3), ((4, 4, 4), 4), ((3, 2, 1), 8)])
def test_block_means_brute_force(dims, f):
    nx, ny, nz = dims
    rng = np.random.default_rng(1)
    d = rng.standard_normal((3, nx * ny * nz)).astype(np.float32)
    got = AG.block_means(d, nx, ny, nz, f)
    assert got.shape == (3, np.prod(AG.level_dims(nx, ny, nz, f)))
    np.testing.assert_allclose(got, _loop_means(d, nx, ny, nz, f), rtol=0, atol=1e-12)


def test_factor_one_is_identity():
    rng = np.random.default_rng(2)
    d = rng.standard_normal((4, 6 * 5 * 3)).astype(np.float32)
    assert np.array_equal(AG.block_means(d, 6, 5, 3, 1), d.astype(np.float64))


@pytest.mark.parametrize("f", [2, 3, 4])
def test_linear_field_closed_form(f):
    nx, ny, nz = 11, 7, 6
    a, b, c, d0 = np.array([0.5, -1.0]), np.array([2.0, 0.25]), np.array([-3.0, 1.5]), np.array([1.0, -2.0])
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    data = np.stack([a[m] * x + b[m] * y + c[m] * z + d0[m] for m in range(2)]).reshape(2, -1)
    got = AG.block_means(data, nx, ny, nz, f)
    NX, NY, NZ = AG.level_dims(nx, ny, nz, f)

    def centre(i, n):
        return f * i + (min(f, n - f * i) - 1) / 2.0

    for Z, Y, X in itertools.product(range(NZ), range(NY), range(NX)):
        cx, cy, cz = centre(X, nx), centre(Y, ny), centre(Z, nz)
        q = X + NX * (Y + NY * Z)
        for m in range(2):
            assert abs(got[m, q] - (a[m] * cx + b[m] * cy + c[m] * cz + d0[m])) <= 1e-12


def test_member_total_is_conserved():
    nx, ny, nz, f = 13, 10, 7, 4
    rng = np.random.default_rng(3)
    d = rng.standard_normal((5, nx * ny * nz))
    got = AG.block_means(d, nx, ny, nz, f)
    ones = AG.block_means(np.ones((1, nx * ny * nz)), nx, ny, nz, f)
    assert np.allclose(ones, 1.0)
    NX, NY, NZ = AG.level_dims(nx, ny, nz, f)
    cnt = np.array([min(f, nx - f * X) * min(f, ny - f * Y) * min(f, nz - f * Z)
                    for Z in range(NZ) for Y in range(NY) for X in range(NX)], np.float64)
    assert cnt.sum() == nx * ny * nz
    np.testing.assert_allclose(got @ cnt, d.sum(axis=1), rtol=1e-12)


def test_tree_property():
    # level 4 from the data equals the count-weighted mean of level 2's blocks
    nx, ny, nz = 13, 10, 7
    rng = np.random.default_rng(4)
    d = rng.standard_normal((3, nx * ny * nz))
    l2 = AG.block_means(d, nx, ny, nz, 2)
    l4 = AG.block_means(d, nx, ny, nz, 4)
    NX, NY, NZ = AG.level_dims(nx, ny, nz, 2)
    cnt2 = np.array([min(2, nx - 2 * X) * min(2, ny - 2 * Y) * min(2, nz - 2 * Z)
                     for Z in range(NZ) for Y in range(NY) for X in range(NX)], np.float64)
    num = AG.block_means(l2 * cnt2, NX, NY, NZ, 2)
    den = AG.block_means(cnt2[None, :], NX, NY, NZ, 2)
    np.testing.assert_allclose(num / den, l4, rtol=0, atol=1e-12)


def test_region_at_level():
    assert AG.region_at_level((32, 64, 0, 32, 32, 20), 2) == (16, 32, 0, 16, 16, 10)
    assert AG.region_at_level((32, 64, 0, 32, 32, 20), 4) == (8, 16, 0, 8, 8, 5)
    # an unaligned brick is covered by every block it touches
    assert AG.region_at_level((3, 0, 1, 4, 5, 2), 2) == (1, 0, 0, 3, 3, 2)


def test_mean_deviation():
    rel, ab = AG.mean_deviation([0.5, 1.0, 0.0], [0.45, 1.1, 0.2])
    assert abs(rel - 0.1) < 1e-12 and abs(ab - (0.05 + 0.1 + 0.2) / 3) < 1e-12


@pytest.mark.parametrize("region,splits", [((3, 1, 0, 32, 32, 20), (2, 2, 2)), ((0, 0, 0, 7, 5, 3), (3, 2, 3)),
                                           ((2, 2, 2, 5, 1, 4), (5, 1, 2))])
def test_split_region_partitions_the_brick(region, splits):
    subs = AG.split_region(region, splits)
    assert len(subs) == splits[0] * splits[1] * splits[2]
    x0, y0, z0, dx, dy, dz = region
    cover = np.zeros((dz, dy, dx), int)
    for (x, y, z, nx, ny, nz) in subs:
        cover[z - z0:z - z0 + nz, y - y0:y - y0 + ny, x - x0:x - x0 + nx] += 1
    assert np.all(cover == 1)  # disjoint and covering
    for j, (d, s) in enumerate(zip((dx, dy, dz), splits)):
        sizes = sorted({sb[3 + j] for sb in subs})
        assert sizes[-1] - sizes[0] <= 1 and sum(sorted({(sb[j], sb[3 + j]) for sb in subs})[i][1]
                                                  for i in range(s)) == d
    # x-fastest: the second sub-brick moves along x when x is split
    if splits[0] > 1:
        assert subs[1][0] > subs[0][0] and subs[1][1:3] == subs[0][1:3]
    with pytest.raises(ValueError):
        AG.split_region((0, 0, 0, 2, 2, 2), (3, 1, 1))


def test_split_region_first_parts_larger():
    assert AG.split_region((0, 0, 0, 7, 1, 1), (3, 1, 1)) == [(0, 0, 0, 3, 1, 1), (3, 0, 0, 2, 1, 1), (5, 0, 0, 2, 1, 1)]
    assert AG.split_region((4, 0, 0, 2, 2, 1), (2, 2, 1)) == [(4, 0, 0, 1, 1, 1), (5, 0, 0, 1, 1, 1),
                                                               (4, 1, 0, 1, 1, 1), (5, 1, 0, 1, 1, 1)]
