"""The long-K contraction on 256 x 256 workgroup tiles (single-pass FP16 and
BF16, taken when the two bricks give at least one such tile per CU) against
the oracle's exhaustive region maximum: bricks of 4000 and 4200 points
(ragged against both the 256-row tiles and the 128-row padding of the staged
rows, so the last tiles read clamped rows that must be masked), a brick
overlapping the other (points paired with themselves left out), the smallest
member count the long-K path takes (129), an uneven one and M = 1000.

A second set plants one strongly correlated pair at chosen positions -- every
wave quadrant and 32 x 32 accumulator block of a tile, the first and last
rows and columns, the ragged edge tiles -- in otherwise independent data;
the returned argmax must be that pair and its value the oracle's r there.

Bars: value within the precision's tolerance, n_evaluated exact, argmax
valid (and equal to the oracle's where its top-2 gap exceeds twice the
tolerance).
"""
import sys

import numpy as np
import pytest

import oracle
from argmax_checks import check_pearson_argmax
import synth

pytestmark = pytest.mark.gpu

TOL = {"f16": 2e-3, "bf16": 7.9e-3}
DIMS = (40, 25, 10)                 # 10 000 points
RA = (0, 0, 0, 20, 20, 10)          # 4000 points
RB = (20, 4, 0, 20, 21, 10)         # 4200 points
RB_OVERLAP = (10, 0, 0, 20, 21, 10)  # shares x = 10..19 with RA


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as pc
    ctx = pc.Context(0)
    yield dict(torch=torch, pc=pc, ctx=ctx)
    ctx.close()


def _field(M, seed):
    rng = np.random.default_rng(seed)
    P = DIMS[0] * DIMS[1] * DIMS[2]
    common = rng.standard_normal((M, 4))
    mix = rng.standard_normal((4, P)) * (rng.uniform(size=P) < 0.3)
    d = rng.standard_normal((M, P)) + common @ mix + rng.uniform(-3, 3, P)
    return np.ascontiguousarray(d.astype(np.float32))


def _indices(r):
    return synth.Region(*r).global_indices(DIMS[0], DIMS[1])


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("M", [129, 300, 1000])
@pytest.mark.parametrize("rb", [RB, RB_OVERLAP], ids=["disjoint", "overlapping"])
def test_wide_tiles_against_oracle(env, M, prec, rb):
    pc, ctx, torch = env["pc"], env["ctx"], env["torch"]
    data = _field(M, seed=M + (7 if rb is RB_OVERLAP else 0))
    f = pc.Field(torch.from_numpy(data).cuda(), *DIMS)
    got = ctx.corr_region_max(f, pc.region(*RA), pc.region(*rb), "pearson", prec)
    ia, ib = _indices(RA), _indices(rb)
    ref = oracle.pearson_region_max_matmul(data, ia, ib)
    _say(f"  wide M={M} {prec} {RA}x{rb}: gpu {got['value']:.6f} oracle {ref['value']:.6f}")
    assert abs(got["value"] - ref["value"]) <= TOL[prec]
    assert got["n_evaluated"] == ref["n_evaluated"]
    check_pearson_argmax(got, ref, data, ia, ib, TOL[prec])


def _plant_positions():
    # (local row in A, local column in B): first / last rows and columns,
    # each wave quadrant and accumulator block of the first tile, interior
    # tiles, and the ragged edge tiles (rows 3840..3999, columns 4096..4199)
    pos = [(0, 0), (3999, 4199), (0, 4199), (3999, 0), (3840, 4096), (3999, 4096)]
    for wr in range(2):
        for wc in range(2):
            for i in range(4):
                pos.append((wr * 128 + i * 32 + (5 * i + 3) % 32, wc * 128 + ((i + 1) % 4) * 32 + (7 * i + 11) % 32))
    rng = np.random.default_rng(11)
    for _ in range(6):
        pos.append((int(rng.integers(0, 4000)), int(rng.integers(0, 4200))))
    return pos


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_wide_tiles_planted_pairs(env, prec):
    pc, ctx, torch = env["pc"], env["ctx"], env["torch"]
    M = 300
    rng = np.random.default_rng(5)
    base = rng.standard_normal((M, DIMS[0] * DIMS[1] * DIMS[2])).astype(np.float32)
    ia, ib = _indices(RA), _indices(RB)
    for la, lb in _plant_positions():
        pa, pb = int(ia[la]), int(ib[lb])
        data = base.copy()
        data[:, pb] = 0.98 * data[:, pa] + 0.2 * rng.standard_normal(M).astype(np.float32)
        f = pc.Field(torch.from_numpy(data).cuda(), *DIMS)
        got = ctx.corr_region_max(f, pc.region(*RA), pc.region(*RB), "pearson", prec)
        r = float(oracle.pearson_pairs(data, np.array([[pa, pb]], np.int32))[0])
        _say(f"  planted ({la},{lb}) {prec}: gpu ({got['pa']},{got['pb']}) {got['value']:.5f}, oracle r {r:.5f}")
        assert (int(got["pa"]), int(got["pb"])) == (pa, pb)
        assert abs(got["value"] - abs(r)) <= TOL[prec]
        assert abs(got["signed_value"] - r) <= TOL[prec]


# Bricks of 6000 x 6300 points: 24 x 25 = 600 tiles, at least two per CU, so
# the eight-wave layout runs (2 x 4 waves of 128 x 64); ragged against the
# 256-row tiles and the 128-row padding.
DIMS8 = (50, 40, 8)
RA8 = (0, 0, 0, 25, 40, 6)
RB8 = (25, 0, 0, 25, 36, 7)


def _indices8(r):
    return synth.Region(*r).global_indices(DIMS8[0], DIMS8[1])


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("M", [129, 300])
def test_eight_wave_tiles_against_oracle(env, M, prec):
    pc, ctx, torch = env["pc"], env["ctx"], env["torch"]
    rng = np.random.default_rng(100 + M)
    P = DIMS8[0] * DIMS8[1] * DIMS8[2]
    common = rng.standard_normal((M, 4))
    mix = rng.standard_normal((4, P)) * (rng.uniform(size=P) < 0.3)
    data = np.ascontiguousarray((rng.standard_normal((M, P)) + common @ mix).astype(np.float32))
    f = pc.Field(torch.from_numpy(data).cuda(), *DIMS8)
    got = ctx.corr_region_max(f, pc.region(*RA8), pc.region(*RB8), "pearson", prec)
    ia, ib = _indices8(RA8), _indices8(RB8)
    ref = oracle.pearson_region_max_matmul(data, ia, ib)
    _say(f"  eight-wave M={M} {prec}: gpu {got['value']:.6f} oracle {ref['value']:.6f}")
    assert abs(got["value"] - ref["value"]) <= TOL[prec]
    assert got["n_evaluated"] == ref["n_evaluated"]
    check_pearson_argmax(got, ref, data, ia, ib, TOL[prec])


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_eight_wave_tiles_planted_pairs(env, prec):
    pc, ctx, torch = env["pc"], env["ctx"], env["torch"]
    M = 160
    rng = np.random.default_rng(6)
    base = rng.standard_normal((M, DIMS8[0] * DIMS8[1] * DIMS8[2])).astype(np.float32)
    ia, ib = _indices8(RA8), _indices8(RB8)
    # every wave (2 rows x 4 columns of 128 x 64) and accumulator block of a
    # tile, the first / last rows and columns, the ragged edge tiles
    pos = [(0, 0), (5999, 6299), (5888, 6144), (5999, 0), (0, 6299)]
    for wr in range(2):
        for wc in range(4):
            for i in range(4):
                pos.append((256 * 3 + wr * 128 + i * 32 + (7 * i + 5) % 32, 256 * 5 + wc * 64 + (i % 2) * 32 + (3 * i + 9) % 32))
    for la, lb in pos:
        pa, pb = int(ia[la]), int(ib[lb])
        data = base.copy()
        data[:, pb] = 0.98 * data[:, pa] + 0.2 * rng.standard_normal(M).astype(np.float32)
        f = pc.Field(torch.from_numpy(data).cuda(), *DIMS8)
        got = ctx.corr_region_max(f, pc.region(*RA8), pc.region(*RB8), "pearson", prec)
        r = float(oracle.pearson_pairs(data, np.array([[pa, pb]], np.int32))[0])
        assert (int(got["pa"]), int(got["pb"])) == (pa, pb), ((la, lb), got)
        assert abs(got["value"] - abs(r)) <= TOL[prec]
        assert abs(got["signed_value"] - r) <= TOL[prec]
