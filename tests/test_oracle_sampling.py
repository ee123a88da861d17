"""Pins of the sampling oracle (Sec. 3.1 random / quasi-random sampling,
Sec. 5 sampling strategy): textbook values of the radical inverse, the
defining equation of the generalised plastic constant, the Kronecker step of
the plastic sequence, the stratification that makes the sequences
low-discrepancy (versus the uniform sampler's binomial scatter), uniformity of
every sampler's marginals, the sampled maximum as a plain argmax, and the
strategy rule at its thresholds.
"""
import math

import numpy as np
import pytest

import synth
from oracle import sampling_ref as SR


def test_radical_inverse_textbook_values():
    assert [SR.radical_inverse(n, 2) for n in range(1, 9)] == [0.5, 0.25, 0.75, 0.125, 0.625, 0.375, 0.875, 0.0625]
    third = [SR.radical_inverse(n, 3) for n in range(1, 7)]
    np.testing.assert_allclose(third, [1 / 3, 2 / 3, 1 / 9, 4 / 9, 7 / 9, 2 / 9], rtol=0, atol=1e-16)
    assert SR.radical_inverse(13 ** 3, 13) == 1 / 13 ** 4  # 1000 in base 13 -> 0.0001


def test_plastic_constant():
    p = SR.PHI6
    assert abs(p ** 7 - p - 1) < 1e-14
    assert 1.0 < p < 1.2
    al = SR.plastic_alphas()
    assert all(abs(al[j] - p ** -(j + 1)) < 1e-15 for j in range(6))


def test_plastic_kronecker_step():
    c = SR.shifts(5, 3)
    al = SR.plastic_alphas()
    for s in (0, 7, 100):
        u0 = SR.unit_point(SR.PLASTIC, 5, 3, s)
        u1 = SR.unit_point(SR.PLASTIC, 5, 3, s + 1)
        for j in range(6):
            d = (u1[j] - u0[j]) % 1.0
            assert abs(d - al[j] % 1.0) < 1e-9
    assert all(0.0 <= x < 1.0 for x in c)


def test_halton_stratification():
    # 2^k consecutive base-2 points (any shift) put exactly 2^k / 16 points
    # in each of 16 equal cells, up to one point moved by the shift's wrap
    dims = (16, 9, 5, 16, 8, 7)
    cells = SR.sample_cells(SR.HALTON, 11, 0, dims, 1024)
    cnt = np.bincount(cells[:, 0], minlength=16)
    assert np.abs(cnt - 64).max() <= 1
    cnt3 = np.bincount(cells[:, 1], minlength=9)  # base 3, 9 cells, 1024 points
    assert np.abs(cnt3 - 1024 / 9).max() <= 2


@pytest.mark.parametrize("sampler", [SR.UNIFORM, SR.HALTON, SR.PLASTIC])
def test_marginals_uniform(sampler):
    dims = (8, 8, 4, 8, 8, 4)
    n = 4096
    cells = SR.sample_cells(sampler, 3, 2, dims, n)
    assert cells.min() >= 0 and all(cells[:, j].max() < dims[j] for j in range(6))
    for j in range(6):
        cnt = np.bincount(cells[:, j], minlength=dims[j])
        exp = n / dims[j]
        chi2 = float(((cnt - exp) ** 2 / exp).sum())
        assert chi2 < 30.0, (sampler, j, chi2)  # df <= 7: p < 1e-4 beyond 30
        if sampler != SR.UNIFORM:  # low discrepancy: within one binomial sd (21 here)
            assert np.abs(cnt - exp).max() <= 20, (sampler, j, cnt)


def test_uniform_sampler_is_the_bos_generator():
    from oracle import bos_ref as B
    u = SR.unit_point(SR.UNIFORM, 9, 4, 17)
    assert u == [B.u01(B.philox4x64((4, SR.S_SAMPLE, 17, j), (9, B.KEY_HI))[0]) for j in range(6)]


def test_sample_points_are_in_the_bricks():
    ra, rb = synth.Region(3, 1, 0, 5, 4, 3), synth.Region(10, 2, 1, 6, 2, 2)
    nx, ny = 20, 8
    ia, ib = set(ra.global_indices(nx, ny).tolist()), set(rb.global_indices(nx, ny).tolist())
    for smp in (SR.UNIFORM, SR.HALTON, SR.PLASTIC):
        p = SR.sample_points(smp, 1, 0, ra, rb, nx, ny, 300)
        assert all(int(a) in ia for a in p[:, 0]) and all(int(b) in ib for b in p[:, 1])
        assert len(set(map(tuple, p.tolist()))) > 150  # a sequence, not a constant


def test_sampled_max_is_first_argmax():
    vals = np.array([0.1, -0.7, 0.7, 0.3])
    pairs = np.array([[1, 2], [3, 4], [5, 6], [7, 8]])
    assert SR.sampled_max(vals, pairs) == (0.7, -0.7, 3, 4, 4)
    assert SR.sampled_max(vals, pairs, use_abs=False) == (0.7, 0.7, 5, 6, 4)
    selfp = np.array([[1, 2], [4, 4], [5, 6], [7, 8]])
    assert SR.sampled_max(vals, selfp, same_field=True) == (0.7, 0.7, 5, 6, 3)
    assert SR.sampled_max(vals, selfp) == (0.7, -0.7, 4, 4, 4)


def test_strategy_thresholds():
    big = 32 * 32 * 20
    assert SR.choose_strategy(big, big, 1e12) == SR.BOS
    assert SR.choose_strategy(16 ** 3, 16 ** 3, 1.0) == SR.BOS
    assert SR.choose_strategy(16 ** 3 - 1, 16 ** 3, 1e12) == SR.EXHAUSTIVE
    # 4095 x 4096 pairs at 2e6 pairs/s take 8.4 s > 5 s
    assert SR.choose_strategy(16 ** 3 - 1, 16 ** 3, 2e6) == SR.RANDOM
    assert SR.choose_strategy(1000, 1000, 2e5) == SR.EXHAUSTIVE  # exactly 5 s
    assert SR.choose_strategy(1000, 1001, 2e5) == SR.RANDOM
