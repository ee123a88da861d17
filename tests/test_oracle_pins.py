"""Pins for the CPU oracle: checks against mathematics and library routines,
never against the oracle's own formulas retyped.

Each test names the passage (arXiv 2309.03308) whose definition it fixes.
"""
import math

import numpy as np
import pytest
import scipy.special

import oracle
import synth

GAMMA = 0.57721566490153286060651209


# ---------------------------------------------------------------- digamma (Eq. 2)
def test_digamma_matches_scipy():
    for n in list(range(1, 60)) + [99, 100, 101, 999, 1000, 1001]:
        assert abs(oracle.digamma_int(n) - scipy.special.digamma(n)) <= 1e-13 * max(1.0, abs(scipy.special.digamma(n)))


def test_digamma_one_is_minus_gamma():
    assert oracle.digamma_int(1) == pytest.approx(-GAMMA, abs=1e-16)


# ---------------------------------------------------------------- Pearson (Sec. 3.2)
def test_pearson_matches_numpy_corrcoef_cfg1():
    e = synth.make_cfg1()
    ia = e.regions[0].global_indices(e.nx, e.ny)
    ib = e.regions[1].global_indices(e.nx, e.ny)
    pairs = np.stack(np.meshgrid(ia, ib, indexing="ij"), -1).reshape(-1, 2).astype(np.int32)
    r = oracle.pearson_pairs(e.data, pairs).reshape(ia.size, ib.size)
    ref = np.corrcoef(e.data[:, ia].T.astype(np.float64), e.data[:, ib].T.astype(np.float64))[: ia.size, ia.size:]
    assert np.max(np.abs(r - ref)) <= 1e-12
    assert np.max(np.abs(r)) <= 1 + 1e-15


def test_pearson_affine_copy_sign_and_invariance():
    rng = np.random.default_rng(11)
    M = 100
    base = rng.standard_normal(M)
    cols = [base, 3.0 * base + 7.0, -0.25 * base - 2.0, base + 100.0, 2.0 ** 5 * base]
    x = np.stack(cols, 1).astype(np.float64)
    # the affine maps are exact in FP64 above; pass FP32 only where exact
    data = x.astype(np.float32)
    # exact float32 affine copies: scale by powers of two, shift by small ints
    data[:, 1] = data[:, 0] * np.float32(4.0)
    data[:, 2] = data[:, 0] * np.float32(-0.5)
    data[:, 4] = data[:, 0] * np.float32(32.0)
    pairs = np.array([[0, 1], [0, 2], [0, 4], [1, 2], [0, 0]], np.int32)
    r = oracle.pearson_pairs(data, pairs)
    assert r == pytest.approx([1.0, -1.0, 1.0, -1.0, 1.0], abs=1e-15)
    # shift invariance (shift of 100 is not exact in FP32, compare to corrcoef)
    rr = oracle.pearson_pairs(data, np.array([[3, 1]], np.int32))[0]
    assert rr == pytest.approx(np.corrcoef(data[:, 3].astype(np.float64), data[:, 1].astype(np.float64))[0, 1], abs=1e-14)


def test_pearson_symmetry_and_zero_variance():
    rng = np.random.default_rng(5)
    data = rng.standard_normal((50, 6)).astype(np.float32)
    data[:, 5] = 1.5  # constant point -> r = 0
    pairs = np.array([[0, 1], [1, 0], [2, 5], [5, 3]], np.int32)
    r = oracle.pearson_pairs(data, pairs)
    assert r[0] == r[1]
    assert r[2] == 0.0 and r[3] == 0.0


# ---------------------------------------------------------------- KSG (Sec. 3.2)
def test_ksg_hand_worked_example():
    # M = 5 samples, k = 2. Worked by hand from the definition:
    #  i  (x, y)    sorted d_ij        eps  n_x n_y
    #  0  (0, 0)    3, 3, 6, 10        3    1   2
    #  1  (1, 3)    2, 3, 5, 9         3    2   2
    #  2  (3, 1)    2, 3, 3, 8         3    1   3
    #  3  (6, 2)    3, 5, 6, 7         5    2   3
    #  4  (10, 9)   7, 8, 9, 10        8    2   2
    # MI = psi(5) + psi(2) - (1/5) sum[psi(n_x+1) + psi(n_y+1)]
    #    = (37/12 - 2 gamma) - (44/15 - 2 gamma) = 9/60 = 0.15
    x = np.array([0, 1, 3, 6, 10], np.float32)
    y = np.array([0, 3, 1, 2, 9], np.float32)
    mi, c = oracle.ksg_rows(x[None], y[None], np.array([[0, 0]], np.int32), 2)
    assert c[0].tolist() == [[1, 2], [2, 2], [1, 3], [2, 3], [2, 2]]
    assert mi[0] == pytest.approx(0.15, abs=1e-14)


@pytest.mark.parametrize("M,expected", [(100, 2.348409263671367), (1000, 4.655502606582091)])
def test_ksg_identical_rows_closed_form(M, expected):
    # x = y without ties: n_x = n_y = k - 1 for every i, MI = psi(M) - psi(k)
    rng = np.random.default_rng(M)
    x = rng.standard_normal(M).astype(np.float32)
    assert np.unique(x).size == M
    mi, c = oracle.ksg_rows(x[None], x[None], np.array([[0, 0]], np.int32), 10)
    assert (c == 9).all()
    assert mi[0] == pytest.approx(expected, abs=1e-13)
    assert expected == pytest.approx(scipy.special.digamma(M) - scipy.special.digamma(10), abs=1e-12)


def test_ksg_symmetry_permutation_and_scaling():
    rng = np.random.default_rng(3)
    M = 100
    x = rng.standard_normal(M).astype(np.float32)
    y = (0.6 * x + 0.8 * rng.standard_normal(M)).astype(np.float32)
    p = np.array([[0, 0]], np.int32)
    mi_xy, c_xy = oracle.ksg_rows(x[None], y[None], p, 10)
    mi_yx, c_yx = oracle.ksg_rows(y[None], x[None], p, 10)
    assert mi_xy[0] == mi_yx[0]
    assert (c_xy[0][:, ::-1] == c_yx[0]).all()
    perm = rng.permutation(M)
    mi_p, c_p = oracle.ksg_rows(x[perm][None], y[perm][None], p, 10)
    assert (c_p[0] == c_xy[0][perm]).all()
    assert mi_p[0] == pytest.approx(mi_xy[0], abs=1e-12)
    for s in (-3, 4):
        f = np.float32(2.0 ** s)
        mi_s, c_s = oracle.ksg_rows((x * f)[None], (y * f)[None], p, 10)
        assert (c_s == c_xy).all() and mi_s[0] == mi_xy[0]


@pytest.mark.parametrize("M,R,rhos,base_tol", [
    (1000, 100, (0.0, 0.5, 0.8, 0.9), 0.02),
    (1000, 100, (0.95,), 0.05),
    (100, 300, (0.0, 0.5, 0.8), 0.05),
])
def test_ksg_bivariate_gaussian_closed_form(M, R, rhos, base_tol):
    # MI of a bivariate normal with correlation rho is -1/2 log(1 - rho^2) nats.
    rng = np.random.default_rng(1234 + M)
    for rho in rhos:
        x = rng.standard_normal((R, M))
        y = rho * x + math.sqrt(1 - rho * rho) * rng.standard_normal((R, M))
        pairs = np.stack([np.arange(R), np.arange(R)], 1).astype(np.int32)
        mi, _ = oracle.ksg_rows(x.astype(np.float32), y.astype(np.float32), pairs, 10, want_counts=False)
        truth = -0.5 * math.log(1 - rho * rho)
        assert abs(mi.mean() - truth) <= base_tol + 4 * mi.std() / math.sqrt(R), (rho, mi.mean(), truth)


def test_ksg_upper_bound_is_attained_only_by_copy():
    # psi(M) - psi(k) bounds the estimate from above when there are no ties.
    rng = np.random.default_rng(9)
    M, n = 100, 200
    z = rng.standard_normal((n, M)).astype(np.float32)
    pairs = rng.integers(0, n, (300, 2)).astype(np.int32)
    mi, _ = oracle.ksg_rows(z, z, pairs, 10, want_counts=False)
    bound = scipy.special.digamma(M) - scipy.special.digamma(10)
    assert (mi <= bound + 1e-12).all()
    same = pairs[:, 0] == pairs[:, 1]
    assert np.allclose(mi[same], bound, atol=1e-12)


def test_ksg_zero_variance_gives_zero():
    data = np.random.default_rng(1).standard_normal((100, 4)).astype(np.float32)
    data[:, 2] = 3.0
    mi, c = oracle.ksg_pairs(data, np.array([[0, 2], [2, 1], [0, 1]], np.int32), 10)
    assert mi[0] == 0.0 and mi[1] == 0.0 and (c[:2] == 0).all()
    assert mi[2] != 0.0


# ---------------------------------------------------------------- standardisation
def test_standardisation_against_numpy():
    e = synth.make_cfg2()
    pts = np.arange(0, e.P, 97, dtype=np.int32)
    mu, s2, mu32, inv32 = oracle.stats(e.data, pts)
    x = e.data[:, pts].astype(np.float64)
    assert np.allclose(mu, x.mean(0), rtol=0, atol=1e-13)
    assert np.allclose(s2, ((x - x.mean(0)) ** 2).sum(0), rtol=1e-12)
    sd = x.std(0)
    assert np.allclose(1.0 / inv32.astype(np.float64), sd, rtol=2e-7)
    z = oracle.ksg_inputs(e.data, pts).astype(np.float64)
    assert np.max(np.abs(z.sum(1))) < 1e-4
    assert np.max(np.abs((z * z).sum(1) - e.M)) < 1e-3


# ---------------------------------------------------------------- region maxima (Sec. 3)
def test_pearson_region_max_brute_force_cfg1():
    e = synth.make_cfg1()
    ia = e.regions[0].global_indices(e.nx, e.ny)
    ib = e.regions[1].global_indices(e.nx, e.ny)
    res = oracle.pearson_region_max(e.data, ia, ib)
    R = np.corrcoef(e.data[:, ia].T.astype(np.float64), e.data[:, ib].T.astype(np.float64))[: ia.size, ia.size:]
    flat = np.abs(R).reshape(-1)
    t = int(np.argmax(flat))  # first maximum in (la, lb) row-major order
    assert res["value"] == pytest.approx(flat[t], abs=1e-12)
    if np.sort(flat)[-2] < flat[t] - 1e-9:
        assert (res["la"], res["lb"]) == divmod(t, ib.size)
    assert res["n_evaluated"] == ia.size * ib.size
    assert res["value"] > 0.6  # the planted rho = 0.8 blobs are found


def test_region_max_planted_copy():
    e = synth.make_cfg1(copy_variant=True)
    p, q = e.copy_pair
    ia = e.regions[0].global_indices(e.nx, e.ny)
    ib = e.regions[1].global_indices(e.nx, e.ny)
    res = oracle.pearson_region_max(e.data, ia, ib)
    assert res["value"] == pytest.approx(1.0, abs=1e-15)
    assert (res["pa"], res["pb"]) == (p, q)
    pairs = np.stack(np.meshgrid(ia, ib, indexing="ij"), -1).reshape(-1, 2).astype(np.int32)
    mi, _ = oracle.ksg_pairs(e.data, pairs, 10, want_counts=False)
    la = np.repeat(np.arange(ia.size), ib.size)
    lb = np.tile(np.arange(ib.size), ia.size)
    best = oracle.region_max_from_values(mi, la, lb, pairs[:, 0], pairs[:, 1], use_abs=False)
    assert best["value"] == pytest.approx(scipy.special.digamma(100) - scipy.special.digamma(10), abs=1e-12)
    assert (best["pa"], best["pb"]) == (p, q)


def test_region_max_tie_break_smallest_local_index():
    vals = np.array([0.5, 0.9, 0.9, -0.9, 0.1])
    la = np.array([3, 2, 1, 1, 0], np.int32)
    lb = np.array([0, 0, 5, 4, 0], np.int32)
    assert oracle.argmax_pairs(vals, la, lb, use_abs=True) == 3  # (1,4) beats (1,5) and (2,0)
    assert oracle.argmax_pairs(vals, la, lb, use_abs=False) == 2


def test_matmul_region_max_agrees_with_brute_force():
    # the FP64 matrix-product route must agree with the plain loop on every case
    for e in (synth.make_cfg1(), synth.make_cfg1(copy_variant=True)):
        ia = e.regions[0].global_indices(e.nx, e.ny)
        ib = e.regions[1].global_indices(e.nx, e.ny)
        a = oracle.pearson_region_max(e.data, ia, ib)
        b = oracle.pearson_region_max_matmul(e.data, ia, ib, block=100)
        assert b["value"] == pytest.approx(a["value"], abs=1e-13)
        assert (b["la"], b["lb"]) == (a["la"], a["lb"])
        assert b["signed_value"] == pytest.approx(a["signed_value"], abs=1e-13)
        assert b["second"] <= b["value"]
    # overlapping regions of one field: the self pair is skipped
    e = synth.make_cfg1()
    ia = e.regions[0].global_indices(e.nx, e.ny)
    a = oracle.pearson_region_max(e.data, ia, ia)
    b = oracle.pearson_region_max_matmul(e.data, ia, ia, block=64)
    assert a["value"] < 1.0 and b["value"] == pytest.approx(a["value"], abs=1e-13)
    assert (b["la"], b["lb"]) == (a["la"], a["lb"])
    assert a["n_evaluated"] == b["n_evaluated"] == ia.size * (ia.size - 1)


# ------------------------------------------------------------ two variables
def test_two_field_paths_match_one_field_construction():
    """Pairs across two fields equal the same pairs inside one field that holds
    both rows (statistics are per point, so the data_b plumbing must give the
    identical result)."""
    import synth as _s
    U, V, regs = _s.make_two_variables(nx=12, ny=8, nz=4, M=40, seed=3)
    rng = np.random.default_rng(4)
    P = U.nx * U.ny * U.nz
    pa = rng.integers(0, P, 64)
    pb = rng.integers(0, P, 64)
    pairs = np.stack([pa, pb], 1).astype(np.int32)
    r2 = oracle.pearson_pairs(U.data, pairs, data_b=V.data)
    mi2, c2 = oracle.ksg_pairs(U.data, pairs, 5, data_b=V.data)
    for t, (a, b) in enumerate(pairs):
        W = U.data.copy()
        W[:, (a + 1) % P] = V.data[:, b]  # V's row placed next to a in one field
        one = np.array([[a, (a + 1) % P]], np.int32)
        assert oracle.pearson_pairs(W, one)[0] == r2[t]
        mi1, c1 = oracle.ksg_pairs(W, one, 5)
        assert mi1[0] == mi2[t] and np.array_equal(c1[0], c2[t])
        x, y = U.data[:, a].astype(np.float64), V.data[:, b].astype(np.float64)
        assert r2[t] == pytest.approx(np.corrcoef(x, y)[0, 1], abs=1e-12)
