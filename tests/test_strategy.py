"""The library's strategy rule (corr_choose_strategy, Sec. 5 sampling
strategy) against the oracle's, on the thresholds and on random inputs; host
code only, no GPU."""
import numpy as np
import pytest

from oracle import sampling_ref as SR


@pytest.fixture(scope="module")
def pc():
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as m
    return m


def test_strategy_matches_oracle(pc):
    names = {SR.BOS: "bos", SR.RANDOM: "random", SR.EXHAUSTIVE: "exhaustive"}
    cases = [(20480, 20480, 4.5e12), (4096, 4096, 1.0), (4095, 4096, 1e12), (4095, 4096, 2e6), (1000, 1000, 2e5),
             (1000, 1001, 2e5), (1, 1, 1e-9)]
    rng = np.random.default_rng(0)
    for _ in range(500):
        cases.append((int(rng.integers(1, 9000)), int(rng.integers(1, 9000)), float(10 ** rng.uniform(3, 9))))
    for na, nb, rate in cases:
        assert pc.choose_strategy(na, nb, rate) == names[SR.choose_strategy(na, nb, rate)], (na, nb, rate)


def test_strategy_bad_arguments(pc):
    for args in ((0, 5, 1e6), (5, 5, 0.0), (5, 5, -1.0)):
        with pytest.raises(pc.CorrError) as ei:
            pc.choose_strategy(*args)
        assert ei.value.status == 1
