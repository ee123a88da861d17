"""Validity of a returned region-maximum argmax, for use where several
answers are correct (the oracle's top two values lie within twice the
tolerance, so either may come back): the pair must lie in A x B, must not be
a point with itself inside one field, and the oracle's own value at that pair
must equal the returned value (and, for Pearson, the returned sign) within
the tolerance. Where the top-2 gap exceeds twice the tolerance the argmax is
unique and must equal the oracle's exactly."""
import numpy as np

import oracle


def check_pearson_argmax(got, ref, data_a, ia, ib, tol, data_b=None, same_field=True):
    pa, pb = int(got["pa"]), int(got["pb"])
    assert pa in set(int(v) for v in ia) and pb in set(int(v) for v in ib), (pa, pb)
    if same_field and data_b is None:
        assert pa != pb, "a point paired with itself"
    r = float(oracle.pearson_pairs(data_a, np.array([[pa, pb]], np.int32), data_b=data_b)[0])
    assert abs(abs(r) - got["value"]) <= tol, (got, r)
    assert abs(got["signed_value"] - r) <= tol, (got, r)
    if abs(r) > tol:
        assert np.sign(got["signed_value"]) == np.sign(r)
    if ref is not None and ref["value"] - ref["second"] > 2 * tol:
        assert (pa, pb) == (ref["pa"], ref["pb"])


def check_ksg_argmax(got, data_a, ia, ib, k, tol, data_b=None, same_field=True, unique_ref=None):
    pa, pb = int(got["pa"]), int(got["pb"])
    assert pa in set(int(v) for v in ia) and pb in set(int(v) for v in ib), (pa, pb)
    if same_field and data_b is None:
        assert pa != pb, "a point paired with itself"
    mi, _ = oracle.ksg_pairs(data_a, np.array([[pa, pb]], np.int32), k, data_b=data_b, want_counts=False)
    assert abs(float(mi[0]) - got["value"]) <= tol, (got, mi)
    if unique_ref is not None:
        assert (pa, pb) == (unique_ref["pa"], unique_ref["pb"])
