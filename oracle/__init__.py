"""CPU oracle for the correlation hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct FP64 references (C with OpenMP in
``oracle.c``, NumPy in ``bos_ref.py``/``mlp_ref.py``) of what the GPU library
computes. Only ``tests/``, the smoke check in ``__graft_entry__`` and the
benchmark's CPU-baseline leg may import this package. It shares no code with
the GPU library and never imports it.

Pins (what fixes the oracle other than itself) live in ``tests/test_oracle_*``:
closed forms (affine copies give r = +-1, identical KSG rows give
psi(M) - psi(k), bivariate Gaussian MI = -1/2 log(1 - rho^2)), library
routines (``numpy.corrcoef``, ``scipy.special.digamma``), a KSG example worked
by hand, and brute-force maxima.

FP16 fields are passed in upcast to float32 (exact).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None

GCC_FLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C, no GPU code)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        L.orc_digamma_int.argtypes = [I]
        L.orc_digamma_int.restype = ctypes.c_double
        L.orc_stats.argtypes = [P, I64, I, P, I64, P, P, P, P]
        L.orc_ksg_inputs.argtypes = [P, I64, I, P, I64, P]
        L.orc_pearson_pairs.argtypes = [P, I64, P, I64, I, P, I64, P]
        L.orc_ksg_pairs.argtypes = [P, P, I64, I, I, P, I64, P, P, P, P]
        L.orc_argmax_pairs.argtypes = [P, P, P, I64, I]
        L.orc_argmax_pairs.restype = I64
        L.orc_pearson_region_max.argtypes = [P, I64, P, I64, P, I64, P, I64, I, I, P, P, P, P, P]
        L.orc_num_threads.restype = I
        L.orc_set_num_threads.argtypes = [I]
        _lib = L
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _f32(data):
    d = np.ascontiguousarray(data)
    if d.dtype != np.float32:
        d = d.astype(np.float32)  # exact for float16
    return d


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of the C oracle (timing only; results do not depend on it)."""
    lib().orc_set_num_threads(int(n))


def digamma_int(n: int) -> float:
    return lib().orc_digamma_int(int(n))


def stats(data, pts=None):
    """Per-point (mu, s2, mu32, inv32) for a member-major (M, P) field."""
    d = _f32(data)
    M, P = d.shape
    pts = np.arange(P, dtype=np.int32) if pts is None else np.ascontiguousarray(pts, dtype=np.int32)
    n = pts.size
    mu, s2 = np.empty(n), np.empty(n)
    mu32, inv32 = np.empty(n, np.float32), np.empty(n, np.float32)
    lib().orc_stats(_p(d), P, M, _p(pts), n, _p(mu), _p(s2), _p(mu32), _p(inv32))
    return mu, s2, mu32, inv32


def ksg_inputs(data, pts):
    """Point-major FP32 z-scored rows (npts, M) of the listed points."""
    d = _f32(data)
    M, P = d.shape
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    z = np.empty((pts.size, M), np.float32)
    lib().orc_ksg_inputs(_p(d), P, M, _p(pts), pts.size, _p(z))
    return z


def pearson_pairs(data_a, pairs, data_b=None):
    """FP64 Pearson r for each (pA, pB) of an int32 (n, 2) pair list."""
    a = _f32(data_a)
    b = a if data_b is None else _f32(data_b)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32)
    r = np.empty(pairs.shape[0])
    lib().orc_pearson_pairs(_p(a), a.shape[1], _p(b), b.shape[1], a.shape[0], _p(pairs), pairs.shape[0], _p(r))
    return r


def ksg_rows(za, zb, pairs, k, zero_a=None, zero_b=None, want_counts=True):
    """KSG MI on point-major sample rows; pairs index rows of za / zb."""
    za = np.ascontiguousarray(za, dtype=np.float32)
    zb = np.ascontiguousarray(zb, dtype=np.float32)
    assert za.shape[1] == zb.shape[1]
    M = za.shape[1]
    if not (1 <= k <= M - 1):
        raise ValueError("k out of range")
    pairs = np.ascontiguousarray(pairs, dtype=np.int32)
    n = pairs.shape[0]
    mi = np.empty(n)
    counts = np.empty((n, M, 2), np.int32) if want_counts else None
    za8 = None if zero_a is None else np.ascontiguousarray(zero_a, dtype=np.uint8)
    zb8 = None if zero_b is None else np.ascontiguousarray(zero_b, dtype=np.uint8)
    lib().orc_ksg_pairs(_p(za), _p(zb), M, M, int(k), _p(pairs), n, _p(za8), _p(zb8), _p(mi), _p(counts))
    return mi, counts


def ksg_pairs(data_a, pairs, k, data_b=None, raw=False, want_counts=True):
    """KSG MI for (pA, pB) global index pairs of member-major fields.

    Standardises every referenced point (z = fl32(fl32(x - mu32) * inv32)),
    unless ``raw`` (then the FP32 values are used as they are).
    """
    a = _f32(data_a)
    b = a if data_b is None else _f32(data_b)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32)
    ua, ia = np.unique(pairs[:, 0], return_inverse=True)
    ub, ib = np.unique(pairs[:, 1], return_inverse=True)
    if raw:
        za = np.ascontiguousarray(a[:, ua].T)
        zb = np.ascontiguousarray(b[:, ub].T)
        zero_a = zero_b = None
    else:
        za = ksg_inputs(a, ua)
        zb = ksg_inputs(b, ub)
        zero_a = stats(a, ua)[1] <= 0.0
        zero_b = stats(b, ub)[1] <= 0.0
    local = np.ascontiguousarray(np.stack([ia, ib], 1).astype(np.int32))
    return ksg_rows(za, zb, local, k, zero_a, zero_b, want_counts)


def argmax_pairs(values, la, lb, use_abs):
    values = np.ascontiguousarray(values, dtype=np.float64)
    la = np.ascontiguousarray(la, dtype=np.int32)
    lb = np.ascontiguousarray(lb, dtype=np.int32)
    return int(lib().orc_argmax_pairs(_p(values), _p(la), _p(lb), values.size, int(use_abs)))


def pearson_region_max(data_a, idx_a, idx_b, data_b=None, same_field=None):
    """Exhaustive max |r| over region A x region B (global index lists in local order).

    Returns dict(value, signed_value, la, lb, pa, pb, n_evaluated).
    """
    a = _f32(data_a)
    b = a if data_b is None else _f32(data_b)
    if same_field is None:
        same_field = data_b is None or data_b is data_a
    ia = np.ascontiguousarray(idx_a, dtype=np.int32)
    ib = np.ascontiguousarray(idx_b, dtype=np.int32)
    v, s = ctypes.c_double(), ctypes.c_double()
    la, lb, ne = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    lib().orc_pearson_region_max(_p(a), a.shape[1], _p(ia), ia.size, _p(b), b.shape[1], _p(ib), ib.size,
                                 a.shape[0], int(bool(same_field)), ctypes.byref(v), ctypes.byref(s),
                                 ctypes.byref(la), ctypes.byref(lb), ctypes.byref(ne))
    return dict(value=v.value, signed_value=s.value, la=la.value, lb=lb.value,
                pa=int(ia[la.value]), pb=int(ib[lb.value]), n_evaluated=ne.value)


def region_max_from_values(values, la, lb, pa, pb, use_abs=True):
    """Region maximum over a list of evaluated pairs (MI or r) with the tie rule."""
    t = argmax_pairs(values, la, lb, use_abs)
    v = float(values[t])
    return dict(value=abs(v) if use_abs else v, signed_value=v, la=int(la[t]), lb=int(lb[t]),
                pa=int(pa[t]), pb=int(pb[t]), index=t)


def _zrows64(data, idx):
    """FP64 rows (len(idx), M) of (x - mean) / sqrt(sum (x - mean)^2); zero for constant points."""
    x = np.asarray(data[:, idx], dtype=np.float64).T
    x = x - x.mean(axis=1, keepdims=True)
    q = np.sqrt((x * x).sum(axis=1, keepdims=True))
    with np.errstate(invalid="ignore", divide="ignore"):
        z = np.where(q > 0, x / np.where(q > 0, q, 1.0), 0.0)
    return z


def pearson_region_max_matmul(data_a, idx_a, idx_b, data_b=None, same_field=None, block=1024):
    """Exhaustive max |r| over region A x region B with FP64 matrix products.

    Same definition and tie rule as ``pearson_region_max`` (Sec. 3.2 Pearson,
    Sec. 3 maximum over the brick pair); the matrix product of the z-scored
    FP64 rows is the only library step. Also returns ``second``: the largest
    |r| over all other pairs (the top-2 gap decides whether an argmax is
    unique within a tolerance).
    """
    b_data = data_a if data_b is None else data_b
    if same_field is None:
        same_field = data_b is None or data_b is data_a
    ia = np.asarray(idx_a, dtype=np.int64)
    ib = np.asarray(idx_b, dtype=np.int64)
    za = _zrows64(data_a, ia)
    zb = _zrows64(b_data, ib)
    pos_b = {int(p): j for j, p in enumerate(ib)} if same_field else {}
    best = (-1.0, 0.0, -1, -1)
    second = -1.0
    for r0 in range(0, ia.size, block):
        R = za[r0:r0 + block] @ zb.T
        A = np.abs(R)
        if same_field:
            for i in range(A.shape[0]):
                j = pos_b.get(int(ia[r0 + i]))
                if j is not None:
                    A[i, j] = -1.0
        flat = A.reshape(-1)
        t = int(np.argmax(flat))
        v = float(flat[t])
        top2 = np.partition(flat, flat.size - 2)[-2:] if flat.size > 1 else np.array([-1.0, v])
        blk_second = float(top2[0])
        if v > best[0]:
            second = max(second, best[0], blk_second)
            i, j = divmod(t, A.shape[1])
            best = (v, float(R[i, j]), r0 + i, j)
        else:
            second = max(second, v)
    v, s, la, lb = best
    return dict(value=v, signed_value=s, la=la, lb=lb, pa=int(ia[la]) if la >= 0 else -1,
                pb=int(ib[lb]) if lb >= 0 else -1, second=second,
                n_evaluated=ia.size * ib.size - (len(set(ia.tolist()) & set(ib.tolist())) if same_field else 0))
