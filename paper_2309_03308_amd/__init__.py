"""MI355X-native correlation hot path for focus+context views of 3D ensembles
(arXiv 2309.03308): Pearson and Kraskov mutual information between grid points
of two regions across ensemble members, reduced to region-pair maxima.

Python names mirror the C entry points of include/corr.h. Tensors are
torch CUDA(HIP) tensors; the library's kernels do all of the work.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import CorrError, corr_field, corr_max, corr_region, PREC, MEASURE  # noqa: F401


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Field:
    """A member-major ensemble field (M, nx*ny*nz) resident on the GPU."""

    def __init__(self, data, nx: int, ny: int, nz: int):
        torch = _torch()
        if not data.is_cuda:
            raise ValueError("field data must be a device tensor")
        if data.dtype not in (torch.float32, torch.float16):
            raise ValueError("field dtype must be float32 or float16")
        if data.dim() != 2 or data.shape[1] < nx * ny * nz:
            raise ValueError("field data must be (M, >= nx*ny*nz)")
        if data.stride(1) != 1:
            raise ValueError("field rows must be contiguous")
        self.data = data
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.c = corr_field(ctypes.c_void_p(data.data_ptr()), _lib.CORR_F32 if data.dtype == torch.float32 else _lib.CORR_F16,
                            int(data.shape[0]), self.nx, self.ny, self.nz, int(data.stride(0)))

    @property
    def M(self):
        return int(self.data.shape[0])

    @property
    def P(self):
        return self.nx * self.ny * self.nz


def region(x0, y0, z0, dx, dy, dz) -> corr_region:
    return corr_region(int(x0), int(y0), int(z0), int(dx), int(dy), int(dz))


def _pairs_arg(pairs):
    torch = _torch()
    if pairs.dtype != torch.int32 or not pairs.is_cuda or pairs.dim() != 2 or pairs.shape[1] != 2 or not pairs.is_contiguous():
        raise ValueError("pairs must be a contiguous int32 (n, 2) device tensor")
    return ctypes.c_void_p(pairs.data_ptr()), int(pairs.shape[0])


class Context:
    """Owns a corr_ctx (device workspaces, digamma table)."""

    def __init__(self, device: int = 0):
        self.L = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(self.L.corr_create(int(device), ctypes.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.L.corr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ timing
    KERNEL_CLASSES = {"gemm": 0, "ksg": 1, "pairs": 2, "standardize": 3}

    def set_timing(self, on: bool = True):
        _lib.check(self.L.corr_set_timing(self.h, 1 if on else 0))

    def kernel_time_ms(self, which: str) -> float:
        ms = ctypes.c_float()
        _lib.check(self.L.corr_kernel_time_ms(self.h, self.KERNEL_CLASSES[which], ctypes.byref(ms)))
        return float(ms.value)

    # ------------------------------------------------------------------ tuning
    def corr_autotune(self, A: Field, ra: corr_region, rb: corr_region, prec="f16", reps=5, B: Field = None,
                      stream=None):
        B = A if B is None else B
        cfg, ms = ctypes.c_int(), ctypes.c_float()
        _lib.check(self.L.corr_autotune(self.h, ctypes.byref(A.c), ctypes.byref(ra), ctypes.byref(B.c),
                                        ctypes.byref(rb), PREC[prec], int(reps), ctypes.byref(cfg), ctypes.byref(ms),
                                        _stream_ptr(stream)))
        return int(cfg.value), float(ms.value)

    def corr_ksg_autotune(self, A: Field, pairs, k=10, reps=3, B: Field = None, stream=None):
        B = A if B is None else B
        pp, n = _pairs_arg(pairs)
        pw, ms = ctypes.c_int(), ctypes.c_float()
        _lib.check(self.L.corr_ksg_autotune(self.h, ctypes.byref(A.c), ctypes.byref(B.c), pp, n, int(k), int(reps),
                                            ctypes.byref(pw), ctypes.byref(ms), _stream_ptr(stream)))
        return int(pw.value), float(ms.value)

    def corr_tune_save(self, path: str):
        _lib.check(self.L.corr_tune_save(self.h, path.encode()))

    def corr_tune_load(self, path: str):
        _lib.check(self.L.corr_tune_load(self.h, path.encode()))

    # ------------------------------------------------------------------ calls
    def corr_standardize(self, A: Field, stream=None):
        torch = _torch()
        n = A.P
        mu = torch.empty(n, dtype=torch.float32, device=A.data.device)
        inv = torch.empty_like(mu)
        sig = torch.empty_like(mu)
        _lib.check(self.L.corr_standardize(self.h, ctypes.byref(A.c), ctypes.c_void_p(mu.data_ptr()),
                                           ctypes.c_void_p(inv.data_ptr()), ctypes.c_void_p(sig.data_ptr()),
                                           _stream_ptr(stream)))
        return mu, inv, sig

    def corr_pearson_pairs(self, A: Field, pairs, prec="f32", B: Field = None, out=None, stream=None):
        torch = _torch()
        B = A if B is None else B
        pp, n = _pairs_arg(pairs)
        r = torch.empty(n, dtype=torch.float32, device=pairs.device) if out is None else out
        _lib.check(self.L.corr_pearson_pairs(self.h, ctypes.byref(A.c), ctypes.byref(B.c), pp, n, PREC[prec],
                                             ctypes.c_void_p(r.data_ptr()), _stream_ptr(stream)))
        return r

    def corr_ksg_mi_pairs(self, A: Field, pairs, k=10, B: Field = None, raw=False, counts=False, out=None,
                          stream=None):
        torch = _torch()
        B = A if B is None else B
        pp, n = _pairs_arg(pairs)
        mi = torch.empty(n, dtype=torch.float32, device=pairs.device) if out is None else out
        cnt = torch.empty((n, A.M, 2), dtype=torch.int32, device=pairs.device) if counts else None
        _lib.check(self.L.corr_ksg_mi_pairs(self.h, ctypes.byref(A.c), ctypes.byref(B.c), pp, n, int(k),
                                            _lib.CORR_KSG_RAW if raw else 0, ctypes.c_void_p(mi.data_ptr()),
                                            ctypes.c_void_p(cnt.data_ptr()) if counts else None,
                                            _stream_ptr(stream)))
        return (mi, cnt) if counts else mi

    def corr_region_max(self, A: Field, ra: corr_region, rb: corr_region, measure="pearson", prec="f16", k=10,
                        B: Field = None, samples=None, stream=None) -> dict:
        B = A if B is None else B
        out = corr_max()
        if samples is None:
            sp, ns = None, 0
        else:
            sp, ns = _pairs_arg(samples)
        _lib.check(self.L.corr_region_max(self.h, ctypes.byref(A.c), ctypes.byref(ra), ctypes.byref(B.c),
                                          ctypes.byref(rb), MEASURE[measure], PREC[prec], int(k), sp, ns,
                                          ctypes.byref(out), _stream_ptr(stream)))
        return dict(value=out.value, signed_value=out.signed_value, pa=out.pa, pb=out.pb,
                    n_evaluated=out.n_evaluated)


def version() -> str:
    return _lib.load().corr_version().decode()
