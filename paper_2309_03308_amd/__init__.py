"""MI355X-native correlation hot path for focus+context views of 3D ensembles
(arXiv 2309.03308): Pearson and Kraskov mutual information between grid points
of two regions across ensemble members, reduced to region-pair maxima.

Python names mirror the C entry points of include/corr.h. Tensors are
torch CUDA(HIP) tensors; the library's kernels do all of the work.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import CorrError, bos_config, corr_field, corr_max, corr_region, PREC, MEASURE, SAMPLER, STRATEGY  # noqa: F401


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
    KERNEL_CLASSES = {"gemm": 0, "ksg": 1, "pairs": 2, "standardize": 3, "block_means": 4}

    def set_timing(self, on: bool = True):
        _lib.check(self.L.corr_set_timing(self.h, 1 if on else 0))

    def set_workspace_limit(self, nbytes: int):
        """Cap the context's workspace memory (0: no cap); calls that need more return CORR_ENOMEM."""
        _lib.check(self.L.corr_set_workspace_limit(self.h, int(nbytes)))

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

    def corr_prepare(self, A: Field, measure="pearson", prec="f16", stream=None) -> "Prepared":
        """Standardise A once for many pair-list calls (include/corr.h corr_prepare)."""
        h = ctypes.c_void_p()
        _lib.check(self.L.corr_prepare(self.h, ctypes.byref(A.c), MEASURE[measure], PREC[prec], ctypes.byref(h),
                                       _stream_ptr(stream)))
        return Prepared(self, h, A, measure, prec)

    def corr_pearson_pairs_prepared(self, A: "Prepared", pairs, B: "Prepared" = None, out=None, stream=None):
        torch = _torch()
        B = A if B is None else B
        pp, n = _pairs_arg(pairs)
        r = out if out is not None else torch.empty(n, dtype=torch.float32, device=pairs.device)
        _lib.check(self.L.corr_pearson_pairs_prepared(self.h, A.h, B.h, pp, n, ctypes.c_void_p(r.data_ptr()),
                                                      _stream_ptr(stream)))
        return r

    def corr_ksg_mi_pairs_prepared(self, A: "Prepared", pairs, k=10, B: "Prepared" = None, counts=False, out=None,
                                   stream=None):
        torch = _torch()
        B = A if B is None else B
        pp, n = _pairs_arg(pairs)
        mi = out if out is not None else torch.empty(n, dtype=torch.float32, device=pairs.device)
        cnt = torch.empty((n, A.field.M, 2), dtype=torch.int32, device=pairs.device) if counts else None
        _lib.check(self.L.corr_ksg_mi_pairs_prepared(self.h, A.h, B.h, pp, n, int(k), ctypes.c_void_p(mi.data_ptr()),
                                                     ctypes.c_void_p(cnt.data_ptr()) if counts else None,
                                                     _stream_ptr(stream)))
        return (mi, cnt) if counts else mi

    def corr_box_pairs_max(self, A: "Prepared", boxes_a, boxes_b, B: "Prepared" = None, stream=None) -> list:
        """Exhaustive max |r| of many small box pairs (fields prepared with pearson / f32)."""
        B = A if B is None else B
        n = len(boxes_a)
        if len(boxes_b) != n:
            raise ValueError("boxes_a and boxes_b differ in length")
        ba = (corr_region * max(n, 1))(*[b if isinstance(b, corr_region) else region(*b) for b in boxes_a])
        bb = (corr_region * max(n, 1))(*[b if isinstance(b, corr_region) else region(*b) for b in boxes_b])
        out = (corr_max * max(n, 1))()
        _lib.check(self.L.corr_box_pairs_max(self.h, A.h, B.h, ba, bb, n, out, _stream_ptr(stream)))
        return [dict(value=o.value, signed_value=o.signed_value, pa=o.pa, pb=o.pb, n_evaluated=o.n_evaluated)
                for o in out[:n]]

    def corr_region_max(self, A: Field, ra: corr_region, rb: corr_region, measure="pearson", prec="f16", k=10,
                        B: Field = None, samples=None, stream=None) -> dict:
        return self._region_max(self.L.corr_region_max, A, ra, rb, measure, prec, k, B, samples, stream)

    def corr_region_max_noalloc(self, A: Field, ra: corr_region, rb: corr_region, measure="pearson", prec="f16",
                                k=10, B: Field = None, samples=None, stream=None) -> dict:
        """corr_region_max with the library's fixed per-GPU scratch (no device allocation)."""
        return self._region_max(self.L.corr_region_max_noalloc, A, ra, rb, measure, prec, k, B, samples, stream)

    def _region_max(self, fn, A, ra, rb, measure, prec, k, B, samples, stream) -> dict:
        B = A if B is None else B
        out = corr_max()
        if samples is None:
            sp, ns = None, 0
        else:
            sp, ns = _pairs_arg(samples)
        _lib.check(fn(self.h, ctypes.byref(A.c), ctypes.byref(ra), ctypes.byref(B.c), ctypes.byref(rb),
                      MEASURE[measure], PREC[prec], int(k), sp, ns, ctypes.byref(out), _stream_ptr(stream)))
        return dict(value=out.value, signed_value=out.signed_value, pa=out.pa, pb=out.pb,
                    n_evaluated=out.n_evaluated)

    def corr_region_submax(self, A: Field, ra: corr_region, rb: corr_region, splits_a=(2, 2, 2), splits_b=(2, 2, 2),
                           prec="f16", B: Field = None, stream=None):
        """Exhaustive Pearson maxima of every (sub-brick of ra, sub-brick of rb):
        a list of lists of corr_region_max-style dicts, [i][j], sub-bricks x-fastest."""
        B = A if B is None else B
        sa = (ctypes.c_int32 * 3)(*[int(v) for v in splits_a])
        sb = (ctypes.c_int32 * 3)(*[int(v) for v in splits_b])
        na, nb = int(np.prod(splits_a)), int(np.prod(splits_b))
        res = (corr_max * max(1, na * nb))()  # the library rejects bad splits before writing
        _lib.check(self.L.corr_region_submax(self.h, ctypes.byref(A.c), ctypes.byref(ra), ctypes.cast(sa, ctypes.c_void_p),
                                             ctypes.byref(B.c), ctypes.byref(rb), ctypes.cast(sb, ctypes.c_void_p),
                                             PREC[prec], ctypes.cast(res, ctypes.c_void_p), _stream_ptr(stream)))
        return [[dict(value=r.value, signed_value=r.signed_value, pa=r.pa, pb=r.pb, n_evaluated=r.n_evaluated)
                 for r in res[i * nb:(i + 1) * nb]] for i in range(na)]

    # ------------------------------------------------------------------ sampling
    @staticmethod
    def _region_arrays(regions, region_pairs):
        regs = [region(*r) if isinstance(r, tuple) else r for r in regions]
        ra = (corr_region * max(1, len(regs)))(*regs)
        rp = np.ascontiguousarray(np.asarray(region_pairs, dtype=np.int32).reshape(-1, 2))
        return ra, len(regs), rp

    def corr_sample_pairs(self, A: Field, regions, region_pairs, sampler="uniform", n=100, seed=0, B: Field = None,
                          stream=None):
        """Sample point pairs of brick pairs: device int32 (n_pairs, n, 2) global indices."""
        torch = _torch()
        B = A if B is None else B
        ra, nr, rp = self._region_arrays(regions, region_pairs)
        out = torch.empty((rp.shape[0], int(n), 2), dtype=torch.int32, device=A.data.device)
        _lib.check(self.L.corr_sample_pairs(self.h, ctypes.byref(A.c), ctypes.byref(B.c), ctypes.cast(ra, ctypes.c_void_p),
                                            nr, rp.ctypes.data_as(ctypes.c_void_p), rp.shape[0], SAMPLER[sampler],
                                            int(n), int(seed) & (2 ** 64 - 1), ctypes.c_void_p(out.data_ptr()),
                                            _stream_ptr(stream)))
        return out

    def corr_sampled_max(self, A: Field, regions, region_pairs, measure="pearson", prec="f32", k=10,
                         sampler="uniform", n=100, seed=0, B: Field = None, stream=None):
        """Sampled maxima of many brick pairs: a list of dicts like corr_region_max's."""
        B = A if B is None else B
        ra, nr, rp = self._region_arrays(regions, region_pairs)
        res = (corr_max * max(1, rp.shape[0]))()
        _lib.check(self.L.corr_sampled_max(self.h, ctypes.byref(A.c), ctypes.byref(B.c), ctypes.cast(ra, ctypes.c_void_p),
                                           nr, rp.ctypes.data_as(ctypes.c_void_p), rp.shape[0], MEASURE[measure],
                                           PREC[prec], int(k), SAMPLER[sampler], int(n), int(seed) & (2 ** 64 - 1),
                                           ctypes.cast(res, ctypes.c_void_p), _stream_ptr(stream)))
        return [dict(value=r.value, signed_value=r.signed_value, pa=r.pa, pb=r.pb, n_evaluated=r.n_evaluated)
                for r in res[:rp.shape[0]]]

    # ------------------------------------------------------------------ mean tree
    def corr_block_means(self, A: Field, f: int, dtype="f32", out=None, stream=None) -> Field:
        """One mean-tree level: the field of f^3 block means (a new Field, or one over `out`)."""
        torch = _torch()
        if int(f) < 1:  # the library reports the bad factor before anything is sized
            _lib.check(self.L.corr_block_means(self.h, ctypes.byref(A.c), int(f), 0, None, 0, _stream_ptr(stream)))
        NX, NY, NZ = level_dims(A.nx, A.ny, A.nz, f)
        tdt = {"f32": torch.float32, "f16": torch.float16}[dtype]
        if out is None:
            out = torch.empty((A.M, NX * NY * NZ), dtype=tdt, device=A.data.device)
        elif out.dtype != tdt or out.dim() != 2 or out.shape[0] != A.M or out.shape[1] < NX * NY * NZ \
                or out.stride(1) != 1:
            raise ValueError("out must be a (M, >= level points) tensor of the requested dtype")
        _lib.check(self.L.corr_block_means(self.h, ctypes.byref(A.c), int(f),
                                           _lib.CORR_F32 if dtype == "f32" else _lib.CORR_F16,
                                           ctypes.c_void_p(out.data_ptr()), int(out.stride(0)), _stream_ptr(stream)))
        return Field(out, NX, NY, NZ)

    def mean_tree(self, A: Field, factors=(2, 4), dtype="f32", stream=None) -> dict:
        """Levels of the mean tree, each computed from the initial data: {f: Field}."""
        return {int(f): self.corr_block_means(A, f, dtype, stream=stream) for f in factors}


# Exhaustive evaluation rates used by choose_strategy when the caller gives
# none (point pairs per second on one MI355X, measured at M = 100 and scaled
# with the work per pair: M for Pearson, M^2 for KSG).
EXHAUSTIVE_RATE_M100 = {"pearson": 4.5e12, "ksg": 2.2e8}


def exhaustive_rate(measure: str, M: int) -> float:
    r = EXHAUSTIVE_RATE_M100[measure]
    return r * (100.0 / M) if measure == "pearson" else r * (100.0 / M) ** 2


def choose_strategy(na: int, nb: int, pairs_per_s: float, budget_s: float = 5.0) -> str:
    """"bos", "random" or "exhaustive" for bricks of na and nb points (Sec. 5)."""
    st = ctypes.c_int32()
    _lib.check(_lib.load().corr_choose_strategy(int(na), int(nb), float(pairs_per_s), float(budget_s),
                                                ctypes.byref(st)))
    return STRATEGY[st.value]


def brick_max(ctx: Context, A: Field, ra: corr_region, rb: corr_region, measure="pearson", prec="f16x3", k=10,
              budget_s=5.0, n_samples=100, seed=0, pairs_per_s=None, B: Field = None, bos_cfg=None):
    """The maximum of one brick pair by the strategy of Sec. 5: BOS for bricks of
    at least 16^3 points, else every point pair when that fits the time budget,
    else uniform random sampling. Returns (strategy, corr_region_max-style dict)."""
    B = A if B is None else B
    na, nb = ra.dx * ra.dy * ra.dz, rb.dx * rb.dy * rb.dz
    rate = exhaustive_rate(measure, A.M) if pairs_per_s is None else pairs_per_s
    st = choose_strategy(na, nb, rate, budget_s)
    if st == "exhaustive":
        return st, ctx.corr_region_max(A, ra, rb, measure, prec, k, B=B)
    if st == "random":
        return st, ctx.corr_sampled_max(A, [ra, rb], [(0, 1)], measure, prec, k, "uniform", n_samples, seed, B=B)[0]
    bos = Bos(ctx, A, [ra, rb], [(0, 1)], bos_cfg if bos_cfg is not None else bos_defaults(measure=measure, k=k), B=B)
    try:
        bos.bos_run()
        return st, bos.bos_results()[0]
    finally:
        bos.close()


def level_dims(nx, ny, nz, f):
    """Grid extent of the mean-tree level with factor f."""
    return ((nx + f - 1) // f, (ny + f - 1) // f, (nz + f - 1) // f)


def region_at_level(r: corr_region, f: int) -> corr_region:
    """The level-f blocks that cover a brick (exact for bricks aligned to f)."""
    x1, y1, z1 = r.x0 + r.dx, r.y0 + r.dy, r.z0 + r.dz
    x0, y0, z0 = r.x0 // f, r.y0 // f, r.z0 // f
    return corr_region(x0, y0, z0, (x1 + f - 1) // f - x0, (y1 + f - 1) // f - y0, (z1 + f - 1) // f - z0)


def bos_defaults(**overrides) -> bos_config:
    """bos_config with the library defaults, then the given fields."""
    c = bos_config()
    _lib.load().bos_config_default(ctypes.byref(c))
    for k, v in overrides.items():
        if k == "measure" and isinstance(v, str):
            v = MEASURE[v]
        setattr(c, k, v)
    return c


class Prepared:
    """A field standardised once (include/corr.h corr_prepare); owns its device buffers."""

    def __init__(self, ctx, h, field, measure, prec):
        self.ctx, self.h, self.field, self.measure, self.prec = ctx, h, field, measure, prec

    def close(self):
        if getattr(self, "h", None):
            self.ctx.L.corr_prepared_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Bos:
    """Batched Bayesian optimal sampling of region-pair maxima (include/bos.h)."""

    def __init__(self, ctx: Context, A: Field, regions, region_pairs, cfg: bos_config = None, B: Field = None,
                 stream=None):
        import numpy as np
        self.ctx, self.A = ctx, A
        self.B = A if B is None else B
        self.L = ctx.L
        cfg = bos_defaults() if cfg is None else cfg
        self.cfg = cfg
        regs = (corr_region * len(regions))(*[r if isinstance(r, corr_region) else region(*r) for r in regions])
        self._regs = regs
        rp = np.ascontiguousarray(np.asarray(region_pairs, dtype=np.int32).reshape(-1, 2))
        self.n_pairs = rp.shape[0]
        self.region_pairs = rp
        h = ctypes.c_void_p()
        _lib.check(self.L.bos_create(ctx.h, ctypes.byref(A.c), ctypes.byref(self.B.c), regs, len(regions),
                                     ctypes.c_void_p(rp.ctypes.data), self.n_pairs, ctypes.byref(cfg),
                                     ctypes.byref(h), _stream_ptr(stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.bos_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bos_set_launch(self, mode="graph", timeout_s=300.0):
        """Launch iterations through a captured HIP graph or directly; bound every wait."""
        _lib.check(self.L.bos_set_launch(self.h, _lib.BOS_LAUNCH[mode], float(timeout_s)))

    def bos_set_prior(self, cells):
        import numpy as np
        c = np.ascontiguousarray(np.asarray(cells, dtype=np.float32).reshape(self.n_pairs, 6))
        _lib.check(self.L.bos_set_prior(self.h, ctypes.c_void_p(c.ctypes.data)))

    def bos_sample_step(self, stream=None) -> int:
        n = ctypes.c_int32()
        _lib.check(self.L.bos_sample_step(self.h, _stream_ptr(stream), ctypes.byref(n)))
        return int(n.value)

    def bos_run(self, stream=None):
        _lib.check(self.L.bos_run(self.h, _stream_ptr(stream)))

    def bos_results(self, stream=None):
        out = (corr_max * self.n_pairs)()
        _lib.check(self.L.bos_results(self.h, out, _stream_ptr(stream)))
        return [dict(value=o.value, signed_value=o.signed_value, pa=o.pa, pb=o.pb, n_evaluated=o.n_evaluated)
                for o in out]

    def bos_history(self, pair: int, stream=None):
        import numpy as np
        nt = self.cfg.n_total
        cells = np.zeros((nt, 6), np.int32)
        vals = np.zeros(nt, np.float32)
        n = ctypes.c_int32()
        _lib.check(self.L.bos_history(self.h, int(pair), ctypes.c_void_p(cells.ctypes.data),
                                      ctypes.c_void_p(vals.ctypes.data), ctypes.byref(n), _stream_ptr(stream)))
        return cells[: n.value].copy(), vals[: n.value].copy()

    def bos_schedule(self):
        """Per pair, the batch sizes drawn from the seed: a list of lists."""
        import numpy as np
        sched = np.zeros((self.n_pairs, 16), np.int32)
        nb = np.zeros(self.n_pairs, np.int32)
        _lib.check(self.L.bos_schedule(self.h, ctypes.c_void_p(sched.ctypes.data), ctypes.c_void_p(nb.ctypes.data)))
        return [list(sched[p, : nb[p]]) for p in range(self.n_pairs)]

    def bos_save(self, path: str, stream=None):
        _lib.check(self.L.bos_save(self.h, path.encode(), _stream_ptr(stream)))

    def bos_load(self, path: str, stream=None):
        _lib.check(self.L.bos_load(self.h, path.encode(), _stream_ptr(stream)))


class PropMlp:
    """Learned BOS proposal network (include/mlp.h)."""

    def __init__(self, ctx: Context, n_in: int = 42, n_hidden: int = 256, n_out: int = 8, seed: int = 1):
        self.ctx, self.L = ctx, ctx.L
        self.n_in, self.n_hidden, self.n_out = n_in, n_hidden, n_out
        h = ctypes.c_void_p()
        _lib.check(self.L.prop_mlp_create(ctx.h, n_in, n_hidden, n_out, ctypes.c_uint64(seed), ctypes.byref(h)))
        self.h = h
        n = ctypes.c_int64()
        _lib.check(self.L.prop_mlp_num_params(self.h, ctypes.byref(n)))
        self.n_params = int(n.value)

    def close(self):
        if getattr(self, "h", None):
            self.L.prop_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np
        out = np.zeros(self.n_params, np.float32)
        _lib.check(self.L.prop_mlp_get_params(self.h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, np.float32).reshape(self.n_params))
        _lib.check(self.L.prop_mlp_set_params(self.h, ctypes.c_void_p(p.ctypes.data)))

    def get_grads(self):
        import numpy as np
        out = np.zeros(self.n_params, np.float32)
        _lib.check(self.L.prop_mlp_get_grads(self.h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def forward(self, x, out=None, stream=None):
        torch = _torch()
        x = x.contiguous()
        if x.dtype != torch.float32 or not x.is_cuda or x.dim() != 2 or x.shape[1] != self.n_in:
            raise ValueError("x must be a float32 device tensor (B, n_in)")
        y = out if out is not None else torch.empty(x.shape[0], self.n_out, device=x.device, dtype=torch.float32)
        _lib.check(self.L.prop_mlp_forward(self.h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                           ctypes.c_void_p(y.data_ptr()), _stream_ptr(stream)))
        return y

    def train_step(self, x, target, lr=1e-3, wd=1e-4, loss_w=None, stream=None) -> float:
        import numpy as np
        torch = _torch()
        x, target = x.contiguous(), target.contiguous()
        if x.dtype != torch.float32 or target.dtype != torch.float32 or not x.is_cuda or not target.is_cuda:
            raise ValueError("x and target must be float32 device tensors")
        if x.dim() != 2 or x.shape[1] != self.n_in or tuple(target.shape) != (x.shape[0], self.n_out):
            raise ValueError("x (B, n_in) and target (B, n_out) expected")
        wp = None
        if loss_w is not None:
            w = np.ascontiguousarray(np.asarray(loss_w, np.float32).reshape(self.n_out))
            wp = ctypes.c_void_p(w.ctypes.data)
        loss = ctypes.c_float()
        _lib.check(self.L.prop_mlp_train_step(self.h, ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(target.data_ptr()), wp, x.shape[0], float(lr),
                                              float(wd), ctypes.byref(loss), _stream_ptr(stream)))
        return float(loss.value)


def corr_proposal_inputs(ctx: Context, A: Field, regions, region_pairs, n_hot: int = 4, D: int = 1, r_nms: int = 3,
                         stream=None):
    """Proposal-network inputs (n_pairs, 2 (4 n_hot + 5) + n_hot^2) and the picks (n_regions, n_hot), on the device."""
    import numpy as np
    torch = _torch()
    regs = (corr_region * len(regions))(*[r if isinstance(r, corr_region) else region(*r) for r in regions])
    rp = np.ascontiguousarray(np.asarray(region_pairs, dtype=np.int32).reshape(-1, 2))
    width = 2 * (4 * n_hot + 5) + n_hot * n_hot
    x = torch.empty(rp.shape[0], width, device=A.data.device, dtype=torch.float32)
    hot = torch.empty(len(regions), n_hot, device=A.data.device, dtype=torch.int32)
    _lib.check(ctx.L.corr_proposal_inputs(ctx.h, ctypes.byref(A.c), regs, len(regions), ctypes.c_void_p(rp.ctypes.data),
                                          rp.shape[0], int(n_hot), int(D), int(r_nms), ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(hot.data_ptr()), _stream_ptr(stream)))
    return x, hot


def _peak_out(out, n_blocks, dtypes):
    """The probes write one word per thread: out must be a device tensor of n_blocks * 256 words."""
    torch = _torch()
    if not out.is_cuda or out.dtype not in [getattr(torch, d) for d in dtypes] or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous device tensor of dtype {' or '.join(dtypes)}")
    if out.numel() < int(n_blocks) * 256:
        raise ValueError(f"out must hold at least n_blocks * 256 = {int(n_blocks) * 256} elements")


def _peak(name, n_blocks, iters, out, stream, dtypes=("float32",)):
    _peak_out(out, n_blocks, dtypes)
    _lib.check(getattr(_lib.load(), name)(int(n_blocks), int(iters), ctypes.c_void_p(out.data_ptr()),
                                         _stream_ptr(stream)))


def corr_peak_lds(n_blocks: int, iters: int, out, stream=None):
    """LDS read probe (include/corr_peaks.h); out: device uint32/int32, >= n_blocks * 256."""
    _peak("corr_peak_lds", n_blocks, iters, out, stream, ("int32", "uint32"))


def corr_peak_mfma_f16(n_blocks: int, iters: int, out, random_operands: bool = True, stream=None):
    """FP16 MFMA probe (random full-mantissa operands, or small repeated ones); out: device float32."""
    _peak_out(out, n_blocks, ("float32",))
    _lib.check(_lib.load().corr_peak_mfma_f16(int(n_blocks), int(iters), 1 if random_operands else 0,
                                              ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))


def corr_peak_valu_f32(n_blocks: int, iters: int, out, stream=None):
    """FP32 vector FMA probe; out: device float32, >= n_blocks * 256."""
    _peak("corr_peak_valu_f32", n_blocks, iters, out, stream)


def corr_peak_valu_med3(n_blocks: int, iters: int, out, stream=None):
    """FP32 median (v_med3_f32) issue probe; out: device float32, >= n_blocks * 256."""
    _peak("corr_peak_valu_med3", n_blocks, iters, out, stream)


def corr_peak_valu_f64(n_blocks: int, iters: int, out, stream=None):
    """FP64 vector FMA probe; out: device float64, >= n_blocks * 256."""
    _peak("corr_peak_valu_f64", n_blocks, iters, out, stream, ("float64",))


def corr_peak_hbm_read(buf, n_blocks: int, out, stream=None):
    """HBM read probe over the whole device tensor buf (16-byte aligned); out: device uint32, >= n_blocks * 256."""
    _peak_out(out, n_blocks, ("int32", "uint32"))
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous device tensor")
    nbytes = buf.numel() * buf.element_size()
    _lib.check(_lib.load().corr_peak_hbm_read(ctypes.c_void_p(buf.data_ptr()), ctypes.c_size_t(nbytes), int(n_blocks),
                                              ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))


def version() -> str:
    return _lib.load().corr_version().decode()
