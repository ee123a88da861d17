"""ctypes binding of libcorr (see include/corr.h and include/bos.h).

Argument marshalling only: torch tensors supply device memory and the current
HIP stream; every step of the computation runs in the library's kernels.
There is no fallback: if libcorr.so is missing or a call fails, an exception
is raised.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcorr.so")

CORR_OK, CORR_EINVAL, CORR_EUNSUPPORTED, CORR_ENOMEM, CORR_EHIP, CORR_ESTATE = range(6)
CORR_F32, CORR_F16 = 0, 1
PREC = {"f32": 0, "f16": 1, "bf16": 2, "f16x3": 3, "bf16x3": 4}
MEASURE = {"pearson": 0, "ksg": 1}
SAMPLER = {"uniform": 0, "halton": 1, "plastic": 2}
STRATEGY = {0: "bos", 1: "random", 2: "exhaustive"}
CORR_KSG_RAW = 1
BOS_LAUNCH = {"graph": 0, "plain": 1}


class corr_field(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("M", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("member_stride", ctypes.c_int64)]


class corr_region(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_int32), ("y0", ctypes.c_int32), ("z0", ctypes.c_int32),
                ("dx", ctypes.c_int32), ("dy", ctypes.c_int32), ("dz", ctypes.c_int32)]


class corr_max(ctypes.Structure):
    _fields_ = [("value", ctypes.c_float), ("signed_value", ctypes.c_float), ("pa", ctypes.c_int32),
                ("pb", ctypes.c_int32), ("n_evaluated", ctypes.c_int64)]


class bos_config(ctypes.Structure):
    _fields_ = [("measure", ctypes.c_int32), ("k", ctypes.c_int32), ("n_init", ctypes.c_int32),
                ("n_total", ctypes.c_int32), ("n_uniform", ctypes.c_int32), ("n_local", ctypes.c_int32),
                ("kappa", ctypes.c_double), ("lengthscale", ctypes.c_double), ("local_sd", ctypes.c_double),
                ("jitter", ctypes.c_double), ("seed", ctypes.c_uint64)]


class CorrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libcorr status {status}: {msg}")
        self.status = status


_lib = None

# (name, restype, argtypes) for every exported entry point
_P, _I, _I32, _I64, _U32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
SIGNATURES = {
    "corr_version": (ctypes.c_char_p, []),
    "corr_create": (_I, [_I, ctypes.POINTER(_P)]),
    "corr_destroy": (None, [_P]),
    "corr_status_str": (ctypes.c_char_p, [_I]),
    "corr_last_error": (ctypes.c_char_p, []),
    "corr_standardize": (_I, [_P, ctypes.POINTER(corr_field), _P, _P, _P, _P]),
    "corr_pearson_pairs": (_I, [_P, ctypes.POINTER(corr_field), ctypes.POINTER(corr_field), _P, _I64, _I, _P, _P]),
    "corr_ksg_mi_pairs": (_I, [_P, ctypes.POINTER(corr_field), ctypes.POINTER(corr_field), _P, _I64, _I32, _U32,
                               _P, _P, _P]),
    "corr_region_max": (_I, [_P, ctypes.POINTER(corr_field), ctypes.POINTER(corr_region), ctypes.POINTER(corr_field),
                             ctypes.POINTER(corr_region), _I, _I, _I32, _P, _I64, ctypes.POINTER(corr_max), _P]),
    "corr_prepare": (_I, [_P, ctypes.POINTER(corr_field), _I, _I, ctypes.POINTER(_P), _P]),
    "corr_prepared_destroy": (None, [_P]),
    "corr_box_pairs_max": (_I, [_P, _P, _P, _P, _P, _I32, _P, _P]),
    "corr_pearson_pairs_prepared": (_I, [_P, _P, _P, _P, _I64, _P, _P]),
    "corr_ksg_mi_pairs_prepared": (_I, [_P, _P, _P, _P, _I64, _I32, _P, _P, _P]),
    "corr_region_max_noalloc": (_I, [_P, ctypes.POINTER(corr_field), ctypes.POINTER(corr_region),
                                     ctypes.POINTER(corr_field), ctypes.POINTER(corr_region), _I, _I, _I32, _P, _I64,
                                     ctypes.POINTER(corr_max), _P]),
    "corr_autotune": (_I, [_P, ctypes.POINTER(corr_field), ctypes.POINTER(corr_region), ctypes.POINTER(corr_field),
                           ctypes.POINTER(corr_region), _I, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_float), _P]),
    "corr_ksg_autotune": (_I, [_P, ctypes.POINTER(corr_field), ctypes.POINTER(corr_field), _P, _I64, _I32, _I,
                               ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_float), _P]),
    "corr_tune_save": (_I, [_P, ctypes.c_char_p]),
    "corr_tune_load": (_I, [_P, ctypes.c_char_p]),
    "corr_set_timing": (_I, [_P, _I]),
    "corr_set_workspace_limit": (_I, [_P, ctypes.c_size_t]),
    "bos_config_default": (None, [ctypes.POINTER(bos_config)]),
    "bos_create": (_I, [_P, ctypes.POINTER(corr_field), ctypes.POINTER(corr_field), ctypes.POINTER(corr_region),
                        _I32, _P, _I32, ctypes.POINTER(bos_config), ctypes.POINTER(_P), _P]),
    "bos_set_prior": (_I, [_P, _P]),
    "bos_set_launch": (_I, [_P, _I32, ctypes.c_double]),
    "bos_sample_step": (_I, [_P, _P, ctypes.POINTER(_I32)]),
    "bos_run": (_I, [_P, _P]),
    "bos_results": (_I, [_P, ctypes.POINTER(corr_max), _P]),
    "bos_history": (_I, [_P, _I32, _P, _P, ctypes.POINTER(_I32), _P]),
    "bos_schedule": (_I, [_P, _P, _P]),
    "bos_save": (_I, [_P, ctypes.c_char_p, _P]),
    "bos_load": (_I, [_P, ctypes.c_char_p, _P]),
    "bos_destroy": (None, [_P]),
    "corr_kernel_time_ms": (_I, [_P, _I, ctypes.POINTER(ctypes.c_float)]),
    "corr_block_means": (_I, [_P, ctypes.POINTER(corr_field), _I, _I, _P, _I64, _P]),
    "corr_sample_pairs": (_I, [_P, ctypes.POINTER(corr_field), ctypes.POINTER(corr_field), _P, _I32, _P, _I32, _I,
                               _I32, ctypes.c_uint64, _P, _P]),
    "corr_sampled_max": (_I, [_P, ctypes.POINTER(corr_field), ctypes.POINTER(corr_field), _P, _I32, _P, _I32, _I,
                              _I, _I32, _I, _I32, ctypes.c_uint64, _P, _P]),
    "corr_choose_strategy": (_I, [_I64, _I64, ctypes.c_double, ctypes.c_double, ctypes.POINTER(_I32)]),
    "corr_region_submax": (_I, [_P, ctypes.POINTER(corr_field), ctypes.POINTER(corr_region), _P,
                                ctypes.POINTER(corr_field), ctypes.POINTER(corr_region), _P, _I, _P, _P]),
    "prop_mlp_create": (_I, [_P, _I32, _I32, _I32, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "prop_mlp_num_params": (_I, [_P, ctypes.POINTER(_I64)]),
    "prop_mlp_get_params": (_I, [_P, _P]),
    "prop_mlp_set_params": (_I, [_P, _P]),
    "prop_mlp_forward": (_I, [_P, _P, _I32, _P, _P]),
    "prop_mlp_train_step": (_I, [_P, _P, _P, _P, _I32, ctypes.c_float, ctypes.c_float,
                                 ctypes.POINTER(ctypes.c_float), _P]),
    "prop_mlp_get_grads": (_I, [_P, _P]),
    "prop_mlp_destroy": (None, [_P]),
    "corr_proposal_inputs": (_I, [_P, ctypes.POINTER(corr_field), ctypes.POINTER(corr_region), _I32, _P, _I32, _I32,
                                  _I32, _I32, _P, _P, _P]),
    "corr_peak_lds": (_I, [_I, _I, _P, _P]),
    "corr_peak_mfma_f16": (_I, [_I, _I, _I, _P, _P]),
    "corr_peak_valu_f32": (_I, [_I, _I, _P, _P]),
    "corr_peak_valu_med3": (_I, [_I, _I, _P, _P]),
    "corr_peak_valu_f64": (_I, [_I, _I, _P, _P]),
    "corr_peak_hbm_read": (_I, [_P, ctypes.c_size_t, _I, _P, _P]),
}


def load(path: str = LIB_PATH):
    """Load libcorr.so and declare the signatures; raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"libcorr.so not built ({path}); run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != CORR_OK:
        L = load()
        raise CorrError(status, L.corr_last_error().decode())
