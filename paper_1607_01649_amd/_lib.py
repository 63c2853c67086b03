"""ctypes binding of ``librsvd.so`` (the C ABI declared in include/rsvd.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Importing this module fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsvd.so")

RSVD_OK = 0
RSVD_NOT_CERTIFIED = 1
RSVD_E_ARG = -1
RSVD_E_WORKSPACE = -2
RSVD_E_HIP = -3
RSVD_E_NONFINITE = -4
RSVD_E_UNSUPPORTED = -5

RSVD_F64, RSVD_F32, RSVD_BF16, RSVD_FP8_E4M3 = 0, 1, 2, 3
RSVD_RETURN_RANK_L = 0x1
RSVD_TIMING = 0x2
RSVD_SKETCH_SRHT = 0x4
RSVD_NYSTROM = 0x8
RSVD_SINGLE_PASS = 0x10
RSVD_SINGLE_PASS_SYM = 0x20
RSVD_ID_CUR = 0x40

STREAM_OMEGA = 4
STREAM_PROBE = 5
STREAM_CERT = 6


class rsvd_desc(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64),
        ("k", ctypes.c_int32), ("p", ctypes.c_int32), ("q", ctypes.c_int32),
        ("a_dtype", ctypes.c_int32), ("sketch_dtype", ctypes.c_int32), ("proj_dtype", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("eps", ctypes.c_double),
        ("n_probe", ctypes.c_int32), ("est_power", ctypes.c_int32),
        ("fallback_block", ctypes.c_int32), ("max_rank", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("reserved_", ctypes.c_uint32),
    ]


class rsvd_info(ctypes.Structure):
    _fields_ = [
        ("p_used", ctypes.c_int32), ("q_used", ctypes.c_int32), ("rank_out", ctypes.c_int32),
        ("fallback_steps", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("status", ctypes.c_int32),
        ("err_bound", ctypes.c_double), ("sigma1", ctypes.c_double),
        ("stage_ms", ctypes.c_float * 8),
        ("nn_ms", ctypes.c_float), ("tn_ms", ctypes.c_float),
        ("nn_launches", ctypes.c_int32), ("tn_launches", ctypes.c_int32),
        ("jacobi_sweeps", ctypes.c_int32), ("dropped_cols", ctypes.c_int32),
        ("frob_residual", ctypes.c_double),
    ]


_c_void_p = ctypes.c_void_p
_i64 = ctypes.c_int64

# (name, restype, argtypes) for every symbol declared in include/rsvd.h
SIGNATURES = [
    ("rsvd_status_str", ctypes.c_char_p, [ctypes.c_int]),
    ("rsvd_workspace_size", ctypes.c_int, [ctypes.POINTER(rsvd_desc), ctypes.POINTER(ctypes.c_size_t)]),
    ("rsvd_plan", ctypes.c_int, [ctypes.POINTER(rsvd_desc), _c_void_p, ctypes.c_size_t, _c_void_p,
                                 ctypes.POINTER(_c_void_p)]),
    ("rsvd_factor", ctypes.c_int, [_c_void_p, _c_void_p, _i64, _c_void_p, _c_void_p, _i64, _c_void_p, _c_void_p,
                                   _i64, ctypes.POINTER(rsvd_info)]),
    ("rsvd_destroy", None, [_c_void_p]),
    ("rsvd_row_id", ctypes.c_int, [_c_void_p, _c_void_p, _i64, _c_void_p, _c_void_p, _c_void_p, _i64,
                                   ctypes.POINTER(rsvd_info)]),
    ("rsvd_cur", ctypes.c_int, [_c_void_p, _c_void_p, _i64, _c_void_p, _c_void_p, _i64, _c_void_p,
                                ctypes.POINTER(rsvd_info)]),
    ("rsvd_factor_noalloc", ctypes.c_int, [ctypes.POINTER(rsvd_desc), _c_void_p, _i64, _c_void_p, _c_void_p, _i64,
                                           _c_void_p, _c_void_p, _i64, _c_void_p]),
    ("rsvd_gaussian", ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint32, _i64, _i64, _i64, ctypes.c_int32, _c_void_p,
                                     _i64, _c_void_p]),
    ("rsvd_philox4x32_10", ctypes.c_int, [_i64, _c_void_p, ctypes.c_uint32, ctypes.c_uint32, _c_void_p,
                                          _c_void_p]),
    ("rsvd_batched_workspace_size", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    ("rsvd_batched", ctypes.c_int, [ctypes.c_int32, _c_void_p, _c_void_p, _c_void_p, _c_void_p, ctypes.c_double,
                                    ctypes.c_int32, ctypes.c_uint64, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                    _c_void_p, _c_void_p, _c_void_p, ctypes.c_int32, _c_void_p, _c_void_p,
                                    ctypes.c_size_t, _c_void_p]),
    ("rsvd_batched_autotune", ctypes.c_int, [ctypes.c_int32, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                             ctypes.c_double, ctypes.c_int32, ctypes.c_uint64, _c_void_p,
                                             _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                             ctypes.c_int32, _c_void_p, ctypes.c_size_t, _c_void_p, _c_void_p,
                                             _c_void_p]),
    ("rsvd_batched_graph_create", ctypes.c_int, [ctypes.c_int32, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                                 ctypes.c_double, ctypes.c_int32, ctypes.c_uint64, _c_void_p,
                                                 _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                                 ctypes.c_int32, _c_void_p, _c_void_p, ctypes.c_size_t, _c_void_p,
                                                 ctypes.POINTER(_c_void_p)]),
    ("rsvd_graph_launch", ctypes.c_int, [_c_void_p, _c_void_p]),
    ("rsvd_graph_destroy", None, [_c_void_p]),
    ("rsvd_selector_set", ctypes.c_int, [_c_void_p, _c_void_p, ctypes.c_float]),
    ("rsvd_probe_sigma", ctypes.c_int, [_c_void_p, _c_void_p, _i64, _c_void_p, _c_void_p]),
    ("rsvd_prefix_bounds", ctypes.c_int, [_c_void_p, _c_void_p, _i64, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    ("rsvd_mlp_forward", ctypes.c_int, [_c_void_p, ctypes.c_int32, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                        _c_void_p]),
    ("rsvd_mlp_backward", ctypes.c_int, [_c_void_p, ctypes.c_int32, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                         _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    ("rsvd_mlp_adam", ctypes.c_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, ctypes.c_int32, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int32, _c_void_p]),
    # include/rsvd_kernels.h
    ("rsvd_k_srht_sketch", ctypes.c_int, [ctypes.c_int32, _i64, _i64, _c_void_p, _i64, ctypes.c_int32,
                                          ctypes.c_uint64, _c_void_p, _c_void_p, _c_void_p, _i64, _c_void_p]),
    ("rsvd_k_product_nn", ctypes.c_int, [ctypes.c_int32, _i64, _i64, _c_void_p, _i64, _c_void_p, _i64,
                                         ctypes.c_int32, _c_void_p, _i64, _c_void_p]),
    ("rsvd_k_product_tn", ctypes.c_int, [ctypes.c_int32, _i64, _i64, _c_void_p, _i64, _c_void_p, _i64,
                                         ctypes.c_int32, _c_void_p, _i64, ctypes.c_int32, _c_void_p]),
    ("rsvd_k_gram", ctypes.c_int, [ctypes.c_int32, _i64, ctypes.c_int32, _c_void_p, _i64, _c_void_p, _i64,
                                   _c_void_p]),
    ("rsvd_k_cholesky", ctypes.c_int, [ctypes.c_int32, _c_void_p, _i64, ctypes.c_double, _c_void_p, _c_void_p,
                                       _c_void_p, _c_void_p, _c_void_p]),
    ("rsvd_k_small_svd", ctypes.c_int, [ctypes.c_int32, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                        _c_void_p]),
    ("rsvd_k_scratch_bytes", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    ("rsvd_k_convert_bf16", ctypes.c_int, [_i64, _i64, _c_void_p, _i64, _c_void_p, _i64, _c_void_p, _i64, _c_void_p,
                                           _c_void_p]),
    ("rsvd_k_product_bf16", ctypes.c_int, [_i64, _i64, _c_void_p, _i64, _c_void_p, _i64, ctypes.c_int32, _c_void_p,
                                           _i64, _c_void_p, _c_void_p]),
    ("rsvd_k_lp_scratch_bytes", ctypes.c_int, [ctypes.c_int32, _i64, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    ("rsvd_k_convert_fp8", ctypes.c_int, [_i64, _i64, _c_void_p, _i64, _c_void_p, _i64, _c_void_p, _i64, _c_void_p,
                                          _c_void_p, _c_void_p]),
    ("rsvd_k_product_fp8", ctypes.c_int, [_i64, _i64, _c_void_p, _i64, _c_void_p, _i64, _i64, _c_void_p, _i64,
                                          ctypes.c_int32, _c_void_p, _i64, _c_void_p, _c_void_p]),
]

RSVD_F32_ACC64 = 10

# selector network and grid (include/rsvd.h)
RSVD_MLP_IN, RSVD_MLP_HIDDEN, RSVD_MLP_OUT, RSVD_MLP_NPARAM = 16, 64, 40, 7848
RSVD_SEL_P = (0, 5, 10, 20, 40, 80, 160, 320)
RSVD_SEL_NQ = 5

# batched compression tile table (include/rsvd.h)
RSVD_BATCHED_CLASSES, RSVD_BATCHED_TILE_VARIANTS = 4, 8


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class RSVDError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def status_str(status: int) -> str:
    return lib().rsvd_status_str(int(status)).decode()
