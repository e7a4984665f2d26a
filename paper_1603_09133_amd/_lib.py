"""ctypes binding of ``libcae.so`` (the C ABI in ``include/cae.h``).

Argument marshalling only: every numeric step runs in the HIP library.  Device
buffers are PyTorch CUDA (HIP) tensors; their ``data_ptr()`` is passed through.
The library must have been built (``paper_1603_09133_amd.build``); importing the
binding never compiles and never falls back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcae.so")

CAE_OK, CAE_EINVAL, CAE_ENOMEM, CAE_ENOTSPD, CAE_ENOCONV, CAE_EDEVICE = 0, -1, -2, -3, -4, -5
RANK_EPS, RANK_FIXED, RANK_LEARNED, RANK_LEARNED_CAP = 0, 1, 2, 3
RECORD_WIDTH = 17
FP64, FP32, FP32_BF16 = 0, 1, 2
ORDER_PAPER, ORDER_MULTICOLOUR = 0, 1


class CAEError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cae error {code}: {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("rank_mode", C.c_int32), ("fixed_rank", C.c_int32),
                ("precision", C.c_int32), ("order", C.c_int32), ("max_levels", C.c_int32),
                ("timing", C.c_int32), ("compensate", C.c_int32),
                ("coarse_max_dim", C.c_int64), ("stream", C.c_void_p), ("mlp_params", C.c_void_p),
                ("seed", C.c_uint64), ("record", C.c_void_p), ("record_cap", C.c_int64), ("coarsen", C.c_int32),
                ("graphs", C.c_int32), ("apply_split_steps", C.c_int32), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("big_pivot_cap", C.c_int32)]


class Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("vals", C.c_void_p),
                ("ndim", C.c_int32), ("dims", C.c_int32 * 3), ("patch", C.c_int32 * 3)]


class LevelInfo(C.Structure):
    _fields_ = [("M", C.c_int32), ("nclose", C.c_int32), ("nfar", C.c_int32), ("nremoved", C.c_int32),
                ("nwaves", C.c_int32), ("Mnext", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("coarse_dim", C.c_int64), ("tau", C.c_double),
                ("dropped_sq", C.c_double), ("min_pivot", C.c_double), ("factor_bytes", C.c_int64),
                ("factor_ms", C.c_double), ("compress_launches", C.c_int32), ("compress_ms", C.c_double),
                ("compress_flops", C.c_double), ("compressions", C.c_int32), ("sketch_accepted", C.c_int32),
                ("sketch_rejected", C.c_int32), ("record_rows", C.c_int64), ("rotate_flops", C.c_double),
                ("elim_flops", C.c_double), ("schur_flops", C.c_double), ("coarse_flops", C.c_double),
                ("big_untruncated", C.c_int32), ("big_frobenius", C.c_int32), ("big_certified", C.c_int32),
                ("big_uncapped", C.c_int32), ("schur_launches", C.c_int32), ("schur_ms", C.c_double)]


_lib = None

EXPORTS = [
    "cae_default_options", "cae_last_error", "cae_grid_order", "cae_graph_order", "cae_analyze", "cae_analysis_levels",
    "cae_analysis_level_info", "cae_analysis_level_arrays", "cae_analysis_perm", "cae_analysis_destroy",
    "cae_analyze_batched", "cae_analysis_batch_rows", "cae_factor_batched", "cae_pcg_solve_batched",
    "cae_factor_numeric", "cae_workspace_query", "cae_factor", "cae_apply_precond", "cae_apply_precond_noalloc", "cae_apply_factor", "cae_pcg_solve", "cae_minres_solve",
    "cae_get_stats",
    "cae_get_ranks", "cae_get_sizes", "cae_get_drops", "cae_get_level_ms", "cae_export_factor", "cae_destroy", "cae_mlp_param_count", "cae_mlp_train", "cae_mlp_loss_grad",
    "cae_mlp_predict",
]


def lib():
    """Load the built library (raises when it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1603_09133_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    p, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.cae_default_options.argtypes = [C.POINTER(Options)]
    L.cae_default_options.restype = None
    L.cae_last_error.argtypes = [p]
    L.cae_last_error.restype = C.c_char_p
    L.cae_grid_order.argtypes = [i32, p, p, p, p, p, p]
    L.cae_graph_order.argtypes = [i64, p, p, i32, p, p, p]
    L.cae_analyze.argtypes = [i64, p, p, p, p, i32, i32, p, i32, C.POINTER(Options), C.POINTER(p)]
    L.cae_analysis_levels.argtypes = [p, p]
    L.cae_analysis_level_info.argtypes = [p, i32, C.POINTER(LevelInfo)]
    L.cae_analysis_level_arrays.argtypes = [p, i32, p, p, p, p, p, p]
    L.cae_analysis_perm.argtypes = [p, p, p]
    L.cae_analysis_destroy.argtypes = [p]
    L.cae_analysis_destroy.restype = None
    L.cae_factor_numeric.argtypes = [p, p, dbl, C.POINTER(Options), C.POINTER(p)]
    L.cae_workspace_query.argtypes = [p, p, dbl, C.POINTER(Options), C.POINTER(C.c_size_t)]
    L.cae_factor.argtypes = [i64, p, p, p, p, p, i32, i32, p, i32, dbl, C.POINTER(Options), C.POINTER(p)]
    L.cae_apply_precond.argtypes = [p, i32, p, i64, p, i64]
    L.cae_apply_precond_noalloc.argtypes = [p, i32, p, i64, p, i64, p]
    L.cae_apply_factor.argtypes = [p, i32, p, i64, p, i64]
    L.cae_pcg_solve.argtypes = [p, i32, p, i64, p, i64, dbl, i32, p, p]
    L.cae_analyze_batched.argtypes = [i32, C.POINTER(Problem), C.POINTER(Options), C.POINTER(p)]
    L.cae_analysis_batch_rows.argtypes = [p, C.POINTER(i32), p]
    L.cae_factor_batched.argtypes = [i32, C.POINTER(Problem), dbl, C.POINTER(Options), C.POINTER(p)]
    L.cae_pcg_solve_batched.argtypes = [p, i32, p, i64, p, i64, dbl, i32, p, p]
    L.cae_minres_solve.argtypes = [p, i32, p, i64, p, i64, dbl, i32, p, p]
    L.cae_get_stats.argtypes = [p, C.POINTER(Stats)]
    L.cae_get_ranks.argtypes = [p, i32, p]
    L.cae_get_sizes.argtypes = [p, i32, p]
    L.cae_get_drops.argtypes = [p, i32, p]
    L.cae_export_factor.argtypes = [p, C.c_char_p]
    L.cae_get_level_ms.argtypes = [p, i32, C.POINTER(dbl)]
    L.cae_destroy.argtypes = [p]
    L.cae_destroy.restype = None
    L.cae_mlp_param_count.argtypes = []
    L.cae_mlp_param_count.restype = i32
    L.cae_mlp_train.argtypes = [p, i64, p, i32, C.c_float, C.POINTER(C.c_float), p]
    L.cae_mlp_loss_grad.argtypes = [p, p, i64, p, C.POINTER(C.c_float), p]
    L.cae_mlp_predict.argtypes = [p, p, i64, p, p]
    for name in ["cae_grid_order", "cae_graph_order", "cae_analyze", "cae_analysis_levels", "cae_analysis_level_info",
                 "cae_analysis_level_arrays", "cae_analysis_perm", "cae_factor_numeric", "cae_workspace_query", "cae_factor",
                 "cae_apply_precond", "cae_analyze_batched", "cae_analysis_batch_rows", "cae_factor_batched",
                 "cae_pcg_solve_batched",
                 "cae_apply_precond_noalloc", "cae_apply_factor", "cae_pcg_solve", "cae_minres_solve", "cae_get_stats", "cae_get_ranks",
                 "cae_get_sizes", "cae_get_drops", "cae_get_level_ms", "cae_export_factor", "cae_mlp_train", "cae_mlp_loss_grad", "cae_mlp_predict"]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(rc, allow=()):
    if rc != CAE_OK and rc not in allow:
        raise CAEError(rc, lib().cae_last_error(None).decode())
    return rc


def ptr(a):
    """Address of a NumPy array (host) or a torch tensor (host or device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()
