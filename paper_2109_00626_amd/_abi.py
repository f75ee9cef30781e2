"""ctypes declarations of the C ABI in include/ttc.h and the library loader.

Argument marshalling only: every computation happens in libttc.so.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_uint32, c_void_p, c_char_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libttc.so")

TTC_OK = 0
STATUS_NAMES = {
    0: "TTC_OK", 1: "TTC_ERR_NULL", 2: "TTC_ERR_SHAPE", 3: "TTC_ERR_RANK", 4: "TTC_ERR_MODE",
    5: "TTC_ERR_DTYPE", 6: "TTC_ERR_UNSUPPORTED", 7: "TTC_ERR_WORKSPACE", 8: "TTC_ERR_HIP",
}
TTC_F64, TTC_F32, TTC_BF16 = 0, 1, 2
PREC = {"auto": 0, "f64": 1, "f32": 2, "bf16": 3}
FORM = {"junction": 0, "natural": 1, "dense": 2}
SCHED = {"auto": 0, "cores": 1, "dense": 2, "cores_saved": 3}
OP_INNER, OP_SUFFIX2 = 1, 2


class TT(ctypes.Structure):
    _fields_ = [("order", c_int32), ("modes", POINTER(c_int32)), ("ranks", POINTER(c_int32)),
                ("dtype", c_int32), ("cores", POINTER(c_void_p))]


class TTM(ctypes.Structure):
    _fields_ = [("order", c_int32), ("rows", POINTER(c_int32)), ("cols", POINTER(c_int32)),
                ("ranks", POINTER(c_int32)), ("dtype", c_int32), ("cores", POINTER(c_void_p))]


class Pair(ctypes.Structure):
    _fields_ = [("x", TT), ("y", TT)]


class TTCError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


def _declare(lib):
    P = POINTER
    sig = {
        "ttc_last_error": (c_char_p, []),
        "ttc_version": (c_char_p, []),
        "ttc_abi_version": (c_int32, []),
        "tt_contract_inner_query": (c_int32, [P(TT), P(TT), c_int32, P(c_size_t)]),
        "tt_contract_inner": (c_int32, [P(TT), P(TT), c_int32, c_void_p, c_void_p, c_size_t, c_void_p]),
        "tt_contract_inner_noalloc": (c_int32, [P(TT), P(TT), c_int32, c_void_p, c_void_p]),
        "tt_contract_modes_query": (c_int32, [P(TT), P(TT), P(c_int32), c_int32, c_int32, c_int32, P(c_int32),
                                              P(c_int32), P(c_int32), P(c_int64), P(c_size_t)]),
        "tt_contract_modes": (c_int32, [P(TT), P(TT), P(c_int32), c_int32, c_int32, c_int32, c_void_p, P(TT),
                                        c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
        "tt_mode_n_product": (c_int32, [P(TT), c_int32, P(c_int32), P(c_void_p), P(c_int32), P(TT), c_void_p]),
        "ttm_apply_query": (c_int32, [P(TTM), P(TT), P(c_int32), P(c_int64)]),
        "ttm_apply": (c_int32, [P(TTM), P(TT), c_int32, P(TT), c_void_p]),
        "ttm_apply_dense_query": (c_int32, [P(TTM), c_int64, c_int32, c_int32, c_int32, P(c_size_t)]),
        "ttm_apply_dense": (c_int32, [P(TTM), c_void_p, c_int64, c_void_p, c_int32, c_int32, c_void_p,
                                      c_size_t, c_void_p]),
        "ttm_apply_dense_bwd": (c_int32, [P(TTM), c_void_p, c_void_p, c_int64, c_void_p, P(c_void_p),
                                          c_int32, c_int32, c_void_p, c_size_t, c_void_p]),
        "ttc_mse_loss_query": (c_int32, [c_int64, P(c_size_t)]),
        "ttc_mse_loss": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_size_t,
                                   c_void_p]),
        "tt_contract_inner_bwd_query": (c_int32, [P(TT), P(TT), c_int32, P(c_size_t)]),
        "tt_contract_inner_bwd": (c_int32, [P(TT), P(TT), c_void_p, P(c_void_p), P(c_void_p), c_int32,
                                            c_void_p, c_size_t, c_void_p]),
        "tt_contract_pairs_query": (c_int32, [P(TT), P(TT), P(c_int32), P(c_int32), c_int32, c_int32, P(c_int32),
                                              P(c_int32), P(c_int32), P(c_int64), P(c_size_t)]),
        "tt_contract_pairs": (c_int32, [P(TT), P(TT), P(c_int32), P(c_int32), c_int32, c_int32, c_void_p, P(TT),
                                        c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
        "tt_svd_query": (c_int32, [c_int32, P(c_int32), c_int32, c_int32, P(c_int32), P(c_size_t)]),
        "tt_svd": (c_int32, [c_void_p, c_int32, P(c_int32), c_int32, c_double, c_int32, P(c_int32), P(c_void_p),
                             c_void_p, c_size_t, c_void_p]),
        "tt_round_query": (c_int32, [P(TT), c_int32, P(c_int32), P(c_size_t)]),
        "tt_round": (c_int32, [P(TT), c_double, c_int32, P(c_int32), P(c_void_p), c_void_p, c_size_t, c_void_p]),
        "tt_batch_plan_create": (c_int32, [P(Pair), c_int32, c_uint32, c_int32, P(c_void_p)]),
        "tt_batch_plan_query": (c_int32, [P(Pair), c_int32, c_uint32, P(c_int64), P(c_double), P(c_double),
                                          P(c_double), P(c_int32)]),
        "tt_batch_plan_info": (c_int32, [c_void_p, P(c_int64), P(c_double), P(c_double)]),
        "tt_batch_plan_config": (c_int32, [c_void_p, P(c_int32), P(c_int32), P(c_int32)]),
        "tt_batch_run": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
        "tt_batch_run_plain": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
        "tt_batch_run_traced": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
        "tt_batch_plan_destroy": (None, [c_void_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return sig


def load(path: str = None):
    # TTC_LIBRARY selects another build of the same library (for comparing builds)
    path = path or os.environ.get("TTC_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(
            f"libttc.so not found at {path}: build it first (python paper_2109_00626_amd/build.py "
            "or __graft_entry__.build()); there is no fallback implementation")
    lib = ctypes.CDLL(path)
    _declare(lib)
    return lib


EXPORTED = [
    "ttc_last_error", "ttc_version", "ttc_abi_version",
    "tt_contract_inner_query", "tt_contract_inner", "tt_contract_inner_noalloc",
    "tt_contract_modes_query", "tt_contract_modes",
    "tt_mode_n_product",
    "ttm_apply_query", "ttm_apply",
    "ttm_apply_dense_query", "ttm_apply_dense", "ttm_apply_dense_bwd",
    "ttc_mse_loss_query", "ttc_mse_loss",
    "tt_contract_inner_bwd_query", "tt_contract_inner_bwd",
    "tt_contract_pairs_query", "tt_contract_pairs",
    "tt_svd_query", "tt_svd", "tt_round_query", "tt_round",
    "tt_batch_plan_create", "tt_batch_plan_query", "tt_batch_plan_info", "tt_batch_plan_config", "tt_batch_run", "tt_batch_run_plain",
    "tt_batch_run_traced",
    "tt_batch_plan_destroy",
]
