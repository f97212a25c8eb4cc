"""ctypes declarations of libhyperef.so (include/hyperef.h)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhyperef.so")

HEF_OK = 0
STATUS = {
    0: "HEF_OK", 1: "HEF_ERR_INVALID_ARGUMENT", 2: "HEF_ERR_INVALID_HYPERGRAPH",
    3: "HEF_ERR_WORKSPACE_TOO_SMALL", 4: "HEF_ERR_DEVICE", 5: "HEF_ERR_NUMERICAL",
    6: "HEF_ERR_UNSUPPORTED",
}
(OP_RESISTANCE, OP_COARSEN, OP_CLUSTER_LEVEL, OP_BACKWARD, OP_APPLY, OP_CONDUCTANCE,
 OP_REBUILD, OP_RATING) = range(8)
BASIS_FP32, BASIS_BF16, BASIS_FP64 = 0, 1, 2
STATIC_SCRATCH_BYTES = 64 << 20  # HEF_STATIC_SCRATCH_BYTES
FLAG_ASSUME_VALID, FLAG_STAR_ONLY, FLAG_CLIQUE_ONLY, FLAG_TAPED = 1, 2, 4, 8

EXPORTS = [
    "hef_params_default", "hef_pool_width", "hef_workspace_size", "hef_validate_host",
    "hef_resistance", "hef_resistance_static", "hef_coarsen", "hef_cluster_level", "hef_resistance_backward",
    "hef_resistance_taped", "hef_conductance", "hef_coarsen_levels", "hef_rebuild",
    "hef_rating",
    "hef_debug_apply", "hef_debug_gram", "hef_debug_gram_ws", "hef_start_block",
    "hef_status_string", "hef_last_error", "hef_timing_enable", "hef_timing_stages",
    "hef_timing_stage_count",
    "hef_timing_stage_name", "hef_timing_read", "hef_last_coarsen_levels",
    "hef_last_coarsen_work",
]


class HefHypergraph(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("nnz", C.c_int64),
                ("eptr", C.c_void_p), ("pins", C.c_void_p), ("w", C.c_void_p)]


class HefParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("b", C.c_int32), ("levels", C.c_int32),
                ("percentile", C.c_float), ("local_clustering", C.c_int32),
                ("basis", C.c_int32), ("seed", C.c_uint64), ("drop_tol", C.c_float),
                ("orth_passes", C.c_int32), ("ckpt_every", C.c_int32), ("flags", C.c_uint32),
                ("target_nr", C.c_float)]


class HefLevelTrace(C.Structure):
    _fields_ = [("cap", C.c_int32), ("levels_run", C.c_int32),
                ("n", C.c_void_p), ("m", C.c_void_p), ("nnz", C.c_void_p),
                ("R", C.c_void_p), ("qh", C.c_void_p), ("rho", C.c_void_p),
                ("label", C.c_void_p), ("eta", C.c_void_p)]


class HefError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")
        self.status = status


_lib = None


def load() -> C.CDLL:
    """Loads the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2511_06600_amd.build` (there is no fallback path)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_size_t
    HG, PR = C.POINTER(HefHypergraph), C.POINTER(HefParams)
    sig = {
        "hef_params_default": (None, [PR]),
        "hef_pool_width": (i32, [PR]),
        "hef_workspace_size": (i32, [HG, PR, i32, C.POINTER(sz)]),
        "hef_validate_host": (i32, [i32, i32, vp, vp, vp]),
        "hef_resistance": (i32, [HG, PR, vp, vp, vp, vp, vp, vp, sz, vp]),
        "hef_resistance_static": (i32, [HG, PR, vp, vp, vp, vp, vp, vp]),
        "hef_coarsen": (i32, [HG, PR, vp, C.POINTER(i32), vp, vp, vp, sz, vp]),
        "hef_coarsen_levels": (i32, [HG, PR, vp, C.POINTER(i32), vp, vp,
                                     C.POINTER(HefLevelTrace), vp, sz, vp]),
        "hef_rebuild": (i32, [HG, vp, i32, vp, vp, vp, vp, C.POINTER(i32), C.POINTER(i64), vp,
                              sz, vp]),
        "hef_rating": (i32, [HG, vp, C.c_float, vp, vp, vp, sz, vp]),
        "hef_cluster_level": (i32, [HG, PR, vp, vp, vp, vp, vp, C.POINTER(i32), vp, vp, sz, vp]),
        "hef_resistance_backward": (i32, [HG, PR, vp, vp, vp, vp, vp, sz, vp]),
        "hef_resistance_taped": (i32, [HG, PR, vp, vp, vp, vp, sz, vp]),
        "hef_conductance": (i32, [HG, vp, i32, vp, vp, vp, vp, vp, sz, vp]),
        "hef_debug_apply": (i32, [HG, i32, i32, vp, vp, vp, sz, vp]),
        "hef_debug_gram": (i32, [vp, i64, i32, vp, vp, sz, vp]),
        "hef_debug_gram_ws": (sz, [i64, i32]),
        "hef_start_block": (i32, [u64, i32, i32, i64, i32, vp, vp]),
        "hef_status_string": (C.c_char_p, [i32]),
        "hef_last_error": (C.c_char_p, []),
        "hef_timing_enable": (None, [i32]),
        "hef_timing_stages": (None, [C.c_uint32]),
        "hef_timing_stage_count": (i32, []),
        "hef_timing_stage_name": (C.c_char_p, [i32]),
        "hef_timing_read": (i32, [vp, vp, i32, i32]),
        "hef_last_coarsen_levels": (i32, [vp, vp, vp, i32]),
        "hef_last_coarsen_work": (i32, [vp, i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != HEF_OK:
        detail = load().hef_last_error().decode(errors="replace")
        raise HefError(status, where, detail)
