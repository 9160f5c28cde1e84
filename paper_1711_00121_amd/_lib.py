"""ctypes declarations of libsimrank's C ABI (include/simrank.h).

The library is loaded after ``torch`` so that both share one HIP runtime (same soname).
There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library links against)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsimrank.so")

SR_OK, SR_EINVAL, SR_ERANGE, SR_EEXIST, SR_ENOENT, SR_ESELF = 0, -1, -2, -3, -4, -5
SR_ECAPACITY, SR_ENOMEM, SR_EMODE, SR_EHIP = -6, -7, -8, -9
SR_S_FP64, SR_S_FP32_HILO, SR_S_FP32 = 0, 1, 2
SR_DENSE, SR_COLUMN = 0, 1
SR_GAMMA_CLOSED, SR_GAMMA_DIRECT = 0, 1
SR_COL_S, SR_COL_DELTA = 0, 1
SR_UPDATE_FP64, SR_UPDATE_FP32 = 0, 1


class sr_config(C.Structure):
    _fields_ = [
        ("C", C.c_double),
        ("K", C.c_int32),
        ("K_ps", C.c_int32),
        ("s_prec", C.c_int32),
        ("mode", C.c_int32),
        ("gamma_form", C.c_int32),
        ("prune", C.c_int32),
        ("node_cap", C.c_int64),
        ("edge_cap", C.c_int64),
        ("init_tol", C.c_double),
        ("init_max_iter", C.c_int32),
        ("batch_chunk", C.c_int32),
        ("fused_batch", C.c_int32),
        ("split_rows", C.c_int32),
        ("profile", C.c_int32),
        ("graphs", C.c_int32),
        ("update_prec", C.c_int32),
        ("block_store", C.c_int32),
        ("tile_skip", C.c_int32),
    ]


class sr_update_stats(C.Structure):
    _fields_ = [
        ("case_id", C.c_int32),
        ("op", C.c_int32),
        ("d_j", C.c_int64),
        ("n_after", C.c_int64),
        ("aff_A", C.c_int64),
        ("aff_B", C.c_int64),
        ("aff_AB", C.c_int64),
        ("pairs", C.c_int64),
        ("bound", C.c_double),
    ]


class sr_batch_stats(C.Structure):
    _fields_ = [
        ("edges_in", C.c_int64),
        ("edges_net", C.c_int64),
        ("blocks", C.c_int64),
        ("blocks_case", C.c_int64 * 4),
        ("lowrank_blocks", C.c_int64),
        ("n_after", C.c_int64),
        ("pairs", C.c_int64),
        ("fused_passes", C.c_int32),
        ("series_replays", C.c_int32),
        ("pass_entries", C.c_int64),
        ("pass_skipped", C.c_int64),
    ]


P = C.c_void_p
I32P = C.POINTER(C.c_int32)
I8P = C.POINTER(C.c_int8)
F64P = C.POINTER(C.c_double)

# name: (restype, argtypes)
SIGNATURES = {
    "sr_default_config": (C.c_int, [C.POINTER(sr_config)]),
    "init_simrank": (C.c_int, [C.POINTER(P), C.c_int64, C.c_int64, I32P, I32P, F64P,
                               C.POINTER(sr_config), P, P]),
    "init_simrank_tree": (C.c_int, [C.POINTER(P), C.c_int64, C.c_int64, I32P, I32P,
                                    C.POINTER(sr_config), P, C.POINTER(sr_batch_stats)]),
    "sr_partition": (C.c_int, [C.c_int64, C.c_int64, I32P, I32P, C.c_int32, I32P]),
    "init_simrank_partitioned": (C.c_int, [C.POINTER(P), C.c_int64, C.c_int64, I32P, I32P, I32P,
                                           C.POINTER(sr_config), P, C.POINTER(sr_batch_stats)]),
    "apply_edge_update": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int32,
                                    C.POINTER(sr_update_stats)]),
    "apply_weight_update": (C.c_int, [P, C.c_int32, C.c_int32, C.c_double,
                                      C.POINTER(sr_update_stats)]),
    "apply_batch": (C.c_int, [P, C.c_int64, I32P, I32P, I8P, C.POINTER(sr_batch_stats)]),
    "apply_batch_columns": (C.c_int, [P, C.c_int64, I32P, I32P, I8P, I32P, C.c_int32, P,
                                      C.c_int64, C.POINTER(sr_batch_stats)]),
    "query_column": (C.c_int, [P, C.c_int32, C.c_int32, P]),
    "query_columns": (C.c_int, [P, I32P, C.c_int32, P, C.c_int64]),
    "query_topk": (C.c_int, [P, I32P, C.c_int32, C.c_int32, C.c_int32, P, P]),
    "query_topk_noalloc": (C.c_int, [P, I32P, C.c_int32, C.c_int32, C.c_int32, P, P]),
    "sr_gather_pairs": (C.c_int, [P, C.c_int64, P, P, P]),
    "backward": (C.c_int, [P, C.c_int64, P, P, P, P]),
    "sr_get_aff": (C.c_int, [P, C.c_int32, P, C.POINTER(C.c_int64), P,
                             C.POINTER(C.c_int64)]),
    "sr_copy_S": (C.c_int, [P, P, C.c_int64]),
    "sr_sizes": (C.c_int, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sr_get_config": (C.c_int, [P, C.POINTER(sr_config)]),
    "sr_store_bytes": (C.c_int, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sr_device_bytes": (C.c_int, [C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int32]),
    "sr_edges": (C.c_int, [P, I32P, I32P, F64P, C.c_int64, C.POINTER(C.c_int64)]),
    "sr_last_plan": (C.c_int, [P, I32P, C.c_int64, C.POINTER(C.c_int64)]),
    "sr_synchronize": (C.c_int, [P]),
    "sr_destroy": (C.c_int, [P]),
    "sr_strerror": (C.c_char_p, [C.c_int]),
    "sr_mfma_layout_probe": (C.c_int, [P, P, P, P]),
    "sr_mfma_layout_probe_f32": (C.c_int, [P, P, P, P]),
    "sr_profile": (C.c_int, [P, C.c_int32]),
    "sr_time_fused": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                C.POINTER(C.c_double)]),
    "sr_set_tuning": (C.c_int, [P, C.c_int32, C.c_int32]),
    "sr_profile_read": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]),
}

_lib = None


class SimRankError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.sr_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")


def load():
    """Loads libsimrank.so (built in-tree by ``paper_1711_00121_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1711_00121_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, where):
    if status != SR_OK:
        raise SimRankError(status, where)
