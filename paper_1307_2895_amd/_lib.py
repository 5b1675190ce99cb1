"""ctypes binding of libhifde.so: argument marshalling only.

Every step of the factorization and of the solves runs inside the shared
library; this module converts Python/torch arguments to the C ABI of
``include/hifde.h`` and back.  Importing it raises if the library has not
been built (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhifde.so")

HIFDE_OK, HIFDE_EINVAL, HIFDE_ENOMEM, HIFDE_EDEVICE, HIFDE_ENOTSPD, HIFDE_ENOCONV, HIFDE_ESTATE = (
    0, -1, -2, -3, -4, -5, -6)
HIFDE_FP64, HIFDE_MIXED, HIFDE_MIXED_ELIM64 = 0, 1, 2
HIFDE_USE_RANK_MODEL, HIFDE_DEBUG_DETERMINISM, HIFDE_AUTOTUNE, HIFDE_NO_GRAPH = 1, 4, 8, 16
HIFDE_PRESIZE_WORST_CASE = 64
HIFDE_SWEEP_ROW_TILES = 128
HIFDE_INDEFINITE = 256
HIFDE_SKETCH_ID = 512
HIFDE_RETRY_FP64 = 1024
HIFDE_MAX_LEVELS = 24

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOTSPD",
                -5: "ENOCONV", -6: "ESTATE"}

EXPORTED = [
    "hifde_build_tree", "hifde_factor", "hifde_solve", "hifde_pcg", "hifde_gmres", "hifde_matvec",
    "hifde_stats", "hifde_export_sets", "hifde_plan_replay", "hifde_profile",
    "hifde_profile_read", "hifde_mlp_workspace", "hifde_mlp_forward", "hifde_mlp_grad",
    "hifde_mlp_grad_noalloc", "hifde_mlp_adam", "hifde_rank_features", "hifde_set_rank_model",
    "hifde_tree_set_memory_limit", "hifde_tree_free", "hifde_factor_free", "hifde_last_error",
]

HIFDE_RANK_FEATURES, HIFDE_RANK_HIDDEN = 16, 64
HIFDE_RANK_PARAMS = 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1
HIFDE_MLP_NOALLOC_MAX_BATCH = 8192

HIFDE_PROF_SWEEP_UP, HIFDE_PROF_SWEEP_DOWN, HIFDE_PROF_INTERP, HIFDE_PROF_TOP = 0, 1, 2, 3
HIFDE_PROF_SWEEP_UP_WHOLE, HIFDE_PROF_SWEEP_DOWN_WHOLE = 4, 5
HIFDE_PROF_GROUP_UP, HIFDE_PROF_GROUP_DOWN = 6, 7
HIFDE_PROF_SWEEP_UP_ONE, HIFDE_PROF_CONTRIB_ADD = 8, 9
HIFDE_PROF_CLASSES = 10


class HifdeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Stats(C.Structure):
    _fields_ = [
        ("N", C.c_int64),
        ("dim", C.c_int32),
        ("levels", C.c_int32),
        ("top_size", C.c_int64),
        ("factor_bytes", C.c_int64),
        ("factor_flops", C.c_double),
        ("factor_ms", C.c_double),
        ("solve_bytes", C.c_double),
        ("cells", C.c_int64 * HIFDE_MAX_LEVELS),
        ("groups", C.c_int64 * HIFDE_MAX_LEVELS),
        ("skel_in", C.c_int64 * HIFDE_MAX_LEVELS),
        ("skel_out", C.c_int64 * HIFDE_MAX_LEVELS),
        ("max_front", C.c_int32 * HIFDE_MAX_LEVELS),
        ("rank_groups", C.c_int64),
        ("rank_mae", C.c_double),
        ("rebuckets", C.c_int64),
        ("skel_panels", C.c_int64),
        ("tuned", C.c_int64),
        ("level_ms", C.c_double * HIFDE_MAX_LEVELS),
        ("top_ms", C.c_double),
        ("precision", C.c_int32),
        ("retried", C.c_int32),
    ]


class Prof(C.Structure):
    _fields_ = [
        ("launches", C.c_int64),
        ("ms", C.c_double),
        ("bytes", C.c_double),
        ("flops", C.c_double),
    ]


class Sets(C.Structure):
    _fields_ = [
        ("count", C.c_int64),
        ("total", C.c_int64 * 4),
        ("ids", C.POINTER(C.c_int64)),
        ("offs", C.POINTER(C.c_int64) * 4),
        ("lists", C.POINTER(C.c_int32) * 4),
    ]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with "
                          "`python -m paper_1307_2895_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
    L.hifde_build_tree.argtypes = [i32, i64, i64, i32, C.POINTER(vp)]
    L.hifde_factor.argtypes = [vp, C.POINTER(vp), vp, dbl, i32, C.c_uint32, vp, C.POINTER(vp)]
    L.hifde_solve.argtypes = [vp, i64, vp, i64, vp, i64, vp]
    L.hifde_matvec.argtypes = [vp, i64, vp, i64, vp, i64, vp]
    L.hifde_pcg.argtypes = [vp, i64, vp, i64, vp, i64, dbl, i32, C.POINTER(C.c_int),
                            C.POINTER(C.c_double), vp]
    L.hifde_gmres.argtypes = [vp, i64, vp, i64, vp, i64, dbl, i32, i32, C.POINTER(C.c_int),
                              C.POINTER(C.c_double), vp]
    L.hifde_stats.argtypes = [vp, C.POINTER(Stats)]
    L.hifde_export_sets.argtypes = [vp, i32, C.POINTER(Sets)]
    L.hifde_plan_replay.argtypes = [vp, vp, C.POINTER(vp)]
    L.hifde_profile.argtypes = [vp, C.c_uint32, i32]
    L.hifde_mlp_workspace.argtypes = [i64, C.POINTER(C.c_int64)]
    L.hifde_mlp_forward.argtypes = [vp, i64, vp, vp, vp]
    L.hifde_mlp_grad.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
    L.hifde_mlp_grad_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.hifde_mlp_adam.argtypes = [vp, vp, vp, vp, i64, C.c_float, vp]
    L.hifde_rank_features.argtypes = [vp, i32, vp, vp, i64, C.POINTER(C.c_int64), vp]
    L.hifde_set_rank_model.argtypes = [vp, vp, i64]
    L.hifde_profile_read.argtypes = [vp, i32, C.POINTER(Prof)]
    L.hifde_tree_free.argtypes = [vp]
    L.hifde_tree_set_memory_limit.argtypes = [vp, i64]
    L.hifde_factor_free.argtypes = [vp]
    L.hifde_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name != "hifde_last_error" and name not in ("hifde_tree_free", "hifde_factor_free"):
            getattr(L, name).restype = C.c_int
    L.hifde_tree_free.restype = None
    L.hifde_factor_free.restype = None
    _lib = L
    return L


def check(rc: int):
    if rc != HIFDE_OK:
        msg = lib().hifde_last_error().decode(errors="replace")
        raise HifdeError(rc, msg)
