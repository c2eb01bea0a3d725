"""ctypes declarations of the C ABI in ``include/fmm.h`` (argument
marshalling only; every computation happens in ``libfmm.so``)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfmm.so")

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EDEVICE, FMM_ENOTSUP, FMM_ESTATE = range(6)
STATUS_NAMES = {0: "FMM_OK", 1: "FMM_EINVAL", 2: "FMM_ENOMEM", 3: "FMM_EDEVICE",
                4: "FMM_ENOTSUP", 5: "FMM_ESTATE"}
FMM_FP64, FMM_FP32 = 0, 1
FMM_MIN_ORDER, FMM_MAX_ORDER = 1, 10
FMM_PLAN_NO_WORKSPACE = 1
FMM_NOALLOC_MAX_BYTES = 128 << 20
FMM_TIE_SOURCE, FMM_TIE_TARGET = 0, 1
FMM_LISTS_CROSS_LEVEL, FMM_LISTS_SAME_LEVEL = 0, 1
FMM_NSTAGES = 7
STAGES = ("sort", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p")


class FmmParams(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("leaf_max", ctypes.c_int),
                ("splits", ctypes.c_int), ("theta", ctypes.c_double),
                ("max_depth", ctypes.c_int), ("precision", ctypes.c_int),
                ("tie_refine", ctypes.c_int), ("max_rhs", ctypes.c_int),
                ("lists", ctypes.c_int)]


class FmmPlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("depth", ctypes.c_int32),
                ("splits", ctypes.c_int32), ("nbox", ctypes.c_int64),
                ("nleaf", ctypes.c_int64), ("n_m2l", ctypes.c_int64),
                ("n_p2p", ctypes.c_int64), ("p2p_interactions", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("p2p_items", ctypes.c_int64)]


class FmmTiles(ctypes.Structure):
    _fields_ = [("p2p_groups", ctypes.c_int), ("leaves_per_wave", ctypes.c_int),
                ("m2l_waves", ctypes.c_int), ("chain_waves", ctypes.c_int),
                ("near_stream", ctypes.c_int), ("batch_p2p_waves", ctypes.c_int)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class FmmAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class FMMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "python -m paper_2511_15269_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i64p, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
        L.fmm_abi_version.restype = ctypes.c_int
        L.fmm_last_error.restype = ctypes.c_char_p
        L.fmm_plan_create.argtypes = [vp, i64, ctypes.POINTER(FmmParams), vp, ctypes.POINTER(vp)]
        L.fmm_plan_create_ex.argtypes = [vp, i64, ctypes.POINTER(FmmParams),
                                         ctypes.POINTER(FmmAllocator), ctypes.c_uint, vp,
                                         ctypes.POINTER(vp)]
        L.fmm_multi_plan_create_ex.argtypes = [vp, i64p, ctypes.c_int, ctypes.POINTER(FmmParams),
                                               ctypes.POINTER(FmmAllocator), ctypes.c_uint, vp,
                                               ctypes.POINTER(vp)]
        L.fmm_plan_workspace_bytes.argtypes = [i64, ctypes.POINTER(FmmParams), i64p]
        L.fmm_evaluate_noalloc.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp]
        L.fmm_plan_create_st.argtypes = [vp, i64, vp, i64, ctypes.POINTER(FmmParams),
                                         ctypes.POINTER(FmmAllocator), ctypes.c_uint, vp,
                                         ctypes.POINTER(vp)]
        L.fmm_plan_get_info.argtypes = [vp, ctypes.POINTER(FmmPlanInfo)]
        L.fmm_evaluate.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp]
        L.fmm_plan_get_tree.argtypes = [vp, i64p, i64p, dp, dp]
        L.fmm_plan_get_lists.argtypes = [vp, i64p, i64p, i64p, i64p]
        L.fmm_plan_destroy.argtypes = [vp]
        L.fmm_direct.argtypes = [vp, i64, vp, ctypes.c_int, vp, i64, vp, vp, vp]
        L.fmm_evaluate_transposed.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp]
        L.fmm_adjoint.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp, vp, vp]
        L.fmm_plan_set_profiling.argtypes = [vp, ctypes.c_int]
        L.fmm_plan_read_profile.argtypes = [vp, dp, i64p]
        L.fmm_multi_plan_create.argtypes = [vp, i64p, ctypes.c_int, ctypes.POINTER(FmmParams),
                                            vp, ctypes.POINTER(vp)]
        L.fmm_graph_create.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp, vp,
                                       ctypes.POINTER(vp)]
        L.fmm_graph_launch.argtypes = [vp, vp]
        L.fmm_graph_destroy.argtypes = [vp]
        L.fmm_plan_autotune.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int)]
        L.fmm_plan_set_tiles.argtypes = [vp, ctypes.POINTER(FmmTiles)]
        L.fmm_plan_get_tiles.argtypes = [vp, ctypes.POINTER(FmmTiles)]
        for f in ("fmm_plan_set_tiles", "fmm_plan_get_tiles", "fmm_plan_create", "fmm_plan_get_info", "fmm_evaluate",
                  "fmm_plan_get_tree", "fmm_plan_get_lists", "fmm_plan_destroy",
                  "fmm_direct", "fmm_plan_set_profiling", "fmm_plan_read_profile",
                  "fmm_evaluate_transposed", "fmm_adjoint", "fmm_multi_plan_create",
                  "fmm_graph_create", "fmm_graph_launch", "fmm_graph_destroy",
                  "fmm_plan_autotune", "fmm_plan_create_ex", "fmm_multi_plan_create_ex",
                  "fmm_plan_workspace_bytes", "fmm_plan_create_st", "fmm_evaluate_noalloc"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != FMM_OK:
        raise FMMError(status, lib().fmm_last_error().decode())
