"""ctypes declarations of libgemm_mi355x.so (the C ABI in include/gemm_mi355x.h).

Loading fails loudly: there is no fallback path. A missing library raises
``RuntimeError`` naming the build command.
"""
from __future__ import annotations

import ctypes
import os
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgemm_mi355x.so")

GEMM_OK, GEMM_EINVAL, GEMM_ENULL, GEMM_ELD, GEMM_EWORKSPACE = 0, 1, 2, 3, 4
GEMM_EUNSUPPORTED, GEMM_EHIP, GEMM_ENOMEM, GEMM_ESTATE = 5, 6, 7, 8
GEMM_F64, GEMM_F32, GEMM_BF16 = 0, 1, 2
GEMM_PLAN_AUTOTUNE, GEMM_PLAN_NO_GRAPH, GEMM_PLAN_NO_PACK = 1, 2, 4

# every symbol the header declares; the CPU tests check they are exported
EXPORTS = (
    "gemm_plain", "gemm_split_workspace_size", "gemm_split_convert", "gemm_split",
    "gemm_split3_workspace_size", "gemm_split3_convert", "gemm_split3", "gemm_split_one_launch",
    "gemm_backward", "gemm_grouped_plan_create", "gemm_grouped_run",
    "gemm_grouped_plan_update", "gemm_grouped_plan_destroy", "gemm_grouped_plan_info",
    "gemm_grouped", "gemm_strerror", "gemm_last_error", "gemm_tile_config_count",
    "gemm_tile_config_name", "gemm_plain_ksplit_workspace_size", "gemm_plain_ksplit",
    "gemm_plain_ksplit_noalloc",
)
# size of the per-device scratch array of gemm_plain_ksplit_noalloc
# (GEMM_NOALLOC_SCRATCH_BYTES in the header)
NOALLOC_SCRATCH_BYTES = 64 << 20
# the tuning knobs of include/gemm_mi355x_tuning.h (tests and tuning tools)
TUNING_EXPORTS = ("gemm_tuning_force_tile_config", "gemm_tuning_force_ksplit_parts",
                  "gemm_tuning_force_split_form")


class GemmProblem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("lda", ctypes.c_int64), ("ldb", ctypes.c_int64), ("ldc", ctypes.c_int64)]


_lock = threading.Lock()
_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load (once) and declare the library. Raises RuntimeError if absent."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(
                f"{p} is missing: build it with `python -m paper_1012_2273_amd.build` "
                "(hipcc, gfx950); there is no non-HIP fallback")
        lib = ctypes.CDLL(p)
        i64, vp, i32, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
        sz = ctypes.c_size_t
        sig = {
            "gemm_plain": (ci, [ci, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp]),
            "gemm_split_workspace_size": (sz, [i64, i64, i64]),
            "gemm_plain_ksplit_workspace_size": (sz, [ci, i64, i64, i64]),
            "gemm_plain_ksplit": (ci, [ci, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, sz, vp]),
            "gemm_plain_ksplit_noalloc": (ci, [ci, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp]),
            "gemm_tuning_force_ksplit_parts": (ci, [ci]),
            "gemm_tuning_force_split_form": (ci, [ci]),
            "gemm_split_convert": (ci, [i64, i64, vp, i64, ci, vp, vp, i64, vp]),
            "gemm_split": (ci, [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, sz, vp]),
            "gemm_split3_workspace_size": (sz, [i64, i64, i64]),
            "gemm_split3_convert": (ci, [i64, i64, vp, i64, ci, vp, vp, vp, i64, vp]),
            "gemm_split3": (ci, [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, sz, vp]),
            "gemm_split_one_launch": (ci, [i64, i64, i64, vp, i64, vp, i64]),
            "gemm_backward": (ci, [ci, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64,
                                   vp, i64, vp]),
            "gemm_grouped_plan_create": (ci, [ctypes.POINTER(vp), ci, ctypes.POINTER(GemmProblem),
                                              i32, ctypes.c_char_p, ci, vp]),
            "gemm_grouped_run": (ci, [vp, vp]),
            "gemm_grouped_plan_update": (ci, [vp, ctypes.POINTER(GemmProblem), i32]),
            "gemm_grouped_plan_destroy": (ci, [vp]),
            "gemm_grouped_plan_info": (ci, [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), i32]),
            "gemm_grouped": (ci, [ci, ctypes.POINTER(GemmProblem), i32, vp]),
            "gemm_strerror": (ctypes.c_char_p, [ci]),
            "gemm_last_error": (ctypes.c_char_p, []),
            "gemm_tile_config_count": (ci, []),
            "gemm_tile_config_name": (ctypes.c_char_p, [ci]),
            "gemm_tuning_force_tile_config": (ci, [ci]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


class GemmError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {detail or 'error'} (status {status})")
        self.status = status


class GemmArgError(GemmError, ValueError):
    pass


def check(status: int, where: str) -> None:
    if status == GEMM_OK:
        return
    lib = load()
    detail = (lib.gemm_last_error() or b"").decode()
    text = (lib.gemm_strerror(status) or b"").decode()
    msg = f"{text}: {detail}" if detail else text
    if status in (GEMM_EHIP, GEMM_ENOMEM):
        raise GemmError(status, where, msg)
    raise GemmArgError(status, where, msg)
