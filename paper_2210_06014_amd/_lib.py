"""ctypes view of libfastertucker.so (the C-ABI declared in include/fastertucker.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfastertucker.so")
MAX_ORDER = 10

FT_KEEP_HOST = 1
FT_WITH_PERM = 2
FT_NO_FIBER_SHARE = 4
FT_NO_C_CACHE = 8
FT_RELAXED = 16
FT_SPLIT_FACTOR = 32
FT_RUN_REUSE = 64

STATUS = {
    0: "FT_OK",
    1: "FT_ERR_ARG",
    2: "FT_ERR_SHAPE",
    3: "FT_ERR_INDEX",
    4: "FT_ERR_UNSUPPORTED",
    5: "FT_ERR_STATE",
    6: "FT_ERR_NOMEM",
    7: "FT_ERR_HIP",
    8: "FT_ERR_WORKSPACE",
}

# every entry point of include/fastertucker.h
SYMBOLS = [
    "ft_plan_create",
    "ft_plan_query",
    "ft_plan_upload",
    "ft_plan_destroy",
    "ft_plan_mode_info",
    "ft_plan_host_csr",
    "ft_refresh",
    "ft_predict",
    "ft_factor_pass",
    "ft_factor_epoch",
    "ft_core_grad",
    "ft_core_pass",
    "ft_core_epoch",
    "ft_epoch",
    "ft_loss",
    "ft_loss_noalloc",
    "ft_forward",
    "ft_grad",
    "ft_profile_enable",
    "ft_profile_read",
    "ft_status_str",
    "ft_last_error",
    "ft_supported",
]


class FtDesc(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("dims", ctypes.c_int64 * MAX_ORDER),
        ("J", ctypes.c_int32 * MAX_ORDER),
        ("R", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("chunk", ctypes.c_int32),
        ("head", ctypes.c_int32),
        ("fanin", ctypes.c_int32),
        ("flags", ctypes.c_int32),
    ]


FT_STORE_F32 = 0
FT_STORE_BF16 = 1


class FtParams(ctypes.Structure):
    _fields_ = [
        ("A", ctypes.c_void_p * MAX_ORDER),
        ("B", ctypes.c_void_p * MAX_ORDER),
        ("C", ctypes.c_void_p * MAX_ORDER),
        ("A16", ctypes.c_void_p * MAX_ORDER),
        ("B16", ctypes.c_void_p * MAX_ORDER),
        ("C16", ctypes.c_void_p * MAX_ORDER),
        ("storage", ctypes.c_int32),
        ("scratch", ctypes.c_void_p),
        ("scratch_bytes", ctypes.c_size_t),
    ]


class FtModeInfo(ctypes.Structure):
    _fields_ = [
        ("rows", ctypes.c_int64),
        ("nonempty_rows", ctypes.c_int64),
        ("max_row", ctypes.c_int64),
        ("light_rows", ctypes.c_int64),
        ("heavy_rows", ctypes.c_int64),
        ("chunks", ctypes.c_int64),
        ("segments", ctypes.c_int64),
        ("combine_levels", ctypes.c_int32),
        ("fiber_shared", ctypes.c_int32),
        ("fibers", ctypes.c_int64),
        ("head", ctypes.c_int32),
        ("chunk", ctypes.c_int32),
        ("runs", ctypes.c_int64),
    ]


KERNELS = ["factor_compose", "factor_apply", "combine", "refresh", "segsum", "reduce", "loss", "fiber_g",
           "factor_fused"]


class FtError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def load():
    """Load the HIP library; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_2210_06014_amd/build.py`"
        )
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "ft_plan_create": ([P(vp), P(FtDesc), vp, vp], i32),
        "ft_plan_query": ([vp, P(ctypes.c_size_t), P(ctypes.c_size_t)], i32),
        "ft_plan_upload": ([vp, vp, ctypes.c_size_t, vp], i32),
        "ft_plan_destroy": ([vp], None),
        "ft_plan_mode_info": ([vp, i32, P(FtModeInfo)], i32),
        "ft_plan_host_csr": ([vp, i32, i32, vp, vp, vp, vp], i32),
        "ft_refresh": ([vp, P(FtParams), i32, vp], i32),
        "ft_predict": ([vp, P(FtParams), vp, i64, vp, vp], i32),
        "ft_factor_pass": ([vp, P(FtParams), i32, dbl, dbl, vp], i32),
        "ft_factor_epoch": ([vp, P(FtParams), dbl, dbl, vp], i32),
        "ft_core_grad": ([vp, P(FtParams), i32, vp, vp], i32),
        "ft_core_pass": ([vp, P(FtParams), i32, dbl, dbl, vp], i32),
        "ft_core_epoch": ([vp, P(FtParams), dbl, dbl, vp], i32),
        "ft_epoch": ([vp, P(FtParams), dbl, dbl, dbl, dbl, vp], i32),
        "ft_loss": ([vp, P(FtParams), dbl, dbl, vp, vp], i32),
        "ft_loss_noalloc": ([vp, P(FtParams), dbl, dbl, vp, vp], i32),
        "ft_forward": ([vp, P(FtParams), vp, vp], i32),
        "ft_grad": ([vp, P(FtParams), vp, vp, vp, vp], i32),
        "ft_profile_enable": ([vp, i32], i32),
        "ft_profile_read": ([vp, vp, vp], i32),
        "ft_status_str": ([i32], ctypes.c_char_p),
        "ft_last_error": ([], ctypes.c_char_p),
        "ft_supported": ([i32, i32, i32], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def check(status: int):
    if status != 0:
        msg = load().ft_last_error()
        raise FtError(status, msg.decode() if msg else "")
