"""ctypes loader for libblocktransform.so (the C ABI in include/blocktransform.h).

There is no fallback: if the library has not been built, importing the binding
raises, so no other code path can stand in for the HIP kernels.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libblocktransform.so")

TF_OK = 0
TF_EINVAL = -1
TF_EUNSUPPORTED = -2
TF_ESINGULAR = -3
TF_EHIP = -4
TF_EWORKSPACE = -5

TF_FP32 = 0
TF_SPLIT_BF16 = 1
TF_SPLIT_FP16 = 2
TF_PLAIN_FP32 = 3

COMPUTE = {"fp32": TF_FP32, "plain_fp32": TF_PLAIN_FP32, "split_bf16": TF_SPLIT_BF16,
           "split_fp16": TF_SPLIT_FP16}

EXPORTED = (
    "transform_forward", "transform_inverse", "transform_adjoint", "transform_inverse_adjoint",
    "transform_workspace_size", "transform_prepare", "transform_status_string",
    "transform_last_error",
    "transform_schedule_count", "transform_schedule_describe", "transform_schedule_select",
    "transform_schedule_selected",
    "transform_load_schedule", "transform_save_schedule",
    "transform_ragged_plan_create", "transform_ragged_plan_create_ex", "transform_ragged_plan_destroy",
    "transform_ragged_execute", "transform_decimated", "transform_decimated_adjoint",
    "nufft_workspace_size", "nufft_type5", "nufft_type4", "nufft_type5_refined", "nufft_type4_refined",
    "nudft_type1", "nudft_type2", "nufft_workspace_size_ex", "nufft_solve", "nufft_setup", "nufft_apply",
    "nfft_workspace_size",
    "nfft_type1", "nfft_type2", "transform_adjoint_noalloc", "transform_noalloc_scratch_bytes",
    "transform_ragged_prefetch_select", "transform_ragged_prefetch_selected",
)

_lib = None


class TransformError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str = ""):
        self.status = status
        msg = f"{fn} failed: {status_string(status)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    lib.transform_forward.argtypes = [vp, vp, vp, i64, i32, i32, i64, i32, vp, sz, vp]
    lib.transform_inverse.argtypes = [vp, vp, vp, i64, i32, i32, i64, i32, vp, vp, sz, vp]
    lib.transform_adjoint.argtypes = [vp, vp, vp, vp, vp, i64, i32, i32, i64, i32, vp, sz, vp]
    lib.transform_inverse_adjoint.argtypes = [vp, vp, vp, vp, vp, i64, i32, i32, i64, i32, vp, sz, vp]
    lib.transform_adjoint_noalloc.argtypes = [vp, vp, vp, vp, vp, i64, i32, i32, i64, vp]
    lib.transform_noalloc_scratch_bytes.argtypes = []
    lib.transform_noalloc_scratch_bytes.restype = sz
    lib.transform_decimated.argtypes = [vp, vp, vp, i64, i32, i32, i64, vp]
    lib.transform_decimated_adjoint.argtypes = [vp, vp, vp, i64, i32, i32, i64, vp]
    lib.transform_workspace_size.argtypes = [i64, i32, i32, i64, i32, i32]
    lib.transform_workspace_size.restype = sz
    lib.transform_prepare.argtypes = [i32, i32, i32]
    lib.transform_status_string.argtypes = [ctypes.c_int]
    lib.transform_status_string.restype = ctypes.c_char_p
    lib.transform_last_error.argtypes = []
    lib.transform_last_error.restype = ctypes.c_char_p
    lib.transform_schedule_count.argtypes = [i32, i32]
    lib.transform_schedule_describe.argtypes = [i32, i32, i32, ctypes.c_char_p, sz]
    lib.transform_schedule_select.argtypes = [i32, i32, i32, i32]
    lib.transform_schedule_selected.argtypes = [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.transform_load_schedule.argtypes = [ctypes.c_char_p]
    lib.transform_save_schedule.argtypes = [ctypes.c_char_p]
    lib.transform_ragged_plan_create.argtypes = [vp, vp, vp, vp, i64, i64, ctypes.POINTER(vp)]
    lib.transform_ragged_plan_create_ex.argtypes = [vp, vp, vp, vp, i64, i64, i32, ctypes.POINTER(vp)]
    lib.transform_ragged_plan_destroy.argtypes = [vp]
    lib.transform_ragged_execute.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, i32, vp]
    lib.transform_ragged_prefetch_select.argtypes = [i32, i32, i32, i32]
    lib.transform_ragged_prefetch_selected.argtypes = [i32, i32, i32, ctypes.POINTER(i32)]
    lib.nufft_workspace_size.argtypes = [i64, i32, i32]
    lib.nufft_workspace_size.restype = sz
    lib.nufft_type5.argtypes = [vp, vp, vp, i64, i32, i32, ctypes.c_double, vp, sz, vp]
    lib.nufft_type4.argtypes = [vp, vp, vp, i64, i32, i32, ctypes.c_double, vp, sz, vp]
    lib.nufft_type5_refined.argtypes = [vp, vp, vp, i64, i32, i32, ctypes.c_double, vp, sz, vp]
    lib.nufft_type4_refined.argtypes = [vp, vp, vp, i64, i32, i32, ctypes.c_double, vp, sz, vp]
    lib.nudft_type1.argtypes = [vp, vp, vp, i64, i32, i32, vp]
    lib.nufft_workspace_size_ex.argtypes = [i64, i32, i32, i32]
    lib.nufft_workspace_size_ex.restype = sz
    lib.nufft_solve.argtypes = [i32, i32, vp, vp, vp, i64, i32, i32, ctypes.c_double, vp, sz, vp]
    lib.nufft_setup.argtypes = [i32, vp, i64, i32, i32, ctypes.c_double, vp, sz, vp]
    lib.nufft_apply.argtypes = [i32, i32, vp, vp, vp, i64, i32, i32, ctypes.c_double, vp, sz, vp]
    lib.nfft_workspace_size.argtypes = [i64, i32]
    lib.nfft_workspace_size.restype = sz
    lib.nfft_type1.argtypes = [vp, vp, vp, i64, i32, i32, vp, sz, vp]
    lib.nfft_type2.argtypes = [vp, vp, vp, i64, i32, i32, vp, sz, vp]
    lib.nudft_type2.argtypes = [vp, vp, vp, i64, i32, i32, vp]
    for name in EXPORTED:
        f = getattr(lib, name)
        if f.restype is ctypes.c_int:   # default
            f.restype = ctypes.c_int
    _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load().transform_status_string(int(status)).decode()
    except ImportError:
        return str(status)


def check(fn: str, status: int):
    if status != TF_OK:
        detail = ""
        if status == TF_EHIP:
            detail = load().transform_last_error().decode()
        raise TransformError(fn, status, detail)
