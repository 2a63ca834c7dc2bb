"""ctypes declarations of libpiv.so (the C ABI in include/piv.h).

Argument marshalling only: every step of the PIV path runs in the HIP
kernels behind these entry points.  Loading fails loudly when the library
has not been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpiv.so")

PIV_OK, PIV_EINVAL, PIV_EUNSUPPORTED, PIV_ENOWORKSPACE, PIV_EDEVICE = 0, 1, 2, 3, 4
PIV_U8, PIV_U16, PIV_F32 = 1, 2, 3
PIV_WARP_B, PIV_WARP_CENTRAL = 0, 1
NOALLOC_SCRATCH_BYTES = 64 << 20   # PIV_NOALLOC_SCRATCH_BYTES
PIV_PEAK_ARGMAX, PIV_PEAK_FIXED_CENTER = 0, 1
F_FLAT, F_BORDER, F_NOCURV, F_OUTLIER, F_REPLACED, F_UNRESOLVED = 1, 2, 4, 8, 16, 32

#: every symbol include/piv.h declares
EXPORTS = [
    "piv_params_default", "piv_plan", "piv_plan_grid", "piv_plan_workspace_bytes",
    "piv_plan_bind_workspace", "piv_plan_bind_slot_mask", "piv_plan_destroy", "piv_predict",
    "piv_correct", "piv_validate", "piv_vorticity", "piv_run", "piv_run_noalloc", "piv_smooth",
    "piv_run_temporal", "piv_highpass", "piv_clahe_lut_bytes", "piv_clahe",
    "piv_ssd_forward", "piv_ssd_backward", "piv_ssd_refine", "piv_status_string", "piv_last_error",
    "piv_debug_correct_impl", "piv_debug_level",
]


class Params(C.Structure):
    _fields_ = [
        ("width", C.c_int32), ("height", C.c_int32), ("max_batch", C.c_int32),
        ("dtype", C.c_int), ("bit_depth", C.c_int32),
        ("win", C.c_int32), ("step", C.c_int32), ("radius", C.c_int32),
        ("levels", C.c_int32), ("block", C.c_int32), ("radius_coarse", C.c_int32),
        ("radius_fine", C.c_int32), ("median", C.c_int32),
        ("warp", C.c_int), ("peak", C.c_int),
        ("uod_threshold", C.c_float), ("uod_epsilon", C.c_float),
        ("sgm", C.c_int32), ("sgm_p1", C.c_int32), ("sgm_p2", C.c_int32),
    ]


class PivError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{status_name(status)}: {detail}")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2504_17987_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, vp, i32, i64, st = C.POINTER(Params), C.c_void_p, C.c_int32, C.c_int64, C.c_int
        L.piv_params_default.argtypes = [P]
        L.piv_params_default.restype = None
        L.piv_plan.argtypes = [P, C.POINTER(vp)]
        L.piv_plan_grid.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.piv_plan_workspace_bytes.argtypes = [vp, i32]
        L.piv_plan_workspace_bytes.restype = C.c_size_t
        L.piv_plan_bind_workspace.argtypes = [vp, vp, C.c_size_t, vp]
        L.piv_plan_bind_slot_mask.argtypes = [vp, vp]
        L.piv_plan_destroy.argtypes = [vp]
        L.piv_plan_destroy.restype = None
        L.piv_predict.argtypes = [vp, vp, vp, i64, i32, vp, vp]
        L.piv_correct.argtypes = [vp, vp, vp, i64, i32, vp, vp, vp, vp, vp]
        L.piv_validate.argtypes = [vp, vp, vp, i32, vp]
        L.piv_vorticity.argtypes = [vp, vp, vp, i32, vp]
        L.piv_run.argtypes = [vp, vp, vp, i64, i32, vp, vp, vp, vp, vp, vp]
        L.piv_run_noalloc.argtypes = [vp, vp, vp, i64, i32, vp, vp, vp, vp, vp, vp]
        L.piv_ssd_forward.argtypes = [vp, vp, vp, vp, i32, vp, vp]
        L.piv_ssd_backward.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, vp]
        f32 = C.c_float
        L.piv_smooth.argtypes = [vp, vp, vp, vp, i32, f32, i32, vp]
        L.piv_run_temporal.argtypes = [vp, vp, vp, i64, i32, vp, i32, vp, vp, f32, f32, vp, vp, vp, vp, vp, vp]
        L.piv_ssd_refine.argtypes = [vp, vp, vp, vp, i32, i32, f32, f32, vp, vp]
        L.piv_highpass.argtypes = [vp, vp, vp, i64, i32, i32, vp]
        L.piv_clahe_lut_bytes.argtypes = [vp, i32, i32, i32]
        L.piv_clahe_lut_bytes.restype = C.c_size_t
        L.piv_clahe.argtypes = [vp, vp, vp, i64, i32, i32, i32, C.c_double, vp, C.c_size_t, vp]
        for name in ["piv_plan", "piv_plan_grid", "piv_plan_bind_workspace", "piv_plan_bind_slot_mask",
                     "piv_predict", "piv_correct", "piv_validate", "piv_vorticity", "piv_run",
                     "piv_run_noalloc", "piv_smooth", "piv_run_temporal", "piv_ssd_forward", "piv_ssd_backward",
                     "piv_ssd_refine", "piv_highpass", "piv_clahe"]:
            getattr(L, name).restype = st
        L.piv_status_string.argtypes = [st]
        L.piv_status_string.restype = C.c_char_p
        L.piv_last_error.argtypes = []
        L.piv_last_error.restype = C.c_char_p
        L.piv_debug_correct_impl.argtypes = [vp]
        L.piv_debug_correct_impl.restype = C.c_int
        L.piv_debug_level.argtypes = [vp, i32, C.POINTER(i32)]
        L.piv_debug_level.restype = C.c_int
        _lib = L
    return _lib


def status_name(s: int) -> str:
    return lib().piv_status_string(s).decode()


def check(status: int) -> None:
    if status != PIV_OK:
        raise PivError(status, lib().piv_last_error().decode())
