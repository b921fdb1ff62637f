"""ctypes binding of libksc.so (argument marshalling only; include/ksc.h
documents every call)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libksc.so")

KSC_OK = 0
STATUS_NAMES = {
    0: "KSC_OK", -1: "KSC_ERR_ARG", -2: "KSC_ERR_SHAPE", -3: "KSC_ERR_UNSUPPORTED",
    -4: "KSC_ERR_HIP", -5: "KSC_ERR_NONFINITE", -6: "KSC_ERR_DIVERGED", -7: "KSC_ERR_STATE",
}
KSC_F32, KSC_F64 = 0, 1
KSC_SPACE_FULL, KSC_SPACE_ODD = 0, 1
KSC_DS_STENCIL, KSC_DS_SPECTRAL = 0, 1
KSC_MAP_RATIONAL, KSC_MAP_FINITE = 0, 1
KSC_FLAG_NONFINITE, KSC_FLAG_INCREASED = 1, 2
KSC_LAUNCH_AUTO, KSC_LAUNCH_PLAIN, KSC_LAUNCH_PERSISTENT = 0, 1, 2
KSC_SCHEME_PAPER, KSC_SCHEME_IMPLICIT_S = 0, 1
KSC_NOALLOC_SCRATCH_BYTES = 8 << 20

# Every symbol include/ksc.h declares.
EXPORTED = (
    "ksc_create", "ksc_create2", "ksc_create_opts", "ksc_destroy", "ksc_set_stream", "ksc_state_numel", "ksc_state_offset",
    "ksc_phys_numel", "ksc_phys_offset", "ksc_n_modes", "ksc_set_endpoints",
    "ksc_phys_to_spec", "ksc_spec_to_phys", "ksc_eval_J", "ksc_eval_grad", "ksc_step",
    "ksc_descend", "ksc_tune", "ksc_set_launch", "ksc_get_launch", "ksc_query_flags",
    "ksc_set_timing", "ksc_read_timing", "ksc_set_scheme", "ksc_get_scheme", "ksc_set_momentum",
    "ksc_get_momentum", "ksc_precondition", "ksc_eval_J_noalloc", "ksc_last_error",
)


class KscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class CurveDescC(ctypes.Structure):
    _fields_ = [
        ("n_s", ctypes.c_int32),
        ("n_x", ctypes.c_int32),
        ("L", ctypes.c_double),
        ("map", ctypes.c_int32),
        ("scale", ctypes.c_double),
        ("s0", ctypes.c_double),
    ]


class OptionsC(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32),
        ("space", ctypes.c_int32),
        ("ds", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libksc.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2301_11704_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "ksc_create": (i32, [ctypes.POINTER(CurveDescC), i32, i32, vp, ctypes.POINTER(vp)]),
        "ksc_create2": (i32, [ctypes.POINTER(CurveDescC), i32, i32, i32, vp, ctypes.POINTER(vp)]),
        "ksc_create_opts": (i32, [ctypes.POINTER(CurveDescC), i32, ctypes.POINTER(OptionsC), vp,
                                  ctypes.POINTER(vp)]),
        "ksc_destroy": (i32, [vp]),
        "ksc_set_stream": (i32, [vp, vp]),
        "ksc_state_numel": (i64, [vp]),
        "ksc_state_offset": (i64, [vp, i32]),
        "ksc_phys_numel": (i64, [vp]),
        "ksc_phys_offset": (i64, [vp, i32]),
        "ksc_n_modes": (i32, [i32]),
        "ksc_set_endpoints": (i32, [vp, vp, i32, vp, vp]),
        "ksc_phys_to_spec": (i32, [vp, vp, vp]),
        "ksc_spec_to_phys": (i32, [vp, vp, vp]),
        "ksc_eval_J": (i32, [vp, vp, vp, vp]),
        "ksc_eval_grad": (i32, [vp, vp, vp, vp, vp]),
        "ksc_step": (i32, [vp, vp, vp, dbl, vp]),
        "ksc_descend": (i32, [vp, vp, vp, i64, dbl, vp, i32, vp]),
        "ksc_tune": (i32, [vp, ctypes.c_char_p]),
        "ksc_set_launch": (i32, [vp, i32, i32]),
        "ksc_get_launch": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "ksc_set_scheme": (i32, [vp, i32]),
        "ksc_get_scheme": (i32, [vp, ctypes.POINTER(i32)]),
        "ksc_set_momentum": (i32, [vp, dbl]),
        "ksc_precondition": (i32, [vp, vp, vp, dbl]),
        "ksc_get_momentum": (i32, [vp, ctypes.POINTER(dbl)]),
        "ksc_query_flags": (i32, [vp, ctypes.POINTER(ctypes.c_uint32)]),
        "ksc_set_timing": (i32, [vp, i32]),
        "ksc_read_timing": (i32, [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                  ctypes.POINTER(i64)]),
        "ksc_eval_J_noalloc": (i32, [ctypes.POINTER(CurveDescC), i32, i32, vp, vp, vp]),
        "ksc_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status: int) -> None:
    if status != KSC_OK:
        msg = lib().ksc_last_error().decode(errors="replace")
        raise KscError(status, msg)
