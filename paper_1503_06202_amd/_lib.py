"""ctypes view of ``libxeng.so`` (the C ABI declared in ``include/xeng.h``).

Argument marshalling only: every step of the correlation runs in the HIP
library.  Importing this module fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes
import os

# the in-tree library; XENG_LIBRARY names another build of the same sources
# (the host-sanitizer build that the CPU tests load in a child process)
LIB_PATH = os.environ.get("XENG_LIBRARY") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libxeng.so")

XENG_OK = 0
XENG_EINVAL = -1
XENG_EPLAN = -2
XENG_EOVERFLOW = -3
XENG_EHIP = -4
XENG_ENOMEM = -5
XENG_ELIMIT = -6

XENG_FORM_I8 = 0
XENG_FORM_F8 = 1
XENG_ACCUMULATE = 1 << 8
XENG_SHARED_VIS = 1 << 9

XENG_T_EXACT_MAX = (1 << 24) - 1
XENG_N_MAX = 32768
XENG_BEAMS_MAX = 1024
XENG_F8_FLUSH_MAX = 32768
XENG_I8_SEG_MAX = 524288
XENG_G_MAX = 65536
XENG_NOALLOC_INST_MAX = 64
XENG_NOALLOC_ITEMS_MAX = 65536

# every symbol include/xeng.h declares
EXPORTS = (
    "xeng_version", "xeng_strerror", "xeng_plan", "xeng_correlate", "xeng_plan_set_tuning",
    "xeng_destroy", "xeng_plan_error", "xeng_plan_batch", "xeng_correlate_batch",
    "xeng_correlate_batch_graph", "xeng_plan_gated", "xeng_correlate_gated",
    "xeng_plan_set_delays", "xeng_plan_flagged", "xeng_correlate_flagged", "xeng_normalize",
    "xeng_plan_beams", "xeng_beam_set_weights", "xeng_beamform", "xeng_correlate_batch_noalloc",
)


class XengInstance(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("F", ctypes.c_int), ("T", ctypes.c_int),
                ("split_t", ctypes.c_int)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1503_06202_amd.build` "
            "(there is no fallback path)")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    ci = ctypes.c_int
    L.xeng_version.restype = ci
    L.xeng_strerror.argtypes = [ci]
    L.xeng_strerror.restype = ctypes.c_char_p
    L.xeng_plan.argtypes = [ctypes.POINTER(vp), ci, ci, ci, ctypes.c_uint]
    L.xeng_plan.restype = ci
    L.xeng_correlate.argtypes = [vp, vp, ci, ci, ci, vp, vp]
    L.xeng_correlate.restype = ci
    L.xeng_plan_set_tuning.argtypes = [vp, ci, ci]
    L.xeng_plan_set_tuning.restype = ci
    L.xeng_destroy.argtypes = [vp]
    L.xeng_destroy.restype = ci
    L.xeng_plan_error.argtypes = [vp]
    L.xeng_plan_error.restype = ctypes.c_char_p
    L.xeng_plan_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(XengInstance), ci,
                                  ctypes.c_uint]
    L.xeng_plan_batch.restype = ci
    L.xeng_correlate_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.xeng_correlate_batch.restype = ci
    L.xeng_correlate_batch_graph.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.xeng_correlate_batch_graph.restype = ci
    L.xeng_plan_gated.argtypes = [ctypes.POINTER(vp), ci, ci, ci, ci, ctypes.c_uint]
    L.xeng_plan_gated.restype = ci
    L.xeng_correlate_gated.argtypes = [vp, vp, ci, ci, ci, ctypes.POINTER(ctypes.c_int32), ci,
                                       vp, vp]
    L.xeng_correlate_gated.restype = ci
    L.xeng_plan_set_delays.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ci]
    L.xeng_plan_set_delays.restype = ci
    L.xeng_plan_flagged.argtypes = [ctypes.POINTER(vp), ci, ci, ci, ctypes.c_uint]
    L.xeng_plan_flagged.restype = ci
    L.xeng_correlate_flagged.argtypes = [vp, vp, vp, ci, ci, ci, vp, vp, vp]
    L.xeng_correlate_flagged.restype = ci
    L.xeng_normalize.argtypes = [vp, vp, vp, ctypes.c_double, vp, vp]
    L.xeng_normalize.restype = ci
    L.xeng_plan_beams.argtypes = [ctypes.POINTER(vp), ci, ci, ci, ci, ctypes.c_uint]
    L.xeng_plan_beams.restype = ci
    L.xeng_beam_set_weights.argtypes = [vp, ctypes.POINTER(ctypes.c_int8)]
    L.xeng_beam_set_weights.restype = ci
    L.xeng_beamform.argtypes = [vp, vp, ci, ci, ci, vp, vp]
    L.xeng_beamform.restype = ci
    L.xeng_correlate_batch_noalloc.argtypes = [ctypes.POINTER(XengInstance), ci, ctypes.c_uint,
                                               ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.xeng_correlate_batch_noalloc.restype = ci
    _lib = L
    return L


class XengError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        text = lib().xeng_strerror(code).decode()
        super().__init__(f"{where}: {text} ({code})" + (f": {detail}" if detail else ""))


def check(code: int, where: str, plan: int | None = None) -> None:
    if code != XENG_OK:
        detail = ""
        if plan and code == XENG_EHIP:
            detail = lib().xeng_plan_error(plan).decode()
        raise XengError(code, where, detail)
