"""ctypes declarations of librtsgrid.so (the C ABI in include/rtsgrid.h).

Argument marshalling only.  Loading fails loudly when the library has not been
built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librtsgrid.so")

RTS_OK, RTS_E_INVALID, RTS_E_NOMEM, RTS_E_HIP, RTS_E_UNSUPPORTED = range(5)
STATUS_NAMES = {0: "RTS_OK", 1: "RTS_E_INVALID", 2: "RTS_E_NOMEM", 3: "RTS_E_HIP", 4: "RTS_E_UNSUPPORTED"}

EXPORTED = (
    "rts_grid_plan", "rts_plan_update", "rts_grid", "rts_degrid", "rts_grid_degrid", "rts_compute_coords",
    "rts_cadence_graph_create", "rts_cadence_graph_launch", "rts_cadence_graph_destroy", "rts_autotune_tile",
    "rts_plan_valid_mask", "rts_image", "rts_polconvert", "rts_plan_set_baseline_kernels", "rts_plan_get_table",
    "rts_plan_get_info", "rts_plan_destroy", "rts_last_error", "rts_version", "rts_stream_copy",
    "rts_grid_backward", "rts_chi2_backward", "rts_grid_degrid_noalloc",
)


class RtsParams(ctypes.Structure):
    _fields_ = [
        ("n_grid", ctypes.c_int32), ("support", ctypes.c_int32), ("oversample", ctypes.c_int32),
        ("n_chan", ctypes.c_int32), ("n_base", ctypes.c_int32), ("n_time", ctypes.c_int32),
        ("cell_lambda", ctypes.c_double), ("beta", ctypes.c_double),
        ("conjugate", ctypes.c_int32), ("tile", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
    ]


class RtsPlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_samples", ctypes.c_int64), ("n_valid", ctypes.c_int64), ("n_flagged", ctypes.c_int64),
        ("n_offgrid", ctypes.c_int64), ("n_segments", ctypes.c_int64), ("n_listings", ctypes.c_int64),
        ("n_dropped", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64), ("tile", ctypes.c_int32), ("seg_max", ctypes.c_int32),
    ]


class RtsError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load librtsgrid.so (built in place by paper_1003_5575_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1003_5575_amd.build` first "
                          "(there is no non-HIP fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.rts_grid_plan.argtypes = [ctypes.POINTER(P), ctypes.POINTER(RtsParams), P, P, P, P]
    lib.rts_plan_update.argtypes = [P, P, P, P]
    lib.rts_grid.argtypes = [P, P, P, P, P]
    lib.rts_degrid.argtypes = [P, P, P, P]
    lib.rts_grid_degrid.argtypes = [P, P, P, P, P, P, P, P]
    lib.rts_compute_coords.argtypes = [ctypes.POINTER(RtsParams), P, P, P, P, P]
    lib.rts_grid_degrid_noalloc.argtypes = [ctypes.POINTER(RtsParams), P, P, P, P, P, P, P, P, P]
    lib.rts_plan_valid_mask.argtypes = [P, P, P]
    lib.rts_polconvert.argtypes = [P, P, P, I64, ctypes.c_int32, I64, P]
    lib.rts_plan_set_baseline_kernels.argtypes = [P, P, P]
    lib.rts_stream_copy.argtypes = [P, P, I64, P]
    lib.rts_grid_backward.argtypes = [P, P, P, P, P, P, P]
    lib.rts_chi2_backward.argtypes = [P, P, P, P, P, P, P, P, P, P]
    lib.rts_cadence_graph_create.argtypes = [ctypes.POINTER(P), P, P, P, P, P, P, P, P, P]
    lib.rts_cadence_graph_launch.argtypes = [P, P]
    lib.rts_cadence_graph_destroy.argtypes = [P]
    lib.rts_autotune_tile.argtypes = [ctypes.POINTER(RtsParams), P, P, P, P, P, P, P, P, P, ctypes.c_int32, P]
    lib.rts_plan_get_table.argtypes = [P, P, I64]
    lib.rts_plan_get_info.argtypes = [P, ctypes.POINTER(RtsPlanInfo)]
    lib.rts_plan_destroy.argtypes = [P]
    for name in ("rts_cadence_graph_create", "rts_cadence_graph_launch", "rts_cadence_graph_destroy",
                 "rts_autotune_tile", "rts_grid_plan", "rts_plan_update", "rts_grid", "rts_degrid", "rts_grid_degrid", "rts_compute_coords",
                 "rts_cadence_graph_create", "rts_cadence_graph_launch", "rts_cadence_graph_destroy", "rts_autotune_tile",
    "rts_plan_valid_mask", "rts_image", "rts_polconvert", "rts_plan_set_baseline_kernels", "rts_plan_get_table",
    "rts_plan_get_info", "rts_plan_destroy", "rts_stream_copy", "rts_grid_backward", "rts_chi2_backward",
                 "rts_grid_degrid_noalloc"):
        getattr(lib, name).restype = I
    lib.rts_last_error.restype = ctypes.c_char_p
    lib.rts_last_error.argtypes = []
    lib.rts_version.restype = ctypes.c_char_p
    lib.rts_version.argtypes = []
    del D
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != RTS_OK:
        msg = load().rts_last_error().decode(errors="replace")
        raise RtsError(status, where, msg)
