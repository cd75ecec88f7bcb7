"""ctypes binding of libspeedysplat.so (the C ABI in include/speedysplat.h).

Argument marshalling only: every stage of the render runs in the library's HIP
kernels.  torch is imported first so that the library binds to the HIP runtime
torch already loaded (both carry the soname libamdhip64.so.7).  A missing or
stale library is an error; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must be loaded before the library, see above)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspeedysplat.so")

SS_OK, SS_ERR_INVALID_ARG, SS_ERR_WORKSPACE, SS_ERR_OVERFLOW, SS_ERR_HIP = range(5)
MODES = {"3sigma": 0, "snugbox": 1, "accutile": 2}

_vp = ctypes.c_void_p
_c_float_p = ctypes.POINTER(ctypes.c_float)


class SSConstants(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("t_min", ctypes.c_float), ("dilation", ctypes.c_float),
                ("fov_clamp", ctypes.c_float), ("disc_floor", ctypes.c_float)]


class SSCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("near_z", ctypes.c_float), ("bg", ctypes.c_float * 3)]


class SSGaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32),
                ("sh_stride", ctypes.c_int32), ("means", _vp), ("scales", _vp), ("quats", _vp),
                ("opacity", _vp), ("sh", _vp)]


class SSFrame(ctypes.Structure):
    _fields_ = [("geom", _vp), ("conic", _vp), ("rgb", _vp), ("counts", _vp),
                ("depth_keys", _vp), ("order", _vp), ("order_counts", _vp), ("order_tmp", _vp),
                ("tile_sets", _vp), ("offsets", _vp), ("scan_tmp", _vp), ("totals", _vp),
                ("ranges", _vp), ("t_final", _vp), ("n_last", _vp), ("n_eval", _vp),
                ("n_contrib", _vp), ("emit_tmp", _vp), ("table", _vp)]


class SSFrameInfo(ctypes.Structure):
    _fields_ = [("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                ("n_tiles", ctypes.c_int32), ("sort_bits", ctypes.c_int32),
                ("scan_tmp_words", ctypes.c_int64), ("order_tmp_words", ctypes.c_int64),
                ("emit_tmp_words", ctypes.c_int64), ("table_bytes", ctypes.c_int64)]


class SSFrameCounts(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_uint64), ("n_visible", ctypes.c_uint64)]


class SSBatchItem(ctypes.Structure):
    _fields_ = [("cam", SSCamera), ("g", SSGaussians), ("out_rgb", _vp)]


class SSBatchInfo(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int64), ("n_pixels", ctypes.c_int64),
                ("n_tiles", ctypes.c_int32), ("sort_bits", ctypes.c_int32),
                ("scan_tmp_words", ctypes.c_int64), ("order_tmp_words", ctypes.c_int64),
                ("emit_tmp_words", ctypes.c_int64), ("table_bytes", ctypes.c_int64)]


class SSPairs(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_uint64), ("keys", _vp * 2), ("values", _vp * 2),
                ("sort_tmp", _vp)]


class SSGrads(ctypes.Structure):
    _fields_ = [("means", _vp), ("scales", _vp), ("quats", _vp), ("opacity", _vp), ("sh", _vp),
                ("g2d", _vp), ("score", _vp)]


class SSStageEvents(ctypes.Structure):
    _fields_ = [("ev", _vp * 9)]


# Exported symbols and their prototypes (restype c_int unless noted).
_P = ctypes.POINTER
PROTOTYPES = {
    "ss_get_constants": [_P(SSConstants)],
    "ss_status_string": [ctypes.c_int],
    "ss_last_error": [],
    "ss_frame_sizes": [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P(SSFrameInfo)],
    "ss_sort_tmp_words": [ctypes.c_uint64, _P(ctypes.c_int64)],
    "ss_preprocess": [_P(SSCamera), _P(SSGaussians), ctypes.c_int32, _P(SSFrame), _vp],
    "ss_depth_order": [ctypes.c_int64, ctypes.c_int64, _P(SSFrame), _vp],
    "ss_scan": [ctypes.c_int64, _P(SSFrame), _vp],
    "ss_emit": [_P(SSCamera), ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _P(SSFrame),
                _P(SSPairs), ctypes.c_int32, ctypes.c_uint64, _vp],
    "ss_sort": [_P(SSCamera), _P(SSPairs), ctypes.c_int32, ctypes.c_uint64,
                _P(ctypes.c_int32), _vp],
    "ss_sort_noalloc": [_P(SSCamera), _P(SSPairs), ctypes.c_int32, ctypes.c_uint64,
                        _P(ctypes.c_int32), _vp],
    "ss_ranges": [_P(SSCamera), _P(SSFrame), _P(SSPairs), ctypes.c_int32, ctypes.c_uint64, _vp],
    "ss_blend": [_P(SSCamera), _P(SSFrame), _P(SSPairs), ctypes.c_int32, _vp, _vp],
    "ss_forward_begin": [_P(SSCamera), _P(SSGaussians), ctypes.c_int32, _P(SSFrame),
                         _P(SSFrameCounts), _P(SSStageEvents), _vp],
    "ss_forward_begin_async": [_P(SSCamera), _P(SSGaussians), ctypes.c_int32, _P(SSFrame),
                               _vp, _P(SSStageEvents), _vp],
    "ss_forward_finish": [_P(SSCamera), ctypes.c_int64, ctypes.c_int32, _P(SSFrame),
                          _P(SSPairs), _P(SSFrameCounts), _vp, _P(ctypes.c_int32),
                          _P(SSStageEvents), _vp],
    "ss_forward_back": [_P(SSCamera), ctypes.c_int64, ctypes.c_int32, _P(SSFrame),
                        _P(SSPairs), _P(SSFrameCounts), _vp, _P(ctypes.c_int32),
                        _P(SSStageEvents), _vp],
    "ss_render": [_P(SSCamera), _P(SSGaussians), ctypes.c_int32, _P(SSFrame), _P(SSPairs), _vp,
                  _P(SSFrameCounts), _P(ctypes.c_int32), _P(SSStageEvents), _vp],
    "ss_render_nosync": [_P(SSCamera), _P(SSGaussians), ctypes.c_int32, _P(SSFrame), _P(SSPairs),
                         _vp, _vp, _P(ctypes.c_int32), _P(SSStageEvents), _vp],
    "ss_render_band": [_P(SSCamera), _P(SSGaussians), ctypes.c_int32, ctypes.c_int32,
                       ctypes.c_int32, _P(SSFrame), _P(SSPairs), _vp, _P(SSFrameCounts),
                       _P(ctypes.c_int32), _P(SSStageEvents), _vp],
    "ss_prune_count": [ctypes.c_int64, ctypes.c_double, _P(ctypes.c_int64)],
    "ss_prune_tmp_words": [ctypes.c_int64, _P(ctypes.c_int64)],
    "ss_prune_select": [_vp, ctypes.c_int64, ctypes.c_double, _vp, _vp, _P(ctypes.c_int64), _vp],
    "ss_gather_gaussians": [_P(SSGaussians), _vp, ctypes.c_int64, _P(SSGaussians), _vp],
    "ss_batch_sizes": [_P(SSBatchItem), ctypes.c_int32, _P(SSBatchInfo)],
    "ss_batch_begin": [_P(SSBatchItem), ctypes.c_int32, ctypes.c_int32, _P(SSFrame),
                       _P(SSFrameCounts), _P(SSStageEvents), _vp],
    "ss_batch_finish": [_P(SSBatchItem), ctypes.c_int32, ctypes.c_int32, _P(SSFrame),
                        _P(SSPairs), _P(SSFrameCounts), _P(ctypes.c_int32), _P(SSStageEvents),
                        _vp],
    "ss_render_backward": [_P(SSCamera), _P(SSGaussians), _P(SSFrame), _P(SSPairs),
                           ctypes.c_int32, _vp, _P(SSGrads), _P(SSStageEvents), _vp],
}
RESTYPES = {"ss_status_string": ctypes.c_char_p, "ss_last_error": ctypes.c_char_p}

_lib = None


class SplatError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def lib():
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2412_00578_amd.csrc.build` (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = RESTYPES.get(name, ctypes.c_int)
        _lib = L
    return _lib


def check(status: int, what: str = "") -> None:
    if status != SS_OK:
        msg = lib().ss_last_error().decode()
        raise SplatError(status, f"{what}: {msg}" if what else msg)


def constants() -> SSConstants:
    c = SSConstants()
    check(lib().ss_get_constants(ctypes.byref(c)), "ss_get_constants")
    return c


def mode_id(mode) -> int:
    return MODES[mode] if isinstance(mode, str) else int(mode)


def make_camera(cam) -> SSCamera:
    """From any object with width, height, fx, fy, cx, cy, R (3x3), t (3), near, bg."""
    c = SSCamera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = [float(x) for row in cam.R for x in row] if hasattr(cam.R[0], "__len__") else \
        [float(x) for x in cam.R]
    for k in range(9):
        c.R[k] = R[k]
    for k in range(3):
        c.t[k] = float(cam.t[k])
    c.near_z = float(getattr(cam, "near", 0.2))
    bg = getattr(cam, "bg", (0.0, 0.0, 0.0))
    for k in range(3):
        c.bg[k] = float(bg[k])
    return c
