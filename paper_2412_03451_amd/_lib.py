"""ctypes binding of libplanesplat.so (the C ABI of include/planesplat.h).

Argument marshalling only: every step of the splatting path runs in the HIP
kernels of the library.  Loading fails loudly when the library is missing.
"""

from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libplanesplat.so")

PS_OK = 0
PS_ERR_INVALID = 1
PS_ERR_CAPACITY = 2
PS_ERR_HIP = 3


class PsCamera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("pad", C.c_int32 * 2)]


class PsParams(C.Structure):
    _fields_ = [("M", C.c_int32), ("tau", C.c_float), ("z_near", C.c_float), ("weight_mode", C.c_int32),
                ("two_sided", C.c_int32), ("flags", C.c_int32)]


class PsSlot(C.Structure):
    _fields_ = [("plane_begin", C.c_int32), ("plane_end", C.c_int32), ("cam", C.c_int32),
                ("width", C.c_int32), ("height", C.c_int32), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("scene", C.c_int32), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("rec_begin", C.c_int32), ("tile_begin", C.c_int32), ("item_begin", C.c_int32),
                ("pad", C.c_int32), ("pix_off", C.c_int64)]


PS_NUM_REGIONS = 24


class PsLayout(C.Structure):
    _fields_ = [("n_slots", C.c_int32), ("n_records", C.c_int32), ("n_tiles", C.c_int32),
                ("n_items", C.c_int32), ("n_pixels", C.c_int64), ("pair_capacity", C.c_int64),
                ("max_sub", C.c_int32), ("n_planes", C.c_int32), ("max_items", C.c_int32), ("max_chunks", C.c_int32),
                ("slots_sorted", C.c_int32), ("pad", C.c_int32),
                ("region", C.c_size_t * PS_NUM_REGIONS), ("ws_bytes", C.c_size_t)]


assert C.sizeof(PsCamera) == 80 and C.sizeof(PsSlot) == 64 and C.sizeof(PsParams) == 24

_P = C.c_void_p
_EXPORTS = {
    "ps_layout_init": (C.c_int, [C.POINTER(PsSlot), C.c_int, C.c_int64, C.POINTER(PsLayout)]),
    "ps_workspace_bytes": (C.c_size_t, [C.POINTER(PsLayout)]),
    "ps_workspace_init": (C.c_int, [C.POINTER(PsLayout), C.POINTER(PsSlot), _P, _P]),
    "ps_set_cameras": (C.c_int, [C.POINTER(PsLayout), _P, _P, _P]),
    "plane_project": (C.c_int, [C.POINTER(PsLayout), _P, _P, _P, _P, C.c_int, _P, C.c_int, _P,
                                C.POINTER(PsParams), _P]),
    "tile_bin": (C.c_int, [C.POINTER(PsLayout), _P, C.POINTER(C.c_int64), _P]),
    "plane_render_fwd": (C.c_int, [C.POINTER(PsLayout), _P, _P, C.c_int, _P, C.POINTER(PsParams), _P, _P, _P, _P,
                                   _P]),
    "loss_depth_normal": (C.c_int, [C.POINTER(PsLayout), _P, _P, _P, _P, _P, _P, C.c_float, C.c_float,
                                    C.c_float, _P, _P, _P, _P]),
    "loss_depth_normal_cam": (C.c_int, [C.POINTER(PsLayout), _P, _P, _P, _P, _P, _P, _P, C.c_int, C.c_float,
                                        C.c_float, C.c_float, _P, _P, _P, _P]),
    "plane_render_bwd": (C.c_int, [C.POINTER(PsLayout), _P, _P, _P, _P, C.c_int, _P, C.c_int, _P,
                                   C.POINTER(PsParams), _P, _P, _P, _P, _P, _P]),
    "adam_step_planes": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, C.c_int, _P, C.c_float, C.c_float,
                                   C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, _P]),
    "plane_render_fwd_loss": (C.c_int, [C.POINTER(PsLayout), _P, _P, C.c_int, _P, C.POINTER(PsParams), _P, _P, _P, _P,
                                        _P, _P, C.c_int, C.c_float, C.c_float, C.c_float, _P, _P, _P, _P]),
    "plane_render_bwd_adam": (C.c_int, [C.POINTER(PsLayout), _P, _P, _P, _P, C.c_int, _P, C.c_int, _P,
                                        C.POINTER(PsParams), _P, _P, _P, _P, _P, _P, _P, _P, C.c_float,
                                        C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, _P, _P]),
    "plane_render_step": (C.c_int, [C.POINTER(PsLayout), _P, _P, _P, _P, C.c_int, _P, C.c_int, _P,
                                    C.POINTER(PsParams), _P, _P, _P, _P, _P, _P, C.c_int, C.c_float, C.c_float,
                                    C.c_float, _P, _P, _P, _P, _P, _P, _P, _P, C.c_float, C.c_float, C.c_float,
                                    C.c_float, C.c_float, C.c_float, C.c_float, _P, _P]),
    "plane_render_fwd_lists": (C.c_int, [C.POINTER(PsLayout), _P, _P, C.c_int, _P, C.POINTER(PsParams), _P, _P, _P,
                                         _P, _P, _P, _P]),
    "plane_render_bwd_lists": (C.c_int, [C.POINTER(PsLayout), _P, _P, _P, _P, C.c_int, _P, C.c_int, _P,
                                         C.POINTER(PsParams), _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "plane_grad_accumulate": (C.c_int, [_P, _P, _P, C.c_int, _P]),
    "plane_split": (C.c_int, [_P, _P, _P, _P, _P, _P, C.c_float, C.c_int, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ps_fit_schedule": (C.c_int, [C.POINTER(PsLayout), _P, _P, _P, C.c_int, _P, _P, _P]),
    "depth_points_ws_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int]),
    "depth_points": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_float, _P, _P, C.c_int, _P, _P,
                               C.c_size_t, _P]),
    "plane_init_points": (C.c_int, [_P, _P, C.c_int, _P, C.c_int, C.c_float, _P, _P, _P, _P]),
    "plane_init_sphere": (C.c_int, [_P, C.c_int, _P, C.c_int, C.c_float, _P, _P, _P, _P, _P]),
    "plane_merge_ws_bytes": (C.c_size_t, [C.c_int]),
    "plane_tie_radii": (C.c_int, [_P, C.c_int, _P]),
    "plane_merge": (C.c_int, [_P, _P, C.c_int, _P, C.c_double, C.c_double, _P, _P, _P, C.c_size_t, _P]),
    "initnet_param_count": (C.c_int64, [C.c_int]),
    "initnet_packed_count": (C.c_int64, [C.c_int]),
    "initnet_forward_ws": (C.c_int64, [C.c_int, C.c_int]),
    "initnet_backward_ws": (C.c_int64, [C.c_int, C.c_int]),
    "initnet_pack": (C.c_int, [_P, C.c_int, _P, _P]),
    "initnet_forward": (C.c_int, [_P, _P, C.c_int, _P, C.c_int, C.c_int, _P, _P, _P, _P, _P, _P]),
    "initnet_set_loss": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _P, _P]),
    "initnet_backward": (C.c_int, [_P, _P, C.c_int, _P, C.c_int, C.c_int, _P, _P, _P, _P, _P, _P]),
    "initnet_adam": (C.c_int, [_P, _P, _P, _P, C.c_int64, _P, C.c_float, C.c_float, C.c_float, C.c_float, _P]),
    "ps_read_counters": (C.c_int, [C.POINTER(PsLayout), _P, C.POINTER(C.c_int64), _P]),
    "ps_valu_probe": (C.c_int, [C.c_int, C.c_int, C.c_int, _P, C.c_size_t, _P]),
    "ps_check_finite": (C.c_int, [_P, C.c_int64, _P, C.POINTER(C.c_int64), _P]),
    "plane_render_fwd_noalloc": (C.c_int, [_P, _P, _P, C.c_int, _P, C.c_int, C.c_int, C.c_int, C.c_int, _P,
                                           C.POINTER(PsParams), _P, _P, _P, _P]),
    "initnet_view_points": (C.c_int, [_P, _P, C.c_int, C.c_int, C.c_int, _P, _P, C.c_int, C.c_int, C.c_float, _P,
                                      _P, _P]),
    "initnet_proposals_to_world": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _P, _P, _P, _P]),
    "initnet_refine_planes": (C.c_int, [_P, _P, _P, C.c_int, _P, _P, _P, _P, C.c_int, C.c_double, C.c_double, _P,
                                        _P, _P, _P]),
    "ps_last_error": (C.c_char_p, []),
}

_lib = None


def exported_names():
    return list(_EXPORTS)


def load(path: str = LIB_PATH):
    """Load the library once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2412_03451_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PlaneSplatError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def check(rc: int):
    if rc != PS_OK:
        raise PlaneSplatError(rc, load().ps_last_error().decode())
