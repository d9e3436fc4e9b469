"""ctypes binding of the C ABI in include/gs_raster.h (argument marshalling only).

The shared library is built in-tree (``python -m paper_2501_06838_amd.build``).
There is no fallback: if the library is missing or fails to load, every call
raises.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgsraster.so")

GS_OK = 0
GS_E_INVALID = -1
GS_E_CAPACITY = -2
GS_E_DEVICE = -3
GS_E_UNSUPPORTED = -4
GS_E_WORKSPACE = -5

ABI_VERSION = 3  # GS_ABI_VERSION of include/gs_raster.h

GS_FLAG_PERSISTENT = 0x1
GS_FLAG_ATOMIC_GRADS = 0x2
GS_FLAG_RADIX_SORT = 0x4
GS_FLAG_PIXEL_CENTER = 0x8
GS_FLAG_ELLIPSE = 0x10

EXPORTED = (
    "gs_abi_version", "gs_status_string", "gs_output_size", "gs_workspace_size",
    "gs_raster_forward", "gs_raster_backward", "gs_l1_loss_grad", "gs_diagnostics",
    "gs_count_pairs", "gs_tile_lists", "gs_raster_bin", "gs_raster_render",
    "gs_raster_render_backward", "gs_raster_gradients", "gs_raster_render_backward_l1",
    "gs_l1_loss_value", "gs_raster_backward_l1", "gs_graph_create", "gs_graph_launch",
    "gs_graph_destroy", "gs_mlp_features", "gs_mlp_forward", "gs_mlp_workspace_size",
    "gs_mlp_grad", "gs_mlp_adam", "gs_radius_stats", "gs_sq_error", "gs_tile_order",
    "gs_raster_render_fused_l1", "gs_raster_step_l1", "gs_raster_step_l1_noalloc",
    "gs_mlp_radius", "gs_closed_form_radius", "gs_gaussian_head_forward",
    "gs_gaussian_head_backward", "gs_psnr_y", "gs_valu_probe",
)


class gs_image(ctypes.Structure):
    _fields_ = [("lr_h", ctypes.c_int32), ("lr_w", ctypes.c_int32),
                ("scale", ctypes.c_double), ("g_begin", ctypes.c_int64),
                ("g_count", ctypes.c_int64), ("out_offset", ctypes.c_int64)]


class gs_config(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("lds_batch", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("pair_capacity", ctypes.c_int64), ("window_r", ctypes.c_double)]


class GSError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None
_vp = ctypes.c_void_p
_cfgp = ctypes.POINTER(gs_config)
_imgp = ctypes.POINTER(gs_image)
_i32, _i64, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t


def lib():
    """The loaded library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2501_06838_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.gs_abi_version.argtypes = []
        L.gs_abi_version.restype = _i32
        L.gs_status_string.argtypes = [_i32]
        L.gs_status_string.restype = ctypes.c_char_p
        L.gs_output_size.argtypes = [_i32, _i32, ctypes.c_double, ctypes.POINTER(_i32),
                                     ctypes.POINTER(_i32)]
        L.gs_output_size.restype = _i32
        L.gs_workspace_size.argtypes = [_cfgp, _imgp, _i32, _i64, ctypes.POINTER(_sz)]
        L.gs_workspace_size.restype = _i32
        L.gs_raster_forward.argtypes = [_cfgp, _imgp, _i32, _vp, _vp, _vp, _vp, _vp, _i64,
                                        _vp, _sz, _vp, _vp]
        L.gs_raster_forward.restype = _i32
        L.gs_raster_backward.argtypes = [_cfgp, _imgp, _i32, _vp, _vp, _vp, _vp, _vp, _i64,
                                         _vp, _sz, _vp, _vp, _vp, _vp, _vp, _vp]
        L.gs_raster_backward.restype = _i32
        L.gs_l1_loss_grad.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp]
        L.gs_l1_loss_grad.restype = _i32
        L.gs_diagnostics.argtypes = [_cfgp, _imgp, _i32, _i64, _vp, _sz,
                                     ctypes.POINTER(_i64), ctypes.POINTER(_i32),
                                     ctypes.POINTER(_i64), ctypes.POINTER(_i64), _vp]
        L.gs_diagnostics.restype = _i32
        L.gs_count_pairs.argtypes = [_cfgp, _imgp, _i32, _vp, _vp, _vp, _i64, _vp, _sz,
                                     ctypes.POINTER(_i64), _vp]
        L.gs_count_pairs.restype = _i32
        L.gs_tile_lists.argtypes = [_cfgp, _imgp, _i32, _i64, _vp, _sz, _vp, _vp, _i64,
                                    ctypes.POINTER(_i64), ctypes.POINTER(_i64), _vp]
        L.gs_tile_lists.restype = _i32
        L.gs_tile_order.argtypes = [_cfgp, _imgp, _i32, _i64, _vp, _sz, _vp, _i64,
                                    ctypes.POINTER(_i32), _vp]
        L.gs_tile_order.restype = _i32
        L.gs_raster_bin.argtypes = [_cfgp, _imgp, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp,
                                    _sz, _vp]
        L.gs_raster_bin.restype = _i32
        L.gs_raster_render.argtypes = [_cfgp, _imgp, _i32, _i64, _vp, _sz, _vp, _vp]
        L.gs_raster_render.restype = _i32
        L.gs_raster_render_backward.argtypes = [_cfgp, _imgp, _i32, _i64, _vp, _sz, _vp, _vp]
        L.gs_raster_render_backward.restype = _i32
        L.gs_raster_gradients.argtypes = [_cfgp, _imgp, _i32, _vp, _vp, _vp, _i64, _vp, _sz,
                                          _vp, _vp, _vp, _vp, _vp]
        L.gs_raster_gradients.restype = _i32
        L.gs_raster_render_backward_l1.argtypes = [_cfgp, _imgp, _i32, _i64, _vp, _sz, _vp,
                                                   _vp, _vp]
        L.gs_raster_render_backward_l1.restype = _i32
        L.gs_l1_loss_value.argtypes = [_cfgp, _imgp, _i32, _i64, _vp, _sz, _vp, _vp]
        L.gs_l1_loss_value.restype = _i32
        L.gs_raster_backward_l1.argtypes = [_cfgp, _imgp, _i32, _vp, _vp, _vp, _i64, _vp, _sz,
                                            _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.gs_raster_backward_l1.restype = _i32
        L.gs_raster_render_fused_l1.argtypes = [_cfgp, _imgp, _i32, _i64, _vp, _sz, _vp, _vp,
                                                _vp]
        L.gs_raster_render_fused_l1.restype = _i32
        L.gs_raster_step_l1.argtypes = [_cfgp, _imgp, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp,
                                        _sz, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.gs_raster_step_l1.restype = _i32
        L.gs_raster_step_l1_noalloc.argtypes = [_cfgp, _imgp, _i32, _vp, _vp, _vp, _vp, _vp,
                                                _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                                _vp]
        L.gs_raster_step_l1_noalloc.restype = _i32
        L.gs_gaussian_head_forward.argtypes = [_imgp, _i32, _i32] + [_vp] * 5 + [_i64] + \
            [_vp] * 5
        L.gs_gaussian_head_forward.restype = _i32
        L.gs_gaussian_head_backward.argtypes = [_i64] + [_vp] * 14
        L.gs_gaussian_head_backward.restype = _i32
        L.gs_psnr_y.argtypes = [_imgp, _i32, _vp, _vp, _i32, _vp, _vp, _vp]
        L.gs_psnr_y.restype = _i32
        L.gs_valu_probe.argtypes = [_i32, _i32, _i32, _vp, _vp]
        L.gs_valu_probe.restype = _i32
        L.gs_graph_create.argtypes = [_cfgp, _imgp, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp,
                                      _sz, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                      ctypes.POINTER(_vp)]
        L.gs_graph_create.restype = _i32
        L.gs_graph_launch.argtypes = [_vp, _vp]
        L.gs_graph_launch.restype = _i32
        L.gs_graph_destroy.argtypes = [_vp]
        L.gs_graph_destroy.restype = _i32
        if L.gs_abi_version() != ABI_VERSION:
            raise ImportError("libgsraster ABI version mismatch")
        _lib = L
    return _lib


def status_string(st: int) -> str:
    try:
        return lib().gs_status_string(st).decode()
    except Exception:  # library not loadable: still format the code
        return "status"


def check(st: int, what: str) -> None:
    if st != GS_OK:
        raise GSError(st, what)
