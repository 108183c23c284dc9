"""ctypes binding of libmsda.so (the C ABI declared in include/msda.h).

Argument marshalling only: every step of the operator runs in the library's
HIP kernels. Loading fails loudly when the library is missing; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmsda.so")

MSDA_OK = 0
MSDA_ERR_INVALID_ARGUMENT = 1
MSDA_ERR_UNSUPPORTED = 2
MSDA_ERR_HIP = 3
MSDA_ERR_WORKSPACE = 4
STATUS_NAMES = {0: "OK", 1: "INVALID_ARGUMENT", 2: "UNSUPPORTED", 3: "HIP", 4: "WORKSPACE"}

MSDA_F32 = 0
MSDA_BF16 = 1
MSDA_FP8_E4M3 = 2
MSDA_F16 = 3

MSDA_DETERMINISTIC = 1
MSDA_WEIGHT_LOGITS = 2
MSDA_WEIGHTS_BF16 = 4

ABI_VERSION = 8

# Every symbol include/msda.h declares.
EXPORTS = (
    "msda_forward", "msda_forward_ws", "msda_forward_workspace_size", "msda_forward_noalloc",
    "msda_backward",
    "msda_backward_workspace_size", "msda_project_keypoints", "msda_forward_visible",
    "msda_forward_visible_workspace_size", "msda_backward_visible",
    "msda_backward_visible_workspace_size", "msda_forward_fused",
    "msda_forward_fused_workspace_size", "msda_backward_fused",
    "msda_backward_fused_workspace_size", "msda_quantize_fp8",
    "msda_quantize_workspace_size", "msda_batched_workspace_size", "msda_forward_batched",
    "msda_backward_batched", "msda_sort_keys", "msda_sort_workspace_size", "msda_stream_copy",
    "msda_set_kernel_events", "msda_set_kernel_event_filter",
    "msda_recorded_kernels", "msda_recorded_kernel_name", "msda_last_error", "msda_abi_version",
)

MSDA_SCATTER_AUTO = 0
MSDA_SCATTER_SORTED = 1
MSDA_SCATTER_ATOMIC = 2
MSDA_SCATTER_SORTED_GLOBAL = 3

MSDA_ORDER_AUTO = 0
MSDA_ORDER_ANCHOR = 1
MSDA_ORDER_VIEW = 2
ORDERS = {"auto": MSDA_ORDER_AUTO, "anchor": MSDA_ORDER_ANCHOR, "view": MSDA_ORDER_VIEW}


class MsdaTile(ctypes.Structure):
    _fields_ = [("waves_per_anchor", ctypes.c_int32), ("chans_per_lane", ctypes.c_int32),
                ("order", ctypes.c_int32), ("scatter", ctypes.c_int32)]


class MsdaDesc(ctypes.Structure):
    _fields_ = [
        ("batch", ctypes.c_int32), ("num_cams", ctypes.c_int32), ("num_levels", ctypes.c_int32),
        ("num_anchors", ctypes.c_int32), ("num_points", ctypes.c_int32),
        ("channels", ctypes.c_int32), ("groups", ctypes.c_int32), ("feat_dtype", ctypes.c_int32),
        ("rows", ctypes.c_int64),
        ("host_spatial_shapes", ctypes.c_void_p), ("host_level_start_index", ctypes.c_void_p),
        ("level_scale", ctypes.c_void_p), ("flags", ctypes.c_uint32),
        ("tile", ctypes.POINTER(MsdaTile)),
    ]


class MsdaProjDesc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("num_anchors", ctypes.c_int32),
                ("num_points", ctypes.c_int32), ("num_cams", ctypes.c_int32),
                ("dt", ctypes.c_float)]


class MsdaScene(ctypes.Structure):
    _fields_ = [
        ("feat", ctypes.c_void_p), ("spatial_shapes", ctypes.c_void_p),
        ("level_start_index", ctypes.c_void_p), ("sampling_loc", ctypes.c_void_p),
        ("weights", ctypes.c_void_p), ("out", ctypes.c_void_p), ("grad_out", ctypes.c_void_p),
        ("grad_feat", ctypes.c_void_p), ("grad_sampling_loc", ctypes.c_void_p),
        ("grad_weights", ctypes.c_void_p), ("rows", ctypes.c_int64), ("num_cams", ctypes.c_int32),
        ("num_anchors", ctypes.c_int32),
    ]


class MsdaBatch(ctypes.Structure):
    _fields_ = [
        ("num_scenes", ctypes.c_int32), ("num_levels", ctypes.c_int32),
        ("num_points", ctypes.c_int32), ("channels", ctypes.c_int32), ("groups", ctypes.c_int32),
        ("feat_dtype", ctypes.c_int32), ("scenes", ctypes.c_void_p),
        ("host_scenes", ctypes.POINTER(MsdaScene)),
        ("host_spatial_shapes", ctypes.POINTER(ctypes.c_void_p)),
        ("host_level_start_index", ctypes.POINTER(ctypes.c_void_p)),
        ("level_scale", ctypes.c_void_p), ("flags", ctypes.c_uint32),
        ("tile", ctypes.POINTER(MsdaTile)),
    ]


class MSDAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libmsda.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_2601_10819_amd.build)")
    lib = ctypes.CDLL(path)
    vp, sz, dp = ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(MsdaDesc)
    lib.msda_forward.argtypes = [vp] * 6 + [dp, vp]
    lib.msda_forward.restype = ctypes.c_int
    lib.msda_forward_ws.argtypes = [vp] * 7 + [sz, dp, vp]
    lib.msda_forward_ws.restype = ctypes.c_int
    lib.msda_forward_workspace_size.argtypes = [dp]
    lib.msda_forward_workspace_size.restype = sz
    lib.msda_forward_noalloc.argtypes = [vp] * 6 + [dp, vp]
    lib.msda_forward_noalloc.restype = ctypes.c_int
    lib.msda_project_keypoints.argtypes = [vp] * 6 + [ctypes.POINTER(MsdaProjDesc), vp]
    lib.msda_project_keypoints.restype = ctypes.c_int
    lib.msda_forward_visible.argtypes = [vp] * 8 + [sz, dp, vp]
    lib.msda_forward_visible.restype = ctypes.c_int
    lib.msda_forward_visible_workspace_size.argtypes = [dp]
    lib.msda_forward_visible_workspace_size.restype = sz
    lib.msda_backward_visible.argtypes = [vp] * 11 + [sz, dp, vp]
    lib.msda_backward_visible.restype = ctypes.c_int
    lib.msda_backward_visible_workspace_size.argtypes = [dp]
    lib.msda_backward_visible_workspace_size.restype = sz
    lib.msda_forward_fused.argtypes = [vp] * 9 + [sz, dp, vp]
    lib.msda_forward_fused.restype = ctypes.c_int
    lib.msda_forward_fused_workspace_size.argtypes = [dp]
    lib.msda_forward_fused_workspace_size.restype = sz
    lib.msda_backward_fused.argtypes = [vp] * 14 + [sz, dp, vp]
    lib.msda_backward_fused.restype = ctypes.c_int
    lib.msda_backward_fused_workspace_size.argtypes = [dp]
    lib.msda_backward_fused_workspace_size.restype = sz
    lib.msda_backward.argtypes = [vp] * 10 + [sz, dp, vp]
    lib.msda_backward.restype = ctypes.c_int
    lib.msda_backward_workspace_size.argtypes = [dp]
    lib.msda_backward_workspace_size.restype = sz
    lib.msda_quantize_fp8.argtypes = [vp] * 6 + [sz, dp, vp]
    lib.msda_quantize_fp8.restype = ctypes.c_int
    lib.msda_quantize_workspace_size.argtypes = [dp]
    lib.msda_quantize_workspace_size.restype = sz
    bp = ctypes.POINTER(MsdaBatch)
    lib.msda_batched_workspace_size.argtypes = [bp, ctypes.c_int32]
    lib.msda_batched_workspace_size.restype = sz
    lib.msda_forward_batched.argtypes = [bp, vp, sz, vp]
    lib.msda_forward_batched.restype = ctypes.c_int
    lib.msda_backward_batched.argtypes = [bp, vp, sz, vp]
    lib.msda_backward_batched.restype = ctypes.c_int
    u32 = ctypes.c_uint32
    lib.msda_sort_keys.argtypes = [vp, u32, u32, vp, vp, vp, sz, vp]
    lib.msda_sort_keys.restype = ctypes.c_int
    lib.msda_sort_workspace_size.argtypes = [u32, u32]
    lib.msda_sort_workspace_size.restype = sz
    lib.msda_stream_copy.argtypes = [vp, vp, sz, vp]
    lib.msda_stream_copy.restype = ctypes.c_int
    lib.msda_set_kernel_events.argtypes = [vp, ctypes.c_int32]
    lib.msda_set_kernel_events.restype = ctypes.c_int
    lib.msda_set_kernel_event_filter.argtypes = [ctypes.c_char_p]
    lib.msda_set_kernel_event_filter.restype = ctypes.c_int
    lib.msda_recorded_kernels.argtypes = []
    lib.msda_recorded_kernels.restype = ctypes.c_int32
    lib.msda_recorded_kernel_name.argtypes = [ctypes.c_int32]
    lib.msda_recorded_kernel_name.restype = ctypes.c_char_p
    lib.msda_last_error.argtypes = []
    lib.msda_last_error.restype = ctypes.c_char_p
    lib.msda_abi_version.argtypes = []
    lib.msda_abi_version.restype = ctypes.c_int32
    if lib.msda_abi_version() != ABI_VERSION:
        raise RuntimeError(f"libmsda ABI {lib.msda_abi_version()} != binding ABI {ABI_VERSION}")
    _lib = lib
    return lib


def check(status: int):
    if status != MSDA_OK:
        msg = load().msda_last_error()
        raise MSDAError(status, msg.decode() if msg else "")
