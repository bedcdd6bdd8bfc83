"""ctypes declarations of the libgs2d.so C ABI (include/gs2d.h, include/gs2d_warm.h).

This module only loads the library and marshals arguments.  There is no
fallback: if the library has not been built, loading raises ``ImportError``.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# GS2D_LIB selects another build of the library (the device-check or host-sanitizer
# builds that build.py makes beside it)
LIB_PATH = os.environ.get("GS2D_LIB") or os.path.join(HERE, "libgs2d.so")
INCLUDE_DIR = os.path.join(os.path.dirname(HERE), "include")
HEADER_PATH = os.path.join(INCLUDE_DIR, "gs2d.h")
HEADERS = [os.path.join(INCLUDE_DIR, h) for h in ("gs2d.h", "gs2d_warm.h", "gs2d_map.h")]

OK = 0
ERR_INVALID_ARG = -1
ERR_OOM = -2
ERR_HIP = -3
ERR_CAPACITY = -4
ERR_STATE = -5
ERR_UNSUPPORTED = -6
ERR_NONFINITE = -7
ERR_DEVICE_CHECK = -8
TRACK_FELL_BACK = 4
BUILD_DEVICE_CHECKS = 1
ACCUMULATE = 1
TUNE_FULL_BACKWARD = 1


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class Options(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("filter", ctypes.c_int32), ("z_near", ctypes.c_float), ("pair_capacity", ctypes.c_int64),
                ("keep_unsorted", ctypes.c_int32), ("profile", ctypes.c_int32)]


class Counts(ctypes.Structure):
    _fields_ = [("n_surfels", ctypes.c_int64), ("n_visible", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("pair_capacity", ctypes.c_int64), ("overflow", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("nonfinite", ctypes.c_int32), ("device_checks", ctypes.c_int32)]


PROFILE_FAMILIES = 13


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * PROFILE_FAMILIES), ("launches", ctypes.c_int64 * PROFILE_FAMILIES),
                ("fwd_evaluated", ctypes.c_int64), ("fwd_covering", ctypes.c_int64),
                ("bwd_evaluated", ctypes.c_int64), ("bwd_covering", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("ms", ctypes.c_float), ("n_candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32)]


NOALLOC_MAX_PIXELS = 1 << 24
MAX_VIEWS = 32


class WsAdamW(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("weight_decay", ctypes.c_float)]


class MappingWeights(ctypes.Structure):
    _fields_ = [("w_l1", ctypes.c_float), ("w_ssim", ctypes.c_float), ("w_d", ctypes.c_float),
                ("w_n", ctypes.c_float)]


class LossWeights(ctypes.Structure):
    _fields_ = [("w_rgb", ctypes.c_float), ("w_depth", ctypes.c_float), ("w_normal", ctypes.c_float),
                ("normal_mask", ctypes.c_int32), ("opacity_mask", ctypes.c_int32)]


class LossView(ctypes.Structure):
    _fields_ = [("camera", Camera)] + [(k, ctypes.c_void_p) for k in (
        "rgb", "depth", "normal", "alpha", "tgt_rgb", "tgt_depth", "tgt_normal", "d_rgb", "d_depth", "d_normal")]


class AdamArgs(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 6), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("weight_decay", ctypes.c_float), ("step", ctypes.c_int32),
                ("s_min", ctypes.c_float), ("o_min", ctypes.c_float), ("o_max", ctypes.c_float)]


class View(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("n", ctypes.c_int64), ("camera", Camera), ("pose", ctypes.c_void_p),
                ("rgb", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("normal", ctypes.c_void_p),
                ("alpha", ctypes.c_void_p), ("contrib", ctypes.c_void_p), ("depth_norm", ctypes.c_void_p),
                ("depth_median", ctypes.c_void_p)]


class ViewGrad(ctypes.Structure):
    _fields_ = [("d_rgb", ctypes.c_void_p), ("d_depth", ctypes.c_void_p), ("d_normal", ctypes.c_void_p),
                ("d_alpha", ctypes.c_void_p), ("d_params", ctypes.c_void_p), ("d_pose", ctypes.c_void_p)]


class TrackProblem(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("n", ctypes.c_int64), ("camera", Camera), ("pose", ctypes.c_void_p),
                ("tgt_rgb", ctypes.c_void_p), ("tgt_depth", ctypes.c_void_p), ("fallback_pose", ctypes.c_void_p),
                ("fallback_loss", ctypes.c_void_p)]


class TrackArgs(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("n", ctypes.c_int64), ("camera", Camera),
                ("pose", ctypes.c_void_p), ("tgt_rgb", ctypes.c_void_p), ("tgt_depth", ctypes.c_void_p),
                ("lambda_d", ctypes.c_float), ("use_masks", ctypes.c_int32), ("n_iters", ctypes.c_int32),
                ("lr", ctypes.c_float * 6), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("weight_decay", ctypes.c_float), ("use_graph", ctypes.c_int32),
                ("pose_history", ctypes.c_void_p), ("loss_history", ctypes.c_void_p),
                ("grad_history", ctypes.c_void_p), ("diverge_patience", ctypes.c_int32),
                ("status", ctypes.c_void_p), ("fallback_pose", ctypes.c_void_p), ("fallback_loss", ctypes.c_void_p)]


class Gs2dError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"gs2d error {code}: {message}")
        self.code = code


_lib = None

_P = ctypes.c_void_p
_SIGS = {
    "gs2d_default_options": ([ctypes.POINTER(Options)], ctypes.c_int),
    "gs2d_create": ([ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(Options)], ctypes.c_int),
    "gs2d_destroy": ([_P], ctypes.c_int),
    "gs2d_render": ([_P, _P, ctypes.c_int64, ctypes.POINTER(Camera), _P, _P, _P, _P, _P,
                     ctypes.POINTER(ctypes.c_uint32), _P], ctypes.c_int),
    "gs2d_render_backward": ([_P, _P, _P, _P, _P, _P, _P, ctypes.c_uint32, ctypes.c_int32, _P], ctypes.c_int),
    "gs2d_render_batch": ([_P, ctypes.POINTER(View), ctypes.c_int32, ctypes.POINTER(ctypes.c_uint32), _P],
                          ctypes.c_int),
    "gs2d_render_backward_batch": ([_P, ctypes.POINTER(ViewGrad), ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32,
                                    _P], ctypes.c_int),
    "gs2d_track_batch": ([_P, ctypes.POINTER(TrackProblem), ctypes.c_int32, ctypes.POINTER(TrackArgs), _P],
                         ctypes.c_int),
    "gs2d_tracking_loss": ([_P, ctypes.POINTER(Camera), _P, _P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_int32,
                            _P, _P, _P, _P], ctypes.c_int),
    "gs2d_tracking_error": ([_P, ctypes.POINTER(Camera), _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "gs2d_image_loss": ([_P, ctypes.POINTER(Camera), _P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(LossWeights), _P, _P,
                         _P, _P, _P], ctypes.c_int),
    "gs2d_image_loss_batch": ([_P, ctypes.POINTER(LossView), ctypes.c_int32, ctypes.POINTER(LossWeights), _P, _P],
                              ctypes.c_int),
    "gs2d_image_loss_noalloc": ([ctypes.POINTER(Camera), _P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(LossWeights), _P,
                                 _P, _P, _P, _P], ctypes.c_int),
    "gs2d_track": ([_P, ctypes.POINTER(TrackArgs), _P], ctypes.c_int),
    "gs2d_get_counts": ([_P, ctypes.POINTER(Counts), _P], ctypes.c_int),
    "gs2d_debug_copy": ([_P, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_size_t), _P], ctypes.c_int),
    "gs2d_autotune": ([_P, _P, ctypes.c_int64, ctypes.POINTER(Camera), _P, ctypes.c_int32, ctypes.c_int32,
                       ctypes.POINTER(Tuning), _P], ctypes.c_int),
    "gs2d_pose_exp": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "gs2d_pose_tau_grad": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "gs2d_profile_family": ([ctypes.c_int], ctypes.c_char_p),
    "gs2d_get_profile": ([_P, ctypes.POINTER(Profile), ctypes.c_int32, _P], ctypes.c_int),
    "gs2d_last_hip_error": ([_P], ctypes.c_int),
    "gs2d_error_string": ([ctypes.c_int], ctypes.c_char_p),
    "gs2d_build_info": ([], ctypes.c_int),
    # learned warm start (gs2d_warm.h)
    "gs2d_ws_param_count": ([], ctypes.c_int64),
    "gs2d_ws_create": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int32], ctypes.c_int),
    "gs2d_ws_destroy": ([_P], ctypes.c_int),
    "gs2d_ws_set_params": ([_P, _P, _P], ctypes.c_int),
    "gs2d_ws_get_params": ([_P, _P, _P], ctypes.c_int),
    "gs2d_ws_residual": ([_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P], ctypes.c_int),
    "gs2d_ws_forward": ([_P, _P, ctypes.c_int32, _P, _P], ctypes.c_int),
    "gs2d_ws_gradient": ([_P, _P, _P, ctypes.c_int32, _P, _P, _P, _P], ctypes.c_int),
    "gs2d_ws_adamw_step": ([_P, ctypes.POINTER(WsAdamW), _P], ctypes.c_int),
    "gs2d_warm_start": ([_P, _P, _P, ctypes.c_int64, ctypes.POINTER(Camera), _P, _P, _P, ctypes.c_float,
                         ctypes.c_int32, _P, _P, _P], ctypes.c_int),
    "gs2d_warm_start_propose": ([_P, _P, _P, ctypes.c_int64, ctypes.POINTER(Camera), _P, _P, _P, ctypes.c_float,
                                 _P, _P, _P], ctypes.c_int),
    # map bookkeeping (gs2d_map.h)
    "gs2d_covisibility_workspace": ([ctypes.c_int64], ctypes.c_int64),
    "gs2d_covisibility": ([_P, _P, ctypes.c_int64, ctypes.c_float, _P, _P, _P], ctypes.c_int),
    "gs2d_keyframe_test": ([_P, _P, _P, ctypes.c_double, ctypes.c_double, _P, _P], ctypes.c_int),
    "gs2d_prune_mask": ([_P, _P, ctypes.c_int32, ctypes.c_float, ctypes.c_int64, _P, _P], ctypes.c_int),
    "gs2d_compact_workspace": ([ctypes.c_int64], ctypes.c_int64),
    "gs2d_compact": ([_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, _P, _P, ctypes.c_int64, _P, _P, _P],
                     ctypes.c_int),
    "gs2d_map_state_update": ([_P, ctypes.c_int64, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P,
                               _P, _P, _P], ctypes.c_int),
    "gs2d_map_correct": ([_P, ctypes.c_int64, _P, _P, ctypes.c_int32, _P], ctypes.c_int),
    "gs2d_params_adam": ([_P, _P, _P, _P, ctypes.c_int64, ctypes.POINTER(AdamArgs), _P], ctypes.c_int),
    "gs2d_mapping_loss_workspace": ([ctypes.c_int32, ctypes.c_int32], ctypes.c_int64),
    "gs2d_mapping_loss": ([ctypes.POINTER(Camera), _P, _P, _P, _P, _P, ctypes.POINTER(MappingWeights), _P, _P, _P,
                           _P, _P, _P], ctypes.c_int),
}


def load():
    """Load libgs2d.so (built in-tree) and declare every exported function."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2506_00970_amd.build` "
                              "(the rasterizer has no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def error_string(code: int) -> str:
    return load().gs2d_error_string(int(code)).decode()


def check(code: int, ctx=None) -> None:
    if code != OK:
        msg = error_string(code)
        if ctx is not None and code == ERR_HIP:
            msg += f" (hipError_t {load().gs2d_last_hip_error(ctx)})"
        raise Gs2dError(code, msg)


def declared_functions() -> list:
    """Names of the functions declared with GS2D_API in the public headers."""
    import re

    names = []
    for h in HEADERS:
        with open(h) as f:
            names += re.findall(r"GS2D_API\s+[\w\s\*]+?\b(gs2d_\w+)\s*\(", f.read())
    return names
