"""FP64 CPU oracle of the 2D Gaussian surfel rasterizer.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library (``paper_2506_00970_amd``) and never imports it.

* ``render`` / ``backward`` / ``preprocess``: the C++ rasterizer in
  ``gs2d_oracle.cpp`` (forward, reverse mode, pose gradient in two forms).
* ``se3``: SE(3) exponential and logarithm (closed forms).
* ``loss``: tracking / single-frame losses and their image gradients, and the
  AdamW pose update.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import loss, se3  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs2d_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source, loaded instead
# when GS2D_ORACLE_SANITIZED=1 (the process must preload gcc's libasan and libubsan)
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]

# The oracle's own copy of the method's constants.
Z_NEAR = 0.2            # centre cull and per-pixel depth cut (metres)
RHO_CUTOFF = 9.0        # include a pair when u^2 + v^2 (or the filter term) <= 9 (3 sigma)
ALPHA_MAX = 0.99        # opacity clamp
ALPHA_MIN = 1.0 / 255.0  # pairs below this opacity are skipped
T_MIN = 1e-4            # compositing stops before transmittance drops below this
FILTER_SCALE = 2.0      # low-pass filter term 2 |p - c|^2 (sigma^2 = 1/2 pixel^2)


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the oracle with g++ into ``oracle/liboracle.so`` (``sanitize``:
    ``oracle/liboracle_san.so`` with ASan and UBSan)."""
    lib = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        flags = SANITIZE_FLAGS if sanitize else ["-O2"]
        subprocess.check_call(["g++", *flags, "-std=c++17", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, lib)
    return lib


class _Cam(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double)]


class _Consts(ctypes.Structure):
    _fields_ = [("z_near", ctypes.c_double), ("rho_cutoff", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("alpha_min", ctypes.c_double),
                ("t_min", ctypes.c_double), ("filter_scale", ctypes.c_double),
                ("filter", ctypes.c_int32), ("use_rect", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build(sanitize=os.environ.get("GS2D_ORACLE_SANITIZED") == "1"))
        P = ctypes.c_void_p
        _lib.orc_render.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_int] + [P] * 8
        _lib.orc_backward.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_int] + [P] * 14
        _lib.orc_preprocess.argtypes = [P, ctypes.c_int64, P, P, P] + [P] * 5
        _lib.orc_contribution.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_int, ctypes.c_double, P, P]
        _lib.orc_depth_variants.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_int, P, P, P]
    return _lib


def _cam(camera) -> _Cam:
    t = camera.as_tuple() if hasattr(camera, "as_tuple") else tuple(camera)
    return _Cam(int(t[0]), int(t[1]), float(t[2]), float(t[3]), float(t[4]), float(t[5]))


def _consts(filter: bool, use_rect: bool) -> _Consts:
    return _Consts(Z_NEAR, RHO_CUTOFF, ALPHA_MAX, ALPHA_MIN, T_MIN, FILTER_SCALE,
                   int(bool(filter)), int(bool(use_rect)))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _threads(n):
    return int(n) if n else max(1, min(os.cpu_count() or 1, 16))


def _prep(params, pose):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    assert p.ndim == 2 and p.shape[0] == 15, "params must be [15, N]"
    T = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(3, 4))
    return p, T


def render(params, camera, pose, filter: bool = True, use_rect: bool = True, nthreads=None):
    """Forward render; returns a dict of FP64 planar images and per-pixel state.

    Keys: rgb [3,H,W], depth [H,W], normal [3,H,W], alpha [H,W], t_final [H,W],
    count [H,W] (composited surfels), fmargin / gmargin [H,W] (smallest relative
    margin to any decision that changes the value / the gradient).
    """
    lib = _load()
    p, T = _prep(params, pose)
    c = _cam(camera)
    H, W = c.height, c.width
    out = {
        "rgb": np.zeros((3, H, W)), "depth": np.zeros((H, W)), "normal": np.zeros((3, H, W)),
        "alpha": np.zeros((H, W)), "t_final": np.zeros((H, W)),
        "count": np.zeros((H, W), dtype=np.int32), "fmargin": np.zeros((H, W)),
        "gmargin": np.zeros((H, W)),
    }
    k = _consts(filter, use_rect)
    lib.orc_render(_ptr(p), p.shape[1], ctypes.byref(c), _ptr(T), ctypes.byref(k), _threads(nthreads),
                   _ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["normal"]), _ptr(out["alpha"]),
                   _ptr(out["t_final"]), _ptr(out["count"]), _ptr(out["fmargin"]), _ptr(out["gmargin"]))
    return out


def backward(params, camera, pose, d_rgb=None, d_depth=None, d_normal=None, d_alpha=None,
             filter: bool = True, use_rect: bool = True, nthreads=None, watch=None, scale: bool = False,
             scale_mask=None):
    """Reverse mode for given image gradients.

    Returns a dict: d_params [15,N] (world frame), d_screen [16,N]
    (dL/dM row-major, dL/dn, dL/drgb, dL/do), pose_paper [6] and pose_identity
    [6] (rho, phi of a left perturbation), and, when ``watch`` (bool [H,W]) is
    given, touched [N] (surfels evaluated at a watched pixel).

    With ``scale``: d_scale [15,N] and pose_scale [6], the magnitude scale of each
    result, a bound on the sum over (pixel, surfel) pairs of |the pair's term|
    (each result is a sum of such terms; its floating-point rounding is
    proportional to this scale).  With ``scale_mask`` (bool [H,W]) also
    pose_scale_masked [6], the same over the pairs at the masked pixels only.
    """
    lib = _load()
    p, T = _prep(params, pose)
    c = _cam(camera)
    n = p.shape[1]
    H, W = c.height, c.width

    def g(a, shape):
        if a is None:
            return None
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        assert a.shape == shape, (a.shape, shape)
        return a

    gr, gd, gn, ga = g(d_rgb, (3, H, W)), g(d_depth, (H, W)), g(d_normal, (3, H, W)), g(d_alpha, (H, W))
    d_params = np.zeros((15, n))
    d_screen = np.zeros((16, n))
    pp = np.zeros(6)
    pi = np.zeros(6)
    w = None if watch is None else np.ascontiguousarray(np.asarray(watch, dtype=np.uint8))
    touched = None if watch is None else np.zeros(n, dtype=np.uint8)
    k = _consts(filter, use_rect)
    d_scale = np.zeros((15, n)) if scale else None
    ps = np.zeros(6) if scale else None
    sm = None if scale_mask is None else np.ascontiguousarray(np.asarray(scale_mask, dtype=np.uint8))
    assert sm is None or sm.shape == (H, W)
    psm = np.zeros(6) if (scale and sm is not None) else None
    lib.orc_backward(_ptr(p), n, ctypes.byref(c), _ptr(T), ctypes.byref(k), _threads(nthreads),
                     _ptr(gr), _ptr(gd), _ptr(gn), _ptr(ga), _ptr(d_params), _ptr(d_screen), _ptr(pp),
                     _ptr(pi), _ptr(w), _ptr(touched), _ptr(d_scale), _ptr(ps), _ptr(sm), _ptr(psm))
    out = {"d_params": d_params, "d_screen": d_screen, "pose_paper": pp, "pose_identity": pi}
    if scale:
        out["d_scale"] = d_scale
        out["pose_scale"] = ps
        if psm is not None:
            out["pose_scale_masked"] = psm
    if touched is not None:
        out["touched"] = touched.astype(bool)
    return out


def contribution(params, camera, pose, filter: bool = True, margin: float = 1e-5, nthreads=None):
    """Per-surfel contribution C_k^V = sum over pixels of w_k(p) (eq:contribution).

    Returns {"contrib": [n] FP64, "touched": [n] bool}: touched marks surfels evaluated
    at a pixel whose smallest decision margin is below `margin` (their pixel sets may
    differ in float32).
    """
    lib = _load()
    p, T = _prep(params, pose)
    c = _cam(camera)
    n = p.shape[1]
    contrib = np.zeros(n)
    touched = np.zeros(n, dtype=np.uint8)
    k = _consts(filter, True)
    lib.orc_contribution(_ptr(p), n, ctypes.byref(c), _ptr(T), ctypes.byref(k), _threads(nthreads),
                         ctypes.c_double(margin), _ptr(contrib), _ptr(touched))
    return {"contrib": contrib, "touched": touched.astype(bool)}


def depth_variants(params, camera, pose, filter: bool = True, nthreads=None):
    """The normalised depth D/O and the median depth (depth of the last composited
    intersection whose incoming transmittance exceeds 1/2).

    Returns {"depth_norm", "depth_median", "margin"} ([H,W] each, FP64); margin is the
    pixel's smallest relative margin to any decision, the median's T > 1/2 included.
    """
    lib = _load()
    p, T = _prep(params, pose)
    c = _cam(camera)
    H, W = c.height, c.width
    out = {"depth_norm": np.zeros((H, W)), "depth_median": np.zeros((H, W)), "margin": np.zeros((H, W))}
    k = _consts(filter, True)
    lib.orc_depth_variants(_ptr(p), p.shape[1], ctypes.byref(c), _ptr(T), ctypes.byref(k), _threads(nthreads),
                           _ptr(out["depth_norm"]), _ptr(out["depth_median"]), _ptr(out["margin"]))
    return out


def preprocess(params, camera, pose, filter: bool = True):
    """Per-surfel culling flag, float32 depth key, exact box, pixel rect and cull margin."""
    lib = _load()
    p, T = _prep(params, pose)
    c = _cam(camera)
    n = p.shape[1]
    culled = np.zeros(n, dtype=np.int32)
    key = np.zeros(n, dtype=np.float32)
    aabb = np.zeros((4, n))
    rect = np.zeros((4, n), dtype=np.int32)
    margin = np.zeros(n)
    k = _consts(filter, True)
    lib.orc_preprocess(_ptr(p), n, ctypes.byref(c), _ptr(T), ctypes.byref(k), _ptr(culled), _ptr(key),
                       _ptr(aabb), _ptr(rect), _ptr(margin))
    return {"culled": culled.astype(bool), "key": key, "aabb": aabb, "rect": rect, "cull_margin": margin}
