"""ctypes front end of the FP64 C rasterizer oracle (test infrastructure).

Follows the Gaussian-splatting preliminaries (Sec. 3.1, Eq. 1-3) with the
readings stated in ``orc.c``.  Inputs are the FP32 parameter planes and
cameras; all arithmetic is FP64.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

FLAG_NAMES = {1: "alpha_min", 2: "T_min", 4: "depth_tie", 8: "alpha_max", 16: "near",
              32: "colour_clamp", 64: "jacobian_clip"}


class _Cam(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("W", ctypes.c_int), ("H", ctypes.c_int)]


class _Cfg(ctypes.Structure):
    _fields_ = [("near_z", ctypes.c_double), ("alpha_min", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("T_min", ctypes.c_double),
                ("dilation", ctypes.c_double), ("jac_clip", ctypes.c_double),
                ("bg", ctypes.c_double * 3)]


@dataclass
class Camera:
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @classmethod
    def of(cls, c):
        return cls(np.asarray(c.R, np.float64), np.asarray(c.t, np.float64), float(c.fx), float(c.fy),
                   float(c.cx), float(c.cy), int(c.width), int(c.height))

    def _c(self):
        s = _Cam()
        R = np.asarray(self.R, np.float32).astype(np.float64).ravel()
        t = np.asarray(self.t, np.float32).astype(np.float64).ravel()
        for k in range(9):
            s.R[k] = R[k]
        for k in range(3):
            s.t[k] = t[k]
        s.fx, s.fy = float(np.float32(self.fx)), float(np.float32(self.fy))
        s.cx, s.cy = float(np.float32(self.cx)), float(np.float32(self.cy))
        s.W, s.H = self.width, self.height
        return s


@dataclass
class RasterConfig:
    """Constants of the stated readings: near plane 0.2, alpha in [1/255, 0.99],
    T_min 1e-4, 0.3 px^2 screen-space dilation, Jacobian clamp at 1.3x the
    half field of view, black background."""
    near_z: float = 0.2
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    dilation: float = 0.3
    jac_clip: float = 1.3
    bg: tuple = (0.0, 0.0, 0.0)

    def _c(self):
        s = _Cfg()
        # the GPU path holds these constants in FP32; use the same rounded values
        f = lambda v: float(np.float32(v))  # noqa: E731
        s.near_z, s.alpha_min, s.alpha_max = f(self.near_z), f(self.alpha_min), f(self.alpha_max)
        s.T_min, s.dilation, s.jac_clip = f(self.T_min), f(self.dilation), f(self.jac_clip)
        for k in range(3):
            s.bg[k] = f(self.bg[k])
        return s


_lib = None


def load_library():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        P = ctypes.POINTER
        dp, ip, lp = P(ctypes.c_double), P(ctypes.c_int), P(ctypes.c_long)
        lib.orc_project.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_long, P(_Cam), P(_Cfg), dp]
        lib.orc_render.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_long, P(_Cam), P(_Cfg),
                                   lp, ctypes.c_long, dp, dp, ip, ip, dp]
        lib.orc_backward.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_long, P(_Cam), P(_Cfg),
                                     lp, ctypes.c_long, dp, dp, dp]
        lib.orc_sh_basis.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp, dp]
        lib.orc_quat_rot.argtypes = [ctypes.c_long, dp, dp]
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None else None


def _planes(params):
    """FP64 copy of the planes.  FP32 inputs convert exactly; FP64 inputs are
    used as given (finite-difference checks perturb them)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    A, n = p.shape
    deg = int(round(((A - 11) / 3) ** 0.5)) - 1
    if 11 + 3 * (deg + 1) ** 2 != A or not 0 <= deg <= 3:
        raise ValueError("parameter planes do not match an SH degree in 0..3")
    return p, n, deg


def project(params, cam, cfg=None) -> dict:
    """Per-Gaussian projection into one view (EWA reading of X^proj, Sec. 3.1)."""
    cfg = cfg or RasterConfig()
    p, n, deg = _planes(params)
    out = np.zeros((max(n, 1), 20), np.float64)
    lib = load_library()
    rc = lib.orc_project(n, deg, _ptr(p, ctypes.c_double), n, ctypes.byref(Camera.of(cam)._c()),
                         ctypes.byref(cfg._c()), _ptr(out, ctypes.c_double))
    if rc:
        raise ValueError("orc_project failed")
    out = out[:n]
    return {"valid": out[:, 0] > 0.5, "mean2d": out[:, 1:3], "conic": out[:, 3:6], "depth": out[:, 6],
            "opacity": out[:, 7], "rgb": out[:, 8:11], "cov2d": out[:, 11:14], "tcam": out[:, 14:17],
            "clip_gap": out[:, 17], "colour_gap": out[:, 18], "near_gap": out[:, 19]}


def render(params, cam, cfg=None, pixels=None) -> dict:
    """Eq. 2 at every pixel (or at the listed linear pixel indices y*W + x).

    Returns rgb [3][H][W] (or [3][npix]), final transmittance, contributor
    count, per-pixel decision flags, and first-order bounds on what an FP32
    evaluation of the same pixel may differ by: T_err relative to T, rgb_err
    absolute per channel."""
    cfg = cfg or RasterConfig()
    p, n, deg = _planes(params)
    c = Camera.of(cam)
    if pixels is None:
        npix, pix = c.width * c.height, None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        npix = pix.size
    rgb = np.zeros((max(npix, 1), 3))
    T = np.zeros(max(npix, 1))
    nc = np.zeros(max(npix, 1), np.int32)
    fl = np.zeros(max(npix, 1), np.int32)
    err = np.zeros((max(npix, 1), 4))
    lib = load_library()
    rc = lib.orc_render(n, deg, _ptr(p, ctypes.c_double), n, ctypes.byref(c._c()), ctypes.byref(cfg._c()),
                        _ptr(pix, ctypes.c_long), npix, _ptr(rgb, ctypes.c_double), _ptr(T, ctypes.c_double),
                        _ptr(nc, ctypes.c_int), _ptr(fl, ctypes.c_int), _ptr(err, ctypes.c_double))
    if rc:
        raise ValueError("orc_render failed")
    rgb, T, nc, fl, err = rgb[:npix], T[:npix], nc[:npix], fl[:npix], err[:npix]
    if pixels is None:
        H, W = c.height, c.width
        return {"rgb": rgb.T.reshape(3, H, W).copy(), "T": T.reshape(H, W), "n": nc.reshape(H, W),
                "flags": fl.reshape(H, W), "T_err": err[:, 0].reshape(H, W).copy(),
                "rgb_err": err[:, 1:].T.reshape(3, H, W).copy()}
    return {"rgb": rgb.T.copy(), "T": T, "n": nc, "flags": fl, "T_err": err[:, 0].copy(), "rgb_err": err[:, 1:].T.copy()}


def backward(params, cam, dLdC, cfg=None, pixels=None, screen=False):
    """Gradient of sum(dLdC * C) w.r.t. the raw parameter planes (FP64, [A][N]).

    dLdC is [3][H][W] (or [3][npix] with ``pixels``).  With ``screen=True``
    also returns the per-Gaussian screen-space gradients
    (mean2d x, y, conic a, b, c, opacity, r, g, b) as [N][9]."""
    cfg = cfg or RasterConfig()
    p, n, deg = _planes(params)
    c = Camera.of(cam)
    g = np.asarray(dLdC, np.float64)
    if pixels is None:
        npix, pix = c.width * c.height, None
        gl = np.ascontiguousarray(g.reshape(3, -1).T)
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        npix = pix.size
        gl = np.ascontiguousarray(g.reshape(3, -1).T)
    grad = np.zeros((p.shape[0], max(n, 1)))
    sg = np.zeros((max(n, 1), 9)) if screen else None
    lib = load_library()
    rc = lib.orc_backward(n, deg, _ptr(p, ctypes.c_double), n, ctypes.byref(c._c()), ctypes.byref(cfg._c()),
                          _ptr(pix, ctypes.c_long), npix, _ptr(gl, ctypes.c_double), _ptr(grad, ctypes.c_double),
                          _ptr(sg, ctypes.c_double))
    if rc:
        raise ValueError("orc_backward failed")
    grad = grad[:, :n]
    return (grad, sg[:n]) if screen else grad


def sh_basis(deg, dirs, with_grad=False):
    """Real orthonormal SH (Condon-Shortley phase, m = -l..l) at unit dirs [n][3]."""
    d = np.ascontiguousarray(dirs, np.float64)
    n = d.shape[0]
    nk = (deg + 1) ** 2
    Y = np.zeros((n, nk))
    dY = np.zeros((n, nk, 3)) if with_grad else None
    load_library().orc_sh_basis(deg, n, _ptr(d, ctypes.c_double), _ptr(Y, ctypes.c_double), _ptr(dY, ctypes.c_double))
    return (Y, dY) if with_grad else Y


def quat_rotation(q):
    q = np.ascontiguousarray(q, np.float64).reshape(-1, 4)
    R = np.zeros((q.shape[0], 9))
    load_library().orc_quat_rot(q.shape[0], _ptr(q, ctypes.c_double), _ptr(R, ctypes.c_double))
    return R.reshape(-1, 3, 3)


def l1_loss_and_grad(rgb, target, weight=1.0):
    """L1 part of Eq. 3: weight * mean |C - target| over 3HW, and dL/dC
    (sign(0) = 0)."""
    d = np.asarray(rgb, np.float64) - np.asarray(target, np.float64)
    n = d.size
    return weight * np.abs(d).sum() / n, weight * np.sign(d) / n
