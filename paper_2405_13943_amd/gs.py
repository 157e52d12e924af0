"""ctypes binding of libgs (``include/gs.h``): argument marshalling only.

Every step of the rasterizer training step runs in the HIP kernels of
``libgs.so``; this module turns torch device tensors into pointers, builds the
C structs and raises on a non-OK status.  There is no fallback: if the library
is not built, importing this module fails.

torch is imported first so that libgs resolves the HIP runtime to the copy
torch already loaded (one runtime per process).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import build as _build

c_f, c_i32, c_i64, c_u64, c_vp = ctypes.c_float, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p

GS_OK, GS_E_INVALID, GS_E_CAPACITY, GS_E_DEVICE, GS_E_UNSUPPORTED = range(5)
GS_STATUS_PAIR_OVERFLOW, GS_STATUS_NONFINITE = 1, 2
GS_WAVES_ADAPTIVE = -1
CTR_VISIBLE, CTR_PAIRS, CTR_STATUS, CTR_OVERFLOWED, N_COUNTERS = 0, 1, 2, 3, 4
LOSS_L1, LOSS_EXTERNAL = 0, 1
REC_WORDS, META_WORDS = 12, 4
MEAN_PLANE = 0            # the three mean planes lead the parameter layout


class GsParams(ctypes.Structure):
    _fields_ = [("data", c_vp), ("n", c_i64), ("stride", c_i64), ("sh_degree", c_i32), ("reserved", c_i32)]


class GsCamera(ctypes.Structure):
    _fields_ = [("R", c_f * 9), ("t", c_f * 3), ("fx", c_f), ("fy", c_f), ("cx", c_f), ("cy", c_f),
                ("width", c_i32), ("height", c_i32)]


class GsJob(ctypes.Structure):
    _fields_ = [("cam", c_i32), ("tiles_x", c_i32), ("tiles_y", c_i32), ("tile0", c_i32), ("g0", c_i64),
                ("g1", c_i64), ("rec0", c_i64), ("px0", c_i64), ("loss_weight", c_f), ("reserved", c_i32)]


class GsFrame(ctypes.Structure):
    _fields_ = [("cams", c_vp), ("jobs", c_vp), ("n_jobs", c_i32), ("n_tiles", c_i32), ("n_records", c_i64),
                ("n_pixels", c_i64), ("g_max", c_i64), ("jobs_disjoint", c_i32), ("reserved", c_i32)]


class GsRasterCfg(ctypes.Structure):
    _fields_ = [("tile_w", c_i32), ("tile_h", c_i32), ("near_z", c_f), ("alpha_min", c_f), ("alpha_max", c_f),
                ("T_min", c_f), ("dilation", c_f), ("jac_clip", c_f), ("bg", c_f * 3), ("fwd_waves", ctypes.c_int16),
                ("bwd_waves", ctypes.c_int16)]


class GsBins(ctypes.Structure):
    _fields_ = [("vals", c_vp), ("ranges", c_vp), ("pair_off", c_vp), ("counters", c_vp), ("capacity", c_u64),
                ("tile_order", c_vp), ("qmask", c_vp)]


class GsAdamCfg(ctypes.Structure):
    _fields_ = [("lr", c_f * 5), ("rho", c_f * 5), ("beta1", c_f), ("beta2", c_f), ("eps", c_f),
                ("reserved", c_i32), ("step", c_i64)]


class GsTuneChoice(ctypes.Structure):
    _fields_ = [("tile_w", c_i32), ("tile_h", c_i32), ("fwd_waves", c_i32), ("bwd_waves", c_i32)]


TUNE_STEP_FN = ctypes.CFUNCTYPE(c_i32, ctypes.POINTER(GsTuneChoice), c_vp)


class GsError(RuntimeError):
    pass


def _load():
    path = os.environ.get("GS_LIBRARY", _build.LIB)
    if not os.path.exists(path):
        raise ImportError(f"libgs.so not found at {path}; build it with `python -m paper_2405_13943_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    sigs = {
        "gs_abi_version": ([], c_i32),
        "gs_last_error": ([], ctypes.c_char_p),
        "gs_raster_cfg_default": ([P(GsRasterCfg)], None),
        "gs_frame_plan": ([P(GsCamera), c_i32, P(GsJob), c_i32, P(GsRasterCfg), P(c_i64), P(c_i64), P(c_i32),
                           P(c_i64), P(c_i32)], c_i32),
        "gs_project": ([P(GsParams), P(GsFrame), P(GsRasterCfg), c_vp, c_vp, c_vp, c_vp], c_i32),
        "gs_project_f64": ([P(GsParams), P(GsFrame), P(GsRasterCfg), c_vp, c_vp, c_vp, c_vp], c_i32),
        "gs_bin_sort_workspace_size": ([c_i64, c_u64, c_i32], ctypes.c_size_t),
        "gs_bin_sort": ([P(GsFrame), P(GsRasterCfg), c_vp, P(GsBins), c_vp, ctypes.c_size_t, c_vp], c_i32),
        "gs_bin_sort_noalloc_max_bytes": ([], ctypes.c_size_t),
        "gs_bin_sort_noalloc": ([P(GsFrame), P(GsRasterCfg), c_vp, P(GsBins), c_vp], c_i32),
        "gs_render_fwd": ([P(GsFrame), P(GsRasterCfg), c_vp, P(GsBins), c_vp, c_vp, c_vp, c_vp], c_i32),
        "gs_render_fwd_f64": ([P(GsFrame), P(GsRasterCfg), c_vp, P(GsBins), c_vp, c_vp, c_vp, c_vp], c_i32),
        "gs_render_fwd_stats": ([P(GsFrame), P(GsRasterCfg), c_vp, P(GsBins), c_vp, c_vp, c_vp, c_vp, c_vp], c_i32),
        "gs_render_bwd_workspace_size": ([c_u64, c_i32], ctypes.c_size_t),
        "gs_render_bwd": ([P(GsParams), P(GsFrame), P(GsRasterCfg), c_vp, c_vp, P(GsBins), c_vp, c_vp, c_i32, c_vp,
                           c_vp, P(GsParams), c_vp, ctypes.c_size_t, c_vp], c_i32),
        "gs_render_bwd_f64": ([P(GsParams), P(GsFrame), P(GsRasterCfg), c_vp, c_vp, P(GsBins), c_vp, c_vp, c_i32,
                               c_vp, c_vp, P(GsParams), c_vp, ctypes.c_size_t, c_vp], c_i32),
        "gs_adam_admm": ([P(GsParams), P(GsParams), P(GsParams), P(GsParams), P(GsParams), c_vp, P(GsAdamCfg),
                          c_vp, c_vp], c_i32),
        "gs_render_bwd_adam": ([P(GsParams), P(GsFrame), P(GsRasterCfg), c_vp, c_vp, P(GsBins), c_vp, c_vp, c_i32,
                                c_vp, c_vp, P(GsParams), P(GsParams), P(GsParams), c_vp, P(GsAdamCfg), c_vp,
                                ctypes.c_size_t, c_vp], c_i32),
        "gs_consensus": ([P(GsParams), P(GsParams), P(GsParams), P(GsParams), c_vp, c_vp, c_f, c_vp, c_vp], c_i32),
        "gs_penalty_update": ([P(c_f), P(c_f), c_f, c_f, c_f, P(c_f)], c_i32),
        "gs_ssim_workspace_size": ([c_i64], ctypes.c_size_t),
        "gs_split_scene": ([c_vp, c_i64, c_i32, c_i32, c_vp, c_vp], c_i32),
        "gs_spatial_order": ([c_vp, c_i64, c_i64, c_i32, c_i32, c_i32, c_vp], c_i32),
        "gs_split_group": ([c_vp, c_i32, ctypes.c_double, c_i32, c_vp, c_i64, c_vp, c_vp, c_i64, P(c_i64)], c_i32),
        "gs_ssim_loss_grad": ([P(GsFrame), P(GsRasterCfg), c_vp, c_vp, c_f, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp],
                              c_i32),
        "gs_dual_rescale": ([P(GsParams), P(GsParams), P(GsParams), c_vp, c_vp, P(c_f), c_vp], c_i32),
        "gs_set_tune_cache": ([ctypes.c_char_p], c_i32),
        "gs_autotune": ([ctypes.c_char_p, P(GsTuneChoice), c_i32, c_i32, TUNE_STEP_FN, c_vp, c_vp, P(GsTuneChoice),
                         P(ctypes.c_double)], c_i32),
        "gs_profile_set": ([ctypes.c_char_p], c_i32),
        "gs_profile_get": ([ctypes.c_char_p, P(ctypes.c_double), P(c_i64)], c_i32),
        "gs_profile_enable": ([c_i32], c_i32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _check(rc, what):
    if rc != GS_OK:
        raise GsError(f"{what} failed ({rc}): {lib.gs_last_error().decode()}")


def _stream():
    return c_vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return c_vp(t.data_ptr()) if t is not None else None


def n_attr(sh_degree):
    return 11 + 3 * (sh_degree + 1) ** 2


def sh_degree_of(n_planes):
    d = int(round(((n_planes - 11) / 3) ** 0.5)) - 1
    if n_attr(d) != n_planes or not 0 <= d <= 3:
        raise ValueError(f"{n_planes} planes do not match an SH degree in 0..3")
    return d


def params_struct(t: torch.Tensor, sh_degree=None) -> GsParams:
    """[A][N] plane tensor (rows may be strided) -> gs_params."""
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("parameter planes must be a [A][N] tensor with unit inner stride")
    if not t.is_cuda:
        raise ValueError("parameter planes must live on the GPU")
    d = sh_degree_of(t.shape[0]) if sh_degree is None else sh_degree
    return GsParams(t.data_ptr(), t.shape[1], t.stride(0), d, 0)


def raster_cfg(tile=(16, 16), near_z=0.2, alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4, dilation=0.3,
               jac_clip=1.3, bg=(0.0, 0.0, 0.0), fwd_waves=1, bwd_waves=1) -> GsRasterCfg:
    """tile: (w, h) binning tile, optionally followed by the forward's and the
    backward's wavefronts per tile: (w, h, fwd_waves[, bwd_waves])."""
    c = GsRasterCfg()
    lib.gs_raster_cfg_default(ctypes.byref(c))
    tile = tuple(tile)
    if len(tile) >= 3:
        fwd_waves = tile[2]
        bwd_waves = tile[3] if len(tile) >= 4 else tile[2]
    c.tile_w, c.tile_h = tile[:2]
    c.fwd_waves, c.bwd_waves = int(fwd_waves), int(bwd_waves)
    c.near_z, c.alpha_min, c.alpha_max, c.T_min = near_z, alpha_min, alpha_max, T_min
    c.dilation, c.jac_clip = dilation, jac_clip
    for k in range(3):
        c.bg[k] = bg[k]
    return c


def camera_struct(cam) -> GsCamera:
    c = GsCamera()
    R = np.asarray(cam.R, np.float32).ravel()
    t = np.asarray(cam.t, np.float32).ravel()
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
    c.width, c.height = cam.width, cam.height
    return c


@dataclass
class JobSpec:
    cam: int
    g0: int
    g1: int
    loss_weight: float = 1.0


class Frame:
    """A planned set of render jobs with device copies of cameras and jobs."""

    def __init__(self, cams, jobs, cfg: GsRasterCfg, device="cuda"):
        self.cams_host = (GsCamera * max(len(cams), 1))(*[camera_struct(c) for c in cams])
        self.jobs_host = (GsJob * max(len(jobs), 1))()
        for i, j in enumerate(jobs):
            self.jobs_host[i].cam, self.jobs_host[i].g0, self.jobs_host[i].g1 = j.cam, j.g0, j.g1
            self.jobs_host[i].loss_weight = j.loss_weight
        nr, npx, nt, gm, dj = c_i64(), c_i64(), c_i32(), c_i64(), c_i32()
        _check(lib.gs_frame_plan(self.cams_host, len(cams), self.jobs_host, len(jobs), ctypes.byref(cfg),
                                 ctypes.byref(nr), ctypes.byref(npx), ctypes.byref(nt), ctypes.byref(gm),
                                 ctypes.byref(dj)), "gs_frame_plan")
        self.n_jobs, self.n_records, self.n_pixels, self.n_tiles = len(jobs), nr.value, npx.value, nt.value
        self.g_max, self.jobs_disjoint = gm.value, dj.value
        self.cams = [cams[j.cam] for j in jobs]
        cam_bytes = np.frombuffer(bytes(self.cams_host), np.uint8)
        job_bytes = np.frombuffer(bytes(self.jobs_host), np.uint8)
        self.cams_dev = torch.from_numpy(cam_bytes.copy()).to(device)
        self.jobs_dev = torch.from_numpy(job_bytes.copy()).to(device)
        self.struct = GsFrame(self.cams_dev.data_ptr(), self.jobs_dev.data_ptr(), len(jobs), self.n_tiles,
                              self.n_records, self.n_pixels, self.g_max, self.jobs_disjoint, 0)
        self.tile = (cfg.tile_w, cfg.tile_h)

    def job(self, i) -> GsJob:
        return self.jobs_host[i]

    def image(self, buf: torch.Tensor, i: int) -> torch.Tensor:
        """View of job i's [3][H][W] image inside a frame-sized colour buffer."""
        j, c = self.jobs_host[i], self.cams[i]
        return buf[3 * j.px0: 3 * j.px0 + 3 * c.width * c.height].view(3, c.height, c.width)

    def plane(self, buf: torch.Tensor, i: int) -> torch.Tensor:
        j, c = self.jobs_host[i], self.cams[i]
        return buf[j.px0: j.px0 + c.width * c.height].view(c.height, c.width)

    def images(self, buf):
        return [self.image(buf, i) for i in range(self.n_jobs)]


class Buffers:
    """Device buffers of one frame: records, bins, workspaces (torch-owned)."""

    def __init__(self, frame: Frame, capacity: int, dtype=torch.float32, device="cuda"):
        self.dtype = dtype
        self.f64 = dtype == torch.float64
        nr = max(frame.n_records, 1)
        self.rec = torch.empty(nr * REC_WORDS, dtype=dtype, device=device)
        self.meta = torch.empty(nr * META_WORDS, dtype=torch.int32, device=device)
        self.pair_off = torch.empty(nr, dtype=torch.int32, device=device)
        self.ranges = torch.empty(max(frame.n_tiles, 1) * 2, dtype=torch.int32, device=device)
        self.counters = torch.zeros(N_COUNTERS, dtype=torch.int32, device=device)
        self.rgb = torch.empty(max(frame.n_pixels, 1) * 3, dtype=dtype, device=device)
        self.T = torch.empty(max(frame.n_pixels, 1), dtype=dtype, device=device)
        self.ncontrib = torch.empty(max(frame.n_pixels, 1), dtype=torch.int32, device=device)
        self.tile_order = torch.empty(max(frame.n_tiles, 1) + 4, dtype=torch.int32, device=device)
        self.share_qmask = True    # the forward hands its quadrant masks to the backward
        self.frame = frame
        self._alloc_pairs(capacity, device)

    def _alloc_pairs(self, capacity, device="cuda"):
        self.capacity = int(max(capacity, 1))
        self.vals = torch.empty(self.capacity, dtype=torch.int32, device=device)
        self.qmask = torch.empty(self.capacity, dtype=torch.uint8, device=device)
        nb = lib.gs_bin_sort_workspace_size(self.frame.n_records, self.capacity, self.frame.n_tiles)
        self.bin_ws = torch.empty(nb, dtype=torch.uint8, device=device)
        nw = lib.gs_render_bwd_workspace_size(self.capacity, 1 if self.f64 else 0)
        self.bwd_ws = torch.empty(nw, dtype=torch.uint8, device=device)

    def grow(self, capacity):
        self._alloc_pairs(capacity, self.vals.device)

    @property
    def bins(self) -> GsBins:
        return GsBins(self.vals.data_ptr(), self.ranges.data_ptr(), self.pair_off.data_ptr(),
                      self.counters.data_ptr(), self.capacity, self.tile_order.data_ptr(),
                      self.qmask.data_ptr() if self.share_qmask else None)


# ---------------------------------------------------------------------------
# entry points

def status_ptr(buf):
    """Device address of a buffer's status word (its counters[CTR_STATUS])."""
    return c_vp(buf.counters.data_ptr() + 4 * CTR_STATUS)


def project(params: torch.Tensor, frame: Frame, cfg: GsRasterCfg, buf: Buffers):
    """Projection into buf's records; non-finite parameters it reads set
    GS_STATUS_NONFINITE in buf's status word."""
    p = params_struct(params)
    fn = lib.gs_project_f64 if params.dtype == torch.float64 else lib.gs_project
    _check(fn(ctypes.byref(p), ctypes.byref(frame.struct), ctypes.byref(cfg), _ptr(buf.rec), _ptr(buf.meta),
              status_ptr(buf), _stream()), "gs_project")


def bin_sort(frame: Frame, cfg: GsRasterCfg, buf: Buffers):
    b = buf.bins
    _check(lib.gs_bin_sort(ctypes.byref(frame.struct), ctypes.byref(cfg), _ptr(buf.meta), ctypes.byref(b),
                           _ptr(buf.bin_ws), buf.bin_ws.numel(), _stream()), "gs_bin_sort")


def bin_sort_noalloc(frame: Frame, cfg: GsRasterCfg, buf: Buffers):
    """gs_bin_sort with the library's static workspace (buf.bin_ws unused)."""
    b = buf.bins
    _check(lib.gs_bin_sort_noalloc(ctypes.byref(frame.struct), ctypes.byref(cfg), _ptr(buf.meta), ctypes.byref(b),
                                   _stream()), "gs_bin_sort_noalloc")


def render_fwd(frame: Frame, cfg: GsRasterCfg, buf: Buffers):
    b = buf.bins
    fn = lib.gs_render_fwd_f64 if buf.f64 else lib.gs_render_fwd
    _check(fn(ctypes.byref(frame.struct), ctypes.byref(cfg), _ptr(buf.rec), ctypes.byref(b), _ptr(buf.rgb),
              _ptr(buf.T), _ptr(buf.ncontrib), _stream()), "gs_render_fwd")


def render_fwd_stats(frame: Frame, cfg: GsRasterCfg, buf: Buffers) -> int:
    """Forward (FP32) that also counts the frame's (pixel, Gaussian)
    contributions; returns the count (host read)."""
    kept = torch.zeros(1, dtype=torch.int64, device=buf.rgb.device)
    b = buf.bins
    _check(lib.gs_render_fwd_stats(ctypes.byref(frame.struct), ctypes.byref(cfg), _ptr(buf.rec), ctypes.byref(b),
                                   _ptr(buf.rgb), _ptr(buf.T), _ptr(buf.ncontrib), _ptr(kept), _stream()),
           "gs_render_fwd_stats")
    return int(kept.item())


def render_bwd(params: torch.Tensor, frame: Frame, cfg: GsRasterCfg, buf: Buffers, grad_out: torch.Tensor,
               mode=LOSS_L1, grad_in: torch.Tensor = None, loss_out: torch.Tensor = None):
    """Backward into ``grad_out`` ([A][N] like params).  mode LOSS_L1: grad_in
    is the target (frame-sized colour buffer); LOSS_EXTERNAL: grad_in is dL/dC."""
    p = params_struct(params)
    g = params_struct(grad_out)
    b = buf.bins
    fn = lib.gs_render_bwd_f64 if buf.f64 else lib.gs_render_bwd
    _check(fn(ctypes.byref(p), ctypes.byref(frame.struct), ctypes.byref(cfg), _ptr(buf.rec), _ptr(buf.meta),
              ctypes.byref(b), _ptr(buf.rgb), _ptr(buf.ncontrib), mode, _ptr(grad_in), _ptr(loss_out),
              ctypes.byref(g), _ptr(buf.bwd_ws), buf.bwd_ws.numel(), _stream()), "gs_render_bwd")


def ssim_loss_grad(frame: Frame, cfg: GsRasterCfg, rgb: torch.Tensor, target: torch.Tensor, lam: float,
                   grad_out: torch.Tensor = None, loss_out: torch.Tensor = None, ws: torch.Tensor = None):
    """Eq. 3 with the D-SSIM term (gs_ssim_loss_grad): dL/dC into grad_out
    (allocated when None; pass it to the backward with LOSS_EXTERNAL) and
    the per-job loss added into loss_out.  ws: a uint8 device buffer of at
    least gs_ssim_workspace_size bytes (allocated when None)."""
    if grad_out is None:
        grad_out = torch.empty_like(rgb)
    if ws is None:
        ws = torch.empty(int(lib.gs_ssim_workspace_size(frame.n_pixels)), dtype=torch.uint8, device=rgb.device)
    _check(lib.gs_ssim_loss_grad(ctypes.byref(frame.struct), ctypes.byref(cfg), _ptr(rgb), _ptr(target), float(lam),
                                 _ptr(grad_out), _ptr(loss_out), _ptr(ws), ws.numel(), _stream()), "gs_ssim_loss_grad")
    return grad_out


def spatial_order(means, bits=10, chunk=16, strands=1):
    """Z-order of the Gaussians' means (gs_spatial_order): a permutation
    (int64 numpy array) for storing a model as params[:, perm]; with
    strands > 1, chunks of `chunk` Gaussians of the Z-order dealt over that
    many strands.  means: the three mean planes [3][n] (host array, or the
    parameter tensor's first three rows on any device)."""
    if isinstance(means, torch.Tensor):
        means = means[MEAN_PLANE:MEAN_PLANE + 3].detach().float().cpu().numpy()
    m = np.ascontiguousarray(means, dtype=np.float32)
    n = m.shape[1]
    perm = np.zeros(n, np.int64)
    _check(lib.gs_spatial_order(m.ctypes.data, n, n, int(bits), int(chunk), int(strands), perm.ctypes.data),
           "gs_spatial_order")
    return perm


def split_scene(points, K, ground_axes=(0, 2)):
    """Alg. 1 (gs_split_scene): the K cells' tight boxes [K][6] (lo xyz, hi
    xyz) and each point's cell, from host points [n][3]."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n = pts.shape[0]
    boxes = np.zeros((K, 6), np.float64)
    cell = np.zeros(n, np.int64)
    mask = sum(1 << a for a in ground_axes)
    _check(lib.gs_split_scene(pts.ctypes.data, n, int(K), mask, boxes.ctypes.data, cell.ctypes.data),
           "gs_split_scene")
    return boxes, cell


def split_group(boxes, scale, points, axes=(0, 1, 2)):
    """Overlap grouping (gs_split_group): per block, the ascending ids of the
    points its box scaled by ``scale`` covers on ``axes`` (all three for
    points, the ground axes for camera centres)."""
    b = np.ascontiguousarray(boxes, dtype=np.float64)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    K = b.shape[0]
    mask = sum(1 << a for a in axes)
    counts = np.zeros(K, np.int64)
    total = c_i64()
    _check(lib.gs_split_group(b.ctypes.data, K, float(scale), mask, pts.ctypes.data, pts.shape[0],
                              counts.ctypes.data, None, 0, ctypes.byref(total)), "gs_split_group")
    members = np.zeros(max(total.value, 1), np.int64)
    _check(lib.gs_split_group(b.ctypes.data, K, float(scale), mask, pts.ctypes.data, pts.shape[0],
                              counts.ctypes.data, members.ctypes.data, members.size, ctypes.byref(total)),
           "gs_split_group")
    ends = np.cumsum(counts)
    return [members[e - c:e] for c, e in zip(counts, ends)]


def adam_cfg(lr, rho, step, beta1=0.9, beta2=0.999, eps=1e-8) -> GsAdamCfg:
    c = GsAdamCfg()
    for k in range(5):
        c.lr[k], c.rho[k] = float(lr[k]), float(rho[k])
    c.beta1, c.beta2, c.eps, c.step = beta1, beta2, eps, int(step)
    return c


def adam_admm(x, g, m, v, w=None, mask=None, cfg: GsAdamCfg = None, status: Buffers = None):
    """status: a Buffers whose status word gates the update (skipped after a
    pair overflow) and receives GS_STATUS_NONFINITE; None: no status."""
    px, pg, pm, pv = (params_struct(t) for t in (x, g, m, v))
    pw = params_struct(w) if w is not None else None
    _check(lib.gs_adam_admm(ctypes.byref(px), ctypes.byref(pg), ctypes.byref(pm), ctypes.byref(pv),
                            ctypes.byref(pw) if pw is not None else None, _ptr(mask), ctypes.byref(cfg),
                            status_ptr(status) if status is not None else None, _stream()),
           "gs_adam_admm")


def render_bwd_adam(x: torch.Tensor, frame: Frame, cfg: GsRasterCfg, buf: Buffers, m, v, w=None, mask=None,
                    acfg: GsAdamCfg = None, mode=LOSS_L1, grad_in: torch.Tensor = None, loss_out: torch.Tensor = None):
    """Backward and Adam/ADMM update of x in one call (FP32, jobs over
    disjoint Gaussian ranges); equal to render_bwd into a gradient buffer
    followed by adam_admm."""
    px, pm, pv = (params_struct(t) for t in (x, m, v))
    pw = params_struct(w) if w is not None else None
    b = buf.bins
    _check(lib.gs_render_bwd_adam(ctypes.byref(px), ctypes.byref(frame.struct), ctypes.byref(cfg), _ptr(buf.rec),
                                  _ptr(buf.meta), ctypes.byref(b), _ptr(buf.rgb), _ptr(buf.ncontrib), mode,
                                  _ptr(grad_in),
                                  _ptr(loss_out), ctypes.byref(pm), ctypes.byref(pv),
                                  ctypes.byref(pw) if pw is not None else None, _ptr(mask), ctypes.byref(acfg),
                                  _ptr(buf.bwd_ws), buf.bwd_ws.numel(), _stream()), "gs_render_bwd_adam")


def consensus(x, u, w, z, holder_ptr, holder_idx, relax=1.0, resid=None):
    px, pu, pw, pz = (params_struct(t) for t in (x, u, w, z))
    _check(lib.gs_consensus(ctypes.byref(px), ctypes.byref(pu), ctypes.byref(pw), ctypes.byref(pz),
                            _ptr(holder_ptr), _ptr(holder_idx), float(relax), _ptr(resid), _stream()),
           "gs_consensus")


def penalty_update(resid, rho, mu=10.0, tau_inc=2.0, tau_dec=2.0):
    """Residual-balancing penalty update (gs_penalty_update, host only).
    resid: the 10 residual sums of a consensus call (tensor or sequence);
    returns (new rho, old/new scale) as tuples of 5 floats."""
    if isinstance(resid, torch.Tensor):
        resid = resid.detach().float().cpu().tolist()
    r = (c_f * 10)(*[float(v) for v in resid])
    rh = (c_f * 5)(*[float(v) for v in rho])
    sc = (c_f * 5)()
    _check(lib.gs_penalty_update(r, rh, float(mu), float(tau_inc), float(tau_dec), sc), "gs_penalty_update")
    return tuple(rh), tuple(sc)


def dual_rescale(u, w, z, holder_ptr, holder_idx, scale):
    """u_k *= scale[group], w_k = z - u_k over every held copy (gs_dual_rescale)."""
    pu, pw, pz = (params_struct(t) for t in (u, w, z))
    sc = (c_f * 5)(*[float(v) for v in scale])
    _check(lib.gs_dual_rescale(ctypes.byref(pu), ctypes.byref(pw), ctypes.byref(pz), _ptr(holder_ptr),
                               _ptr(holder_idx), sc, _stream()), "gs_dual_rescale")


def read_counters(buf: Buffers):
    c = buf.counters.cpu().numpy().astype(np.uint32)
    return {"visible": int(c[CTR_VISIBLE]), "pairs": int(c[CTR_PAIRS]), "status": int(c[CTR_STATUS]),
            "overflowed": int(c[CTR_OVERFLOWED])}


def rasterize(params: torch.Tensor, frame: Frame, cfg: GsRasterCfg, buf: Buffers = None, capacity=None):
    """project -> bin -> composite, growing the pair capacity when the device
    reports an overflow (one host read of the counters)."""
    if buf is None:
        buf = Buffers(frame, capacity or max(1 << 16, 8 * frame.n_records), params.dtype, params.device)
    project(params, frame, cfg, buf)
    while True:
        buf.counters.zero_()
        bin_sort(frame, cfg, buf)
        c = read_counters(buf)
        if not c["status"] & GS_STATUS_PAIR_OVERFLOW:
            break
        buf.grow(int(c["pairs"] * 1.25) + 1024)
    render_fwd(frame, cfg, buf)
    return buf


def set_tune_cache(path):
    """JSON file of the tuned launch shapes (None: in memory only)."""
    _check(lib.gs_set_tune_cache(path.encode() if path else None), "gs_set_tune_cache")


def autotune(key, candidates, run_step, reps=5):
    """gs_autotune: the fastest of ``candidates`` ((tile_w, tile_h, fwd_waves,
    bwd_waves) tuples) for workload ``key``, timed by the library over
    ``run_step(choice_tuple)`` calls on the current stream (or taken from its
    cache).  Returns (choice tuple, ms per step or -1 when cached without a
    time)."""
    cands = (GsTuneChoice * len(candidates))(*[GsTuneChoice(*map(int, c)) for c in candidates])
    failure = []

    def cb(choice, _user):
        c = choice.contents
        try:
            run_step((c.tile_w, c.tile_h, c.fwd_waves, c.bwd_waves))
            return 0
        except Exception as e:          # reported through the status, re-raised below
            failure.append(e)
            return 1
    fn = TUNE_STEP_FN(cb)
    best, ms = GsTuneChoice(), ctypes.c_double(-1.0)
    stream = _stream() if torch.cuda.is_available() else None   # a cached key needs no device
    rc = lib.gs_autotune(key.encode(), cands, len(candidates), int(reps), fn, None, stream, ctypes.byref(best),
                         ctypes.byref(ms))
    if failure:
        raise failure[0]
    _check(rc, "gs_autotune")
    return (best.tile_w, best.tile_h, best.fwd_waves, best.bwd_waves), ms.value


def profile_set(names):
    """Time the launches of the named kernels (list or comma string, "*" all,
    None off) with HIP events inside the library; resets the totals."""
    if names is not None and not isinstance(names, str):
        names = ",".join(names)
    _check(lib.gs_profile_set(names.encode() if names else None), "gs_profile_set")


def profile_enable(on):
    """Pause (False) or resume (True) event recording of the selected kernels,
    keeping their totals: times a sample of the launches."""
    _check(lib.gs_profile_enable(1 if on else 0), "gs_profile_enable")


def profile_get(name):
    """(summed duration in ms, launches) of a profiled kernel; waits for them."""
    ms, n = ctypes.c_double(), c_i64()
    _check(lib.gs_profile_get(name.encode(), ctypes.byref(ms), ctypes.byref(n)), "gs_profile_get")
    return ms.value, n.value
