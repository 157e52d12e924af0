"""Seeded synthetic scenes, cameras and targets.

This module only draws inputs: Gaussian parameter planes, pinhole cameras and
target images. It contains none of the rasterizer, optimiser or consensus
arithmetic, so that the FP64 oracle and the HIP path can both be fed from it
without sharing any method code.

Parameter layout (one FP32 plane per scalar attribute, ``[A][N]``), following
the attribute list x = {u, q, s, f, o} of the Gaussian-splatting preliminaries
(Sec. 3.1, Eq. 1-3):

    planes 0..2    mean u (x, y, z)
    planes 3..6    rotation quaternion q (w, x, y, z), unnormalised
    planes 7..9    log of the scale s
    plane  10      opacity logit (opacity = sigmoid(logit))
    planes 11..    SH coefficients f: plane 11 + 3*k + channel, k = l*l + l + m

so A = 11 + 3 (d + 1)^2 (14 at degree 0, 59 at degree 3).

Cameras are world-to-camera rigid transforms with OpenCV axes (x right,
y down, z forward), fx/fy/cx/cy in pixels.  Random draws use
``numpy.random.Generator(PCG64(seed))`` in FP64 and are cast to FP32 once.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# plane offsets of the attribute groups (see module docstring)
MEAN, QUAT, LOGSCALE, OPACITY, SH = 0, 3, 7, 10, 11
# 1/(2 sqrt(pi)): value of the constant real spherical harmonic.  Used only to
# draw degree-0 colour coefficients whose rendered colour is a given U(0,1)
# sample (the configuration states colours, not coefficients).
_SH_DC_VALUE = 0.28209479177387814


def n_attr(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Camera:
    R: np.ndarray            # [3,3] world -> camera rotation (rows: right, down, forward)
    t: np.ndarray            # [3]   world -> camera translation
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def center(self) -> np.ndarray:
        return -self.R.T @ self.t


def look_at(eye, target, width, height, fx=None, fy=None, up=(0.0, 1.0, 0.0)) -> Camera:
    """Pinhole camera at ``eye`` looking at ``target`` with world-up +y.

    Rows of R are [right; down; forward] with forward = normalise(target-eye),
    right = normalise(forward x up), down = forward x right.  Focal length
    defaults to a 60 degree horizontal field of view; principal point is the
    image centre."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float32).astype(np.float64)
    t = (-R @ eye).astype(np.float32).astype(np.float64)
    if fx is None:
        fx = width / (2.0 * math.tan(math.radians(30.0)))
    if fy is None:
        fy = fx
    return Camera(R, t, float(np.float32(fx)), float(np.float32(fy)),
                  width / 2.0, height / 2.0, int(width), int(height))


def gaussians(n, sh_degree, seed, lo, hi, logscale_mu, logscale_sigma,
              dc="uniform_coef", rest_sigma=0.05) -> np.ndarray:
    """Draw ``n`` Gaussians as a ``[A][n]`` FP32 plane array.

    Draw order: means, log-scales, quaternions, opacity logits, SH DC, SH rest.
    ``dc='colour'`` draws the rendered degree-0 colour c ~ U(0,1) and stores the
    coefficient whose value is c (coefficient = (c - 0.5) / Y00);
    ``dc='uniform_coef'`` draws the DC coefficients themselves from U(0,1).
    """
    g = rng(seed)
    A = n_attr(sh_degree)
    out = np.zeros((A, n), np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    out[MEAN:MEAN + 3] = (lo[:, None] + (hi - lo)[:, None] * g.random((3, n)))
    out[LOGSCALE:LOGSCALE + 3] = g.normal(logscale_mu, logscale_sigma, (3, n))
    q = g.normal(0.0, 1.0, (4, n))
    out[QUAT:QUAT + 4] = q / np.linalg.norm(q, axis=0, keepdims=True)
    out[OPACITY] = g.normal(0.0, 1.0, n)
    dcv = g.random((3, n))
    if dc == "colour":
        dcv = (dcv - 0.5) / _SH_DC_VALUE
    out[SH:SH + 3] = dcv
    nrest = 3 * ((sh_degree + 1) ** 2 - 1)
    if nrest:
        out[SH + 3:] = g.normal(0.0, rest_sigma, (nrest, n))
    return out.astype(np.float32)


def target_images(seed, cams) -> list:
    """One U(0,1) target [3][H][W] per camera; camera v uses seed + 1 + v."""
    return [rng(seed + 1 + v).random((3, c.height, c.width)).astype(np.float32)
            for v, c in enumerate(cams)]


def ring_cameras(n, radius, height, width, img_h, center=(0.0, 0.0, 0.0), fx=None):
    """n cameras on a horizontal ring around ``center`` looking at it."""
    c = np.asarray(center, np.float64)
    cams = []
    for k in range(n):
        th = 2.0 * math.pi * k / n
        eye = c + np.array([radius * math.cos(th), height, radius * math.sin(th)])
        cams.append(look_at(eye, c, width, img_h, fx, fx))
    return cams


@dataclass
class Scene:
    name: str
    params: np.ndarray               # [A][N] FP32
    sh_degree: int
    cams: list
    targets: list = field(default_factory=list)
    seed: int = 0


def config1() -> Scene:
    """Parity case: 2,000 Gaussians, SH degree 0, four 128x128 views at radius 3."""
    seed = 1001
    p = gaussians(2000, 0, seed, [-1, -1, -1], [1, 1, 1], -4.0, 0.5, dc="colour")
    cams = []
    for k in range(4):
        a = k * math.pi / 2
        cams.append(look_at([3 * math.sin(a), 0.0, 3 * math.cos(a)], [0, 0, 0], 128, 128, 150.0, 150.0))
    return Scene("plain-2k-sh0-4x128", p, 0, cams, target_images(seed, cams), seed)


def config2(n=500_000, n_cams=64, width=1600, height=1066) -> Scene:
    """Scale case: 500k Gaussians, SH degree 3, 1600x1066 views on a 40 m ring."""
    seed = 1002
    p = gaussians(n, 3, seed, [-50, -10, -50], [50, 10, 50], -3.0, 0.7)
    cams = ring_cameras(n_cams, 40.0, 10.0, width, height)
    return Scene(f"plain-{n // 1000}k-sh3-{width}x{height}", p, 3, cams, [], seed)


def config2_targets(scene: Scene, views) -> list:
    return [rng(scene.seed + 1 + v).random((3, scene.cams[v].height, scene.cams[v].width)).astype(np.float32)
            for v in views]


def config5(n=6_000_000) -> Scene:
    """Serving case: the global model, 6M Gaussians, SH degree 3, in the same
    100 x 20 x 100 m box as the scale case (drawn in chunks of 1M, chunk c
    with seed 1005 * 1000 + c, so the FP64 temporaries stay small)."""
    seed = 1005
    step = 1_000_000
    parts = [gaussians(min(step, n - a), 3, seed * 1000 + a // step, [-50, -10, -50], [50, 10, 50], -3.0, 0.7)
             for a in range(0, n, step)]
    p = np.concatenate(parts, axis=1) if len(parts) > 1 else parts[0]
    return Scene(f"serve-{n // 1_000_000}M-sh3", p, 3, [], [], seed)


def config4b(n=2_000_000, width=1920, height=1080) -> Scene:
    """Adjoint case at scale: 2M Gaussians, SH degree 3, in the 100 x 20 x 100 m
    box, one 1920x1080 view from the 40 m ring at 10 m height (drawn in chunks
    of 1M with seed 1044 * 1000 + chunk)."""
    seed = 1044
    step = 1_000_000
    parts = [gaussians(min(step, n - a), 3, seed * 1000 + a // step, [-50, -10, -50], [50, 10, 50], -3.0, 0.7)
             for a in range(0, n, step)]
    p = np.concatenate(parts, axis=1) if len(parts) > 1 else parts[0]
    cams = [look_at([40.0 * math.cos(0.3), 10.0, 40.0 * math.sin(0.3)], [0, 0, 0], width, height)]
    return Scene(f"adjoint-{n // 1_000_000}M-sh3-{width}x{height}", p, 3, cams, [], seed)


def config4a() -> Scene:
    """Adjoint case: 200 Gaussians, SH degree 3, one 64x64 view (fx = 75)."""
    seed = 1004
    p = gaussians(200, 3, seed, [-0.5] * 3, [0.5] * 3, -2.5, 0.3)
    cams = [look_at([0.0, 0.0, 3.0], [0, 0, 0], 64, 64, 75.0, 75.0)]
    return Scene("adjoint-200-sh3-64x64", p, 3, cams, [], seed)


def edge_cases():
    """A 64x64 view (fx = fy = 60, camera at (0, 0, 3) looking at the origin)
    of 60 config-4a-style Gaussians (SH degree 3, seed 1200) plus eight
    placed ones, each making one rule of the rasterizer act (Gaussians 60..67):
      60, 61  negative SH DC: colour clamped at zero (all channels; red only);
      62, 63  opacity logit 10 and 9 at a few pixels' distance scale: the
              alpha clamp at 0.99 acts at the pixels nearest their centres;
      64, 65  beyond 1.3x the half field of view (x/z = 0.86, y/z = 0.75)
              and large: the Jacobian clamp acts, their footprints reach the
              image;
      66      camera depth 0.23, just past the near plane at 0.2;
      67      camera depth 0.15, before the near plane (culled).
    Depths are all distinct.  Returns (planes [A][68] FP32, camera); render
    with a non-black background."""
    base = gaussians(60, 3, 1200, [-0.5] * 3, [0.5] * 3, -2.5, 0.3).astype(np.float64)
    A = base.shape[0]
    placed = []

    def add(mean, logscale, logit, dc, q=(1.0, 0.0, 0.0, 0.0), seed=0):
        g = np.zeros(A, np.float64)
        g[MEAN:MEAN + 3] = mean
        g[QUAT:QUAT + 4] = q
        g[LOGSCALE:LOGSCALE + 3] = logscale
        g[OPACITY] = logit
        g[SH:SH + 3] = dc
        g[SH + 3:] = rng(1277 + seed).normal(0.0, 0.02, A - SH - 3)
        placed.append(g)

    add((-0.3, 0.2, 0.0), (-2.3, -2.1, -2.4), 0.5, (-2.5, -2.5, -2.5), seed=1)
    add((0.1, -0.25, 0.2), (-2.2, -2.2, -2.0), 0.8, (-2.5, 1.0, -1.5), q=(0.9, 0.3, -0.2, 0.1), seed=2)
    add((0.0, 0.0, 0.3), (-1.0, -1.1, -1.0), 10.0, (1.0, 0.5, 0.2), seed=3)
    add((-0.25, -0.3, 0.1), (-0.9, -1.3, -1.0), 9.0, (0.2, 1.2, 0.4), q=(0.8, 0.0, 0.5, 0.3), seed=4)
    add((2.55, 0.0, 0.05), (0.0, -0.2, -0.1), 0.0, (0.8, 0.6, 0.4), seed=5)
    add((0.1, -2.4, -0.2), (-0.3, -0.1, -0.3), -0.5, (0.3, 0.9, 0.7), q=(0.7, 0.1, 0.1, 0.7), seed=6)
    add((0.05, -0.03, 2.77), (-4.5, -4.4, -4.6), 1.0, (0.9, 0.1, 0.6), seed=7)
    add((-0.02, 0.04, 2.85), (-4.0, -4.0, -4.0), 1.0, (0.9, 0.9, 0.9), seed=8)
    p = np.concatenate([base, np.stack(placed, 1)], 1).astype(np.float32)
    cam = look_at([0.0, 0.0, 3.0], [0, 0, 0], 64, 64, 60.0, 60.0)
    return p, cam


SLAB_BOUNDS = (-50.0, -39.333, -19.333, 10.0, 50.0)
BLOCK_COUNTS = (800_000, 1_500_000, 2_200_000, 3_000_000)


@dataclass
class BlockScene:
    """K spatial blocks sharing boundary Gaussians (global ids)."""
    params_global: np.ndarray        # [A][N_global]
    sh_degree: int
    local_gid: list                  # per block: int64 global ids of its local copies
    own: list                        # per block: number of own Gaussians (first entries)
    cams: list                       # per block: list of cameras
    seed: int


def block_scene(counts=BLOCK_COUNTS, bounds=SLAB_BOUNDS, share=0.10, n_cams=32,
                width=1600, height=1066, sh_degree=3, seed=1003, y_range=(-10.0, 10.0), z_range=(-50.0, 50.0),
                logscale=(-3.0, 0.7), ring_radius=40.0, ring_height=10.0, fx=None) -> BlockScene:
    """Blocks as x-slabs of uniform density; the ``share`` fraction of each
    block's own Gaussians nearest the plane it shares with neighbour
    n(k) = k + 1 (n(K-1) = K-2) is copied into n(k) under the same global id.
    Block k draws with seed 100 * seed + k; its cameras sit on a ring around
    its slab centre."""
    K = len(counts)
    parts, gids, base = [], [], 0
    for k in range(K):
        lo = [bounds[k], y_range[0], z_range[0]]
        hi = [bounds[k + 1], y_range[1], z_range[1]]
        parts.append(gaussians(counts[k], sh_degree, seed * 100 + k, lo, hi, logscale[0], logscale[1]))
        gids.append(np.arange(base, base + counts[k], dtype=np.int64))
        base += counts[k]
    params_global = np.concatenate(parts, axis=1)
    received = [[] for _ in range(K)]
    for k in range(K):
        nb = k + 1 if k + 1 < K else K - 2
        plane = bounds[k + 1] if nb > k else bounds[k]
        xs = parts[k][MEAN]
        m = int(round(share * counts[k]))
        near = np.argsort(np.abs(xs.astype(np.float64) - plane), kind="stable")[:m]
        received[nb].append(np.sort(gids[k][near]))
    local_gid = [np.concatenate([gids[k]] + received[k]) for k in range(K)]
    cams = []
    for k in range(K):
        cx = 0.5 * (bounds[k] + bounds[k + 1])
        cams.append(ring_cameras(n_cams, ring_radius, ring_height, width, height, center=(cx, 0.0, 0.0), fx=fx))
    return BlockScene(params_global, sh_degree, local_gid, list(counts), cams, seed)


@dataclass
class SplitInput:
    """A global model and a global camera set, to be split into blocks."""
    params_global: np.ndarray        # [A][N]
    sh_degree: int
    cams: list                       # global training views
    seed: int


def split_input(n=7_500_000, n_grid=8, width=1600, height=1066, sh_degree=3, seed=1005) -> SplitInput:
    """Global Gaussians with uneven density, 70% uniform over the
    100 x 20 x 100 m box and 30% in a cluster around (15, 0, -20) with
    standard deviations (8, 3, 8) (drawn in chunks of 1M with seed
    seed * 1000 + chunk); views on an n_grid x n_grid lattice 25 m above the
    ground plane over x, z in [-45, 45], each looking at the ground 15 m ahead
    along +z."""
    n_u = int(round(0.7 * n))
    step = 1_000_000
    parts = []
    for a in range(0, n, step):
        m = min(step, n - a)
        sd = seed * 1000 + a // step
        p = gaussians(m, sh_degree, sd, [-50, -10, -50], [50, 10, 50], -3.0, 0.7)
        lo_c = max(a, n_u) - a                  # entries of this chunk that belong to the cluster
        if lo_c < m:
            g = rng(sd + 500)
            k = m - lo_c
            p[MEAN:MEAN + 3, lo_c:] = (np.array([15.0, 0.0, -20.0])[:, None]
                                       + g.normal(0.0, 1.0, (3, k)) * np.array([8.0, 3.0, 8.0])[:, None])
        parts.append(p)
    params = np.concatenate(parts, axis=1)
    xs = np.linspace(-45.0, 45.0, n_grid)
    cams = [look_at([x, 25.0, z], [x, 0.0, z + 15.0], width, height) for z in xs for x in xs]
    return SplitInput(params, sh_degree, cams, seed)


def poisson_arrivals(rate, duration, seed):
    g = rng(seed)
    t, out = 0.0, []
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            return np.asarray(out)
        out.append(t)


SERVE_RESOLUTIONS = ((800, 600), (1280, 720), (1600, 1066), (1920, 1080))


def serve_requests(n, seed, radius=40.0, height=10.0):
    """Random render requests: resolution uniform over SERVE_RESOLUTIONS, pose
    azimuth U[0, 2 pi) on a ring looking at the origin."""
    g = rng(seed)
    cams = []
    for _ in range(n):
        w, h = SERVE_RESOLUTIONS[int(g.integers(0, len(SERVE_RESOLUTIONS)))]
        th = g.random() * 2.0 * math.pi
        cams.append(look_at([radius * math.cos(th), height, radius * math.sin(th)], [0, 0, 0], w, h))
    return cams
