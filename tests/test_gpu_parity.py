"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the
parity scene (2,000 Gaussians, SH degree 0, four 128x128 views) and on small
edge cases.

Tolerances (FP32 kernels vs FP64 oracle):
  - images: |C - C_ref| <= 1e-4 |C_ref| + 1e-6 on pixels the oracle does not
    flag as near a decision threshold;
  - gradients: per attribute group ||g - g_ref|| / ||g_ref|| <= 1e-3;
  - projection: 1e-5 relative (a few FP32 rounding steps);
  - Adam / consensus: 1e-6 relative + small absolute (a handful of FP32 ops);
  - binning: bit-exact against a stable sort of the same integer keys.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2405_13943_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2405_13943_amd import gs  # noqa: E402

LOG2E = 1.0 / math.log(2.0)
GROUPS = {"p": [0, 1, 2], "q": [3, 4, 5, 6], "s": [7, 8, 9], "o": [10]}


def group_planes(A):
    d = dict(GROUPS)
    d["f"] = list(range(11, A))
    return d


def make_frame(scene, cfg, views=None, weight=None):
    views = list(range(len(scene.cams))) if views is None else views
    n = scene.params.shape[1]
    w = weight if weight is not None else 1.0 / len(views)
    jobs = [gs.JobSpec(v, 0, n, w) for v in views]
    return gs.Frame(scene.cams, jobs, cfg)


def frame_target(frame, scene, views):
    return torch.cat([torch.from_numpy(scene.targets[v]).reshape(-1) for v in views]).cuda()


@pytest.fixture(scope="module")
def cfg1():
    return scenes.config1()


@pytest.fixture(scope="module")
def gpu1(cfg1):
    print("\n[gpu] config-1 forward (2000 G, 4 x 128x128)", flush=True)
    cfg = gs.raster_cfg((16, 16))
    frame = make_frame(cfg1, cfg)
    params = torch.from_numpy(cfg1.params).cuda()
    buf = gs.rasterize(params, frame, cfg)
    torch.cuda.synchronize()
    return cfg, frame, params, buf


@pytest.fixture(scope="module")
def ref1(cfg1):
    return [oracle.render(cfg1.params, c) for c in cfg1.cams]


def images(frame, buf):
    return [frame.image(buf.rgb, i).cpu().numpy().astype(np.float64) for i in range(frame.n_jobs)]


def assert_image_close(got, ref, flags, rtol=1e-4, atol=1e-6):
    ok = flags == 0
    err = np.abs(got - ref["rgb"])
    bad = (err > rtol * np.abs(ref["rgb"]) + atol) & ok[None]
    assert not bad.any(), f"{bad.sum()} pixel-channels off, max err {err[:, ok].max():.3e}"


# ---------------------------------------------------------------------------

def test_project_matches_oracle(cfg1, gpu1):
    cfg, frame, params, buf = gpu1
    rec = buf.rec.view(-1, gs.REC_WORDS).cpu().numpy().astype(np.float64)
    meta = buf.meta.view(-1, gs.META_WORDS).cpu().numpy().view(np.uint32)
    for v in range(4):
        pr = oracle.project(cfg1.params, cfg1.cams[v])
        r = rec[v * 2000:(v + 1) * 2000]
        m = meta[v * 2000:(v + 1) * 2000]
        vis = m[:, 1] > 0
        assert vis.sum() > 500
        assert pr["valid"][vis].all()
        np.testing.assert_allclose(r[vis, 0:2], pr["mean2d"][vis], rtol=0, atol=2e-4)
        conic = np.stack([r[:, 2] / (-0.5 * LOG2E), r[:, 3] / -LOG2E, r[:, 4] / (-0.5 * LOG2E)], axis=1)
        scale = np.abs(pr["conic"][vis]).max(axis=1, keepdims=True)
        np.testing.assert_allclose(conic[vis] / scale, pr["conic"][vis] / scale, atol=2e-5)
        np.testing.assert_allclose(2.0 ** r[vis, 5], pr["opacity"][vis], rtol=2e-6)
        np.testing.assert_allclose(r[vis, 6:9], pr["rgb"][vis], atol=2e-6)
        np.testing.assert_allclose(m[vis, 0].view(np.float32), pr["depth"][vis], rtol=1e-6)
        # moment frame: the conic's largest-eigenvalue axis (cos, sin), cos >= 0
        t = r[vis, 9]
        cs, sn = (1 - t * t) / (1 + t * t), 2 * t / (1 + t * t)
        a, b, c = (pr["conic"][vis, k] for k in range(3))
        d11 = a * cs * cs + 2 * b * cs * sn + c * sn * sn
        d22 = a * sn * sn - 2 * b * cs * sn + c * cs * cs
        d12 = (c - a) * cs * sn + b * (cs * cs - sn * sn)
        spread = np.sqrt((a - c) ** 2 + 4 * b * b)
        assert (np.abs(t) <= 1.0 + 1e-6).all()
        assert (np.abs(d12) <= 1e-3 * spread + 1e-6 * (a + c)).all()
        assert (d11 - d22 >= -1e-3 * spread - 1e-6 * (a + c)).all()


def _bins_check(frame, buf):
    meta = buf.meta.view(-1, gs.META_WORDS).cpu().numpy().view(np.uint32)
    c = gs.read_counters(buf)
    rects = np.stack([meta[:, 2] & 0xFFFF, meta[:, 2] >> 16, meta[:, 3] & 0xFFFF, meta[:, 3] >> 16], axis=1)
    rects = rects.astype(np.int64)
    rects[meta[:, 1] == 0] = [1, 1, 0, 0]
    job_of = np.zeros(frame.n_records, np.int64)
    for j in range(frame.n_jobs):
        job_of[frame.job(j).rec0: frame.job(j).rec0 + frame.job(j).g1 - frame.job(j).g0] = j
    tb = [frame.job(j).tile0 for j in range(frame.n_jobs)]
    tx = [frame.job(j).tiles_x for j in range(frame.n_jobs)]
    vals, ranges = oracle.bin_reference(rects, meta[:, 0], tb, tx, job_of, frame.n_tiles)
    assert c["status"] == 0
    assert c["pairs"] == len(vals)
    assert c["visible"] == int((meta[:, 1] > 0).sum())
    got = buf.vals[:len(vals)].cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got, vals)
    np.testing.assert_array_equal(buf.ranges.view(-1, 2).cpu().numpy().view(np.uint32), ranges)


def test_bins_bit_exact(gpu1):
    cfg, frame, params, buf = gpu1
    _bins_check(frame, buf)


def plan_check(frame, cfg, buf):
    """The compositing plan: a permutation of the tiles grouped by their
    wavefront count (4 above 4x the mean list length, 2 above 1.25x, never
    more than the tile's quadrants), the counts in front; inside a group the
    lists by bucket of half the mean length, longest first (last bucket
    open-ended).  Which of several tiles of one bucket comes first is free."""
    nt = frame.n_tiles
    order = buf.tile_order.cpu().numpy().view(np.uint32)
    rg = buf.ranges.view(-1, 2).cpu().numpy().view(np.uint32).astype(np.int64)
    n = rg[:nt, 1] - rg[:nt, 0]
    pairs = int(gs.read_counters(buf)["pairs"])
    quads = (cfg.tile_w // 8) * (cfg.tile_h // 8)
    a = 4 * n * nt
    waves = np.minimum(np.where(a > 16 * pairs, 4, np.where(a > 5 * pairs, 2, 1)), quads)
    n4, n2, n1 = (int(v) for v in order[:3])
    assert (n4, n2, n1) == tuple(int((waves == w).sum()) for w in (4, 2, 1))
    lst = order[4:4 + nt].astype(np.int64)
    assert np.array_equal(np.sort(lst), np.arange(nt))
    bucket = np.minimum(2 * n * nt // max(pairs, 1), 15)
    for lo, hi, w in ((0, n4, 4), (n4, n4 + n2, 2), (n4 + n2, nt, 1)):
        part = lst[lo:hi]
        assert (waves[part] == w).all()
        assert (np.diff(bucket[part]) <= 0).all()


@pytest.mark.parametrize("tile", [(16, 16), (32, 8), (16, 8)])
def test_compositing_plan(cfg1, tile):
    cfg = gs.raster_cfg((*tile, -1, -1))
    frame = make_frame(cfg1, cfg)
    buf = gs.rasterize(torch.from_numpy(cfg1.params).cuda(), frame, cfg)
    plan_check(frame, cfg, buf)
    assert int(buf.tile_order[0]) + int(buf.tile_order[1]) > 0      # some tiles split


@pytest.mark.parametrize("n", [300, 1500, 3000, 6000, 9000])
def test_bins_bit_exact_long_tile_lists(n):
    """Large Gaussians in front of a small view put n entries in every tile
    (above 256: the in-LDS merge sort, 4 keys per thread up to 1024 and 16
    beyond, the capacity making the frame dense; above 4096: the long-list
    kernel; above 8192: its chunks and merges), with many equal depths (ties
    ordered by record), against the reference."""
    p = scenes.gaussians(n, 0, 4100 + n, [-0.3, -0.3, -0.3], [0.3, 0.3, 0.3], 0.0, 0.1)
    p[scenes.MEAN + 2, ::3] = 0.25                  # every third Gaussian at the same depth
    params = torch.from_numpy(p).cuda()
    cam = scenes.look_at([0.0, 0.0, 3.0], [0, 0, 0], 64, 48, 60.0, 60.0)
    for tile in [(16, 16), (8, 8)]:
        cfg = gs.raster_cfg(tile)
        frame = gs.Frame([cam], [gs.JobSpec(0, 0, n, 1.0)], cfg)
        buf = gs.rasterize(params, frame, cfg, capacity=n * frame.n_tiles + 1024)
        lens = np.diff(buf.ranges.view(-1, 2).cpu().numpy().view(np.uint32), axis=1)
        assert lens.max() > min(n - 10, 256)
        _bins_check(frame, buf)


@pytest.mark.parametrize("n", [1500, 3000])
def test_bins_bit_exact_long_lists_in_sparse_frame(n):
    """A cluster of n small Gaussians in a 1600x1066 view: a few tiles hold
    about n entries while the mean list stays short, so the tile sort keeps
    its small form (8 keys per thread, lists up to 2048 on chip) and sends
    the longer lists to the long-list kernel; bins against the reference."""
    p = scenes.gaussians(n, 0, 4400 + n, [-0.01, -0.01, -0.3], [0.01, 0.01, 0.3], -5.0, 0.3)
    p[scenes.MEAN + 2, ::4] = 0.1                   # every fourth Gaussian at the same depth
    params = torch.from_numpy(p).cuda()
    cam = scenes.look_at([0.0, 0.0, 3.0], [0, 0, 0], 1600, 1066, 1200.0, 1200.0)
    cfg = gs.raster_cfg((16, 16))
    frame = gs.Frame([cam], [gs.JobSpec(0, 0, n, 1.0)], cfg)
    buf = gs.rasterize(params, frame, cfg, capacity=64 * n + 1024)
    assert buf.capacity <= frame.n_tiles * 1024        # the sparse form of the tile sort
    lens = np.diff(buf.ranges.view(-1, 2).cpu().numpy().view(np.uint32), axis=1)
    assert lens.max() > min(n - 100, 2048) and lens.mean() < 64
    _bins_check(frame, buf)


@pytest.mark.parametrize("size", [(16, 16), (17, 16), (48, 16), (200, 16)])
def test_bins_bit_exact_few_tiles(size):
    """1, 2, 3 and 13 tiles: no radix pass at all, then one pass of a 1-, 2-
    and 4-bit digit; every Gaussian in front of the camera."""
    n = 400
    p = scenes.gaussians(n, 0, 4300, [-0.4, -0.2, -0.2], [0.4, 0.2, 0.2], 0.0, 0.3)
    params = torch.from_numpy(p).cuda()
    w, h = size
    cam = scenes.look_at([0.0, 0.0, 3.0], [0, 0, 0], w, h, 40.0, 40.0)
    cfg = gs.raster_cfg((16, 16))
    frame = gs.Frame([cam], [gs.JobSpec(0, 0, n, 1.0)], cfg)
    buf = gs.rasterize(params, frame, cfg)
    assert frame.n_tiles == (w + 15) // 16 and gs.read_counters(buf)["pairs"] > 0
    _bins_check(frame, buf)


def test_bins_bit_exact_large_pair_capacity():
    """A pair capacity above 2^22 takes the tile radix sort's large form (16
    keys per thread and iteration, here over many iterations and a ragged
    last one); the bins do not change."""
    n = 1500
    p = scenes.gaussians(n, 0, 4200, [-0.3, -0.3, -0.3], [0.3, 0.3, 0.3], 0.0, 0.1)
    params = torch.from_numpy(p).cuda()
    cam = scenes.look_at([0.0, 0.0, 3.0], [0, 0, 0], 64, 48, 60.0, 60.0)
    cfg = gs.raster_cfg((8, 8))
    frame = gs.Frame([cam], [gs.JobSpec(0, 0, n, 1.0)], cfg)
    buf = gs.rasterize(params, frame, cfg, capacity=(1 << 22) + 4096)
    assert gs.read_counters(buf)["pairs"] > 4096 * 8
    _bins_check(frame, buf)


@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (32, 8)])
def test_bins_bit_exact_other_tiles(cfg1, tile):
    cfg = gs.raster_cfg(tile)
    frame = make_frame(cfg1, cfg)
    buf = gs.rasterize(torch.from_numpy(cfg1.params).cuda(), frame, cfg)
    _bins_check(frame, buf)


def test_render_fwd_matches_oracle(gpu1, ref1):
    cfg, frame, params, buf = gpu1
    nflag = 0
    for v, img in enumerate(images(frame, buf)):
        ref = ref1[v]
        nflag += int((ref["flags"] != 0).sum())
        assert_image_close(img, ref, ref["flags"])
        T = frame.plane(buf.T, v).cpu().numpy()
        ok = ref["flags"] == 0
        np.testing.assert_allclose(T[ok], ref["T"][ok], rtol=1e-4, atol=1e-6)
    assert nflag < 50


def test_tile_shape_and_batch_invariance(cfg1, gpu1):
    """Forward images are bit-identical across tile shapes, wavefronts per
    tile, and whether views are rendered batched or one at a time."""
    cfg, frame, params, buf = gpu1
    base = images(frame, buf)
    for tile in [(8, 8), (16, 8), (32, 8), (16, 8, 2), (16, 16, 2), (16, 16, 4), (32, 8, 2), (32, 8, 4),
                 (16, 16, -1), (32, 8, -1), (16, 8, -1), (8, 8, -1)]:
        c2 = gs.raster_cfg(tile)
        f2 = make_frame(cfg1, c2)
        b2 = gs.rasterize(params, f2, c2)
        for a, b in zip(base, images(f2, b2)):
            np.testing.assert_array_equal(a, b)
    for v in range(4):
        f1 = make_frame(cfg1, cfg, [v])
        b1 = gs.rasterize(params, f1, cfg)
        np.testing.assert_array_equal(images(f1, b1)[0], base[v])


def test_forward_deterministic(gpu1):
    cfg, frame, params, buf = gpu1
    a = buf.rgb.clone()
    gs.rasterize(params, frame, cfg, buf)
    assert torch.equal(a, buf.rgb)


def _oracle_dldc(scene, views, ref, weight):
    """L1 gradient from the oracle image, zero at flagged pixels and where
    |C - target| is within rounding of the kink."""
    out = []
    for v in views:
        C = ref[v]["rgb"]
        d = C - scene.targets[v]
        g = weight * np.sign(d) / d.size
        g[:, ref[v]["flags"] != 0] = 0
        g[np.abs(d) < 1e-5] = 0
        out.append(g)
    return out


def test_contribution_count_matches_oracle(cfg1, gpu1, ref1):
    """gs_render_fwd_stats counts the (pixel, Gaussian) contributions of
    Eq. 2: the oracle's per-pixel contributor counts summed over the frame,
    up to one per flagged pixel; the image is the plain forward's."""
    cfg, frame, params, buf = gpu1
    rgb = buf.rgb.clone()
    kept = gs.render_fwd_stats(frame, cfg, buf)
    assert torch.equal(buf.rgb, rgb)
    n_ref = sum(int(r["n"].sum()) for r in ref1)
    flagged = sum(int(np.count_nonzero(r["flags"])) for r in ref1)
    assert n_ref > 10_000
    assert abs(kept - n_ref) <= flagged, (kept, n_ref, flagged)


def test_render_bwd_matches_oracle(cfg1, gpu1, ref1):
    cfg, frame, params, buf = gpu1
    views = list(range(4))
    dl = _oracle_dldc(cfg1, views, ref1, 0.25)
    g_ref = sum(oracle.backward(cfg1.params, cfg1.cams[v], dl[v]) for v in views)
    gin = torch.cat([torch.from_numpy(d.astype(np.float32)).reshape(-1) for d in dl]).cuda()
    grad = torch.empty_like(params)
    gs.render_bwd(params, frame, cfg, buf, grad, gs.LOSS_EXTERNAL, gin)
    g = grad.cpu().numpy().astype(np.float64)
    for name, planes in group_planes(params.shape[0]).items():
        num = np.linalg.norm(g[planes] - g_ref[planes])
        den = np.linalg.norm(g_ref[planes])
        assert den > 0, name
        assert num / den <= 1e-3, (name, num / den)
    # determinism of the backward (no float atomics on the gradient path)
    grad2 = torch.empty_like(params)
    gs.render_bwd(params, frame, cfg, buf, grad2, gs.LOSS_EXTERNAL, gin)
    assert torch.equal(grad, grad2)


@pytest.mark.parametrize("tile", [(16, 16, 2), (16, 16, 4), (32, 8, 4), (16, 8, 2), (16, 16, 2, -1), (32, 8, 1, -1),
                                  (16, 8, 2, -1), (8, 8, 1, -1)])
def test_render_bwd_sub_tile_waves_match_oracle(cfg1, ref1, tile):
    """Several wavefronts per tile (fixed, or per tile from its list length),
    each storing its own partials per pair: gradients against the FP64
    oracle as for one wavefront per tile, and deterministic."""
    cfg = gs.raster_cfg(tile)
    frame = make_frame(cfg1, cfg)
    params = torch.from_numpy(cfg1.params).cuda()
    buf = gs.rasterize(params, frame, cfg)
    views = list(range(4))
    dl = _oracle_dldc(cfg1, views, ref1, 0.25)
    g_ref = sum(oracle.backward(cfg1.params, cfg1.cams[v], dl[v]) for v in views)
    gin = torch.cat([torch.from_numpy(d.astype(np.float32)).reshape(-1) for d in dl]).cuda()
    grad = torch.empty_like(params)
    gs.render_bwd(params, frame, cfg, buf, grad, gs.LOSS_EXTERNAL, gin)
    g = grad.cpu().numpy().astype(np.float64)
    for name, planes in group_planes(params.shape[0]).items():
        num = np.linalg.norm(g[planes] - g_ref[planes])
        assert num / np.linalg.norm(g_ref[planes]) <= 1e-3, (name, tile)
    grad2 = torch.empty_like(params)
    gs.render_bwd(params, frame, cfg, buf, grad2, gs.LOSS_EXTERNAL, gin)
    assert torch.equal(grad, grad2)


@pytest.mark.parametrize("tile", [(16, 16, -1), (16, 16, 1), (16, 16, 2, 1), (16, 16, 1, 4), (16, 16, 4, 2),
                                  (32, 8, 2, 4), (32, 8, -1, 1), (16, 8, 2, 1), (8, 8, 1), (16, 16, -1, 2)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_quadrant_masks_from_forward_equal_recomputed(cfg1, tile, dtype):
    """The backward reading the forward's per-entry quadrant masks (bins.qmask)
    gives the gradients it gives when it recomputes them, bit for bit, and the
    same loss, whatever the forward's and the backward's wavefront splits."""
    if dtype == torch.float64 and tile != (16, 16, 2, 1):
        pytest.skip("FP64 on one split pair")
    cfg = gs.raster_cfg(tile)
    frame = make_frame(cfg1, cfg)
    params = torch.from_numpy(cfg1.params).to("cuda", dtype)
    buf = gs.rasterize(params, frame, cfg)
    target = frame_target(frame, cfg1, range(4)).to(dtype)
    out = []
    for share in (True, False):
        buf.share_qmask = share
        g = torch.empty_like(params)
        loss = torch.zeros(4, dtype=dtype, device="cuda")
        gs.render_bwd(params, frame, cfg, buf, g, gs.LOSS_L1, target, loss)
        out.append((g, loss))
    buf.share_qmask = True
    assert torch.equal(out[0][0], out[1][0]), tile
    # the per-job loss is added with atomics in no fixed order
    torch.testing.assert_close(out[0][1], out[1][1], rtol=1e-6, atol=0)


@pytest.mark.parametrize("tile", [(16, 16), (16, 16, -1), (32, 8, -1), (8, 8, -1)])
def test_l1_loss_mode(cfg1, tile):
    """GS_LOSS_L1 equals the external mode fed the oracle's dL/dC of the
    L1 part of Eq. 3 (w sign(C - target) / 3HW on the GPU's own image), and
    the fused loss equals the oracle's w mean |C - target| per job: with one
    wavefront per tile, and with the wavefronts from the plan (whose
    workgroups mix tiles of the four jobs and add their sums per job)."""
    from oracle.raster import l1_loss_and_grad
    cfg = gs.raster_cfg(tile)
    frame = make_frame(cfg1, cfg)
    params = torch.from_numpy(cfg1.params).cuda()
    buf = gs.rasterize(params, frame, cfg)
    target = frame_target(frame, cfg1, range(4))
    loss = torch.zeros(4, dtype=torch.float32, device="cuda")
    g1 = torch.empty_like(params)
    gs.render_bwd(params, frame, cfg, buf, g1, gs.LOSS_L1, target, loss)
    n = 3 * 128 * 128
    rgb, tg = buf.rgb.cpu().numpy(), target.cpu().numpy()
    ref = [l1_loss_and_grad(rgb[i * n:(i + 1) * n], tg[i * n:(i + 1) * n], 0.25) for i in range(4)]
    dl = torch.from_numpy(np.concatenate([r[1] for r in ref]).astype(np.float32)).cuda()
    g2 = torch.empty_like(params)
    gs.render_bwd(params, frame, cfg, buf, g2, gs.LOSS_EXTERNAL, dl)
    torch.testing.assert_close(g1, g2, rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(loss.cpu().numpy(), [r[0] for r in ref], rtol=1e-5)


def _adam_bounds(x, g, m, v, w, lr, rho, step, mask, b1, b2, eps):
    """Per-element FP32 rounding bounds of one Adam + ADMM update, from the
    magnitudes of the terms each result sums (u = 2^-24, a few ops each):
    m' = b1 m + (1-b1) g' can cancel, so its bound scales with
    b1|m| + (1-b1)|g'|, not with |m'|; the step inherits m''s error."""
    from oracle.admm import penalty_groups
    u = 2.0 ** -24
    grp = penalty_groups(x.shape[0])
    x, g, m, v = (np.asarray(a, np.float64) for a in (x, g, m, v))
    r = np.asarray(rho)[grp][:, None] * (1.0 if mask is None else mask[None, :]) if w is not None else 0.0
    gp_terms = np.abs(g) + (np.abs(r) * (np.abs(x) + np.abs(w)) if w is not None else 0.0)
    gp = g + (r * (x - w) if w is not None else 0.0)
    sm = b1 * np.abs(m) + (1 - b1) * gp_terms
    m1 = b1 * m + (1 - b1) * gp
    v1 = b2 * v + (1 - b2) * gp * gp
    bc1, bc2 = 1 - b1 ** step, 1 - b2 ** step
    den = np.sqrt(v1 / bc2) + eps
    lrp = np.asarray(lr)[grp][:, None]
    ratio = np.abs(m1 / bc1) / den
    bm = 16 * u * sm
    bv = 16 * u * (b2 * v + (1 - b2) * gp_terms ** 2)
    bx = 16 * u * np.abs(x) + lrp * (16 * u * ratio + bm / bc1 / den + ratio * bv / (2 * v1 + 1e-300))
    return bx, bm, bv


def test_adam_admm_matches_oracle():
    rng = np.random.default_rng(31)
    A, N = 59, 10_003                      # ragged tail (not a multiple of 4)
    x, g, m, w = (rng.standard_normal((A, N)).astype(np.float32) for _ in range(4))
    v = np.abs(rng.standard_normal((A, N))).astype(np.float32)
    mask = (rng.random(N) < 0.5).astype(np.float32)
    lr, rho = [1e-3, 2e-3, 3e-3, 4e-3, 5e-3], [1e-3, 1e4, 1e4, 1e3, 1e4]
    # the kernel receives its hyper-parameters as FP32; the oracle gets the same values
    f32 = lambda v: [float(np.float32(a)) for a in v]  # noqa: E731
    hp = dict(beta1=f32([0.9])[0], beta2=f32([0.999])[0], eps=f32([1e-8])[0])
    for use_w, use_mask in [(False, False), (True, False), (True, True)]:
        t = {k: torch.from_numpy(a.copy()).cuda() for k, a in dict(x=x, g=g, m=m, v=v, w=w).items()}
        tm = torch.from_numpy(mask).cuda() if use_mask else None
        gs.adam_admm(t["x"], t["g"], t["m"], t["v"], t["w"] if use_w else None, tm, gs.adam_cfg(lr, rho, 7))
        ww, mm = (w if use_w else None), (mask if use_mask else None)
        rx, rm, rv = oracle.adam_admm(x, g, m, v, ww, f32(lr), f32(rho), 7, mask=mm, **hp)
        bx, bm, bv = _adam_bounds(x, g, m, v, ww, f32(lr), f32(rho), 7, mm, hp["beta1"], hp["beta2"], hp["eps"])
        for name, got, ref, bnd in [("x", t["x"], rx, bx), ("m", t["m"], rm, bm), ("v", t["v"], rv, bv)]:
            err = np.abs(got.cpu().numpy() - ref)
            assert (err <= bnd).all(), (name, use_w, use_mask, int((err > bnd).sum()), float((err / bnd).max()))
    # unaligned stride: scalar path
    xs = torch.from_numpy(np.ascontiguousarray(x[:, :N - 1])).cuda()
    big = torch.zeros((A, N), device="cuda")
    big[:, :N - 1] = xs
    sub = big[:, :N - 1]
    gg = torch.from_numpy(np.ascontiguousarray(g[:, :N - 1])).cuda()
    mm = torch.zeros_like(gg)
    vv = torch.zeros_like(gg)
    gs.adam_admm(sub, gg, mm, vv, None, None, gs.adam_cfg(lr, rho, 1))
    z = 0 * g[:, :N - 1]
    rx, _, _ = oracle.adam_admm(x[:, :N - 1], g[:, :N - 1], z, z, None, f32(lr), f32(rho), 1, **hp)
    bx, _, _ = _adam_bounds(x[:, :N - 1], g[:, :N - 1], z, z, None, f32(lr), f32(rho), 1, None, hp["beta1"],
                            hp["beta2"], hp["eps"])
    assert (np.abs(sub.cpu().numpy() - rx) <= bx).all()


def _random_holders(rng, K, G, max_holders, unheld=0.0):
    """Holder CSR over K blocks: each global id is held by 1..max_holders
    blocks (a fraction ``unheld`` by none), locals laid out block by block in
    ascending global id with a padding column after every 97th local copy
    (a column no holder set names)."""
    held = []
    for _ in range(G):
        n = 0 if rng.random() < unheld else int(rng.integers(1, max_holders + 1))
        held.append(sorted(rng.choice(K, n, replace=False)) if n else [])
    cols, local_of, L = [], {}, 0
    for k in range(K):
        for gid in range(G):
            if k in held[gid]:
                local_of[(gid, k)] = L
                cols.append(L)
                L += 1
                if L % 97 == 0:
                    L += 1
    ptr = np.zeros(G + 1, np.int64)
    idx = []
    for gid in range(G):
        idx += [local_of[(gid, k)] for k in held[gid]]
        ptr[gid + 1] = len(idx)
    return ptr, np.asarray(idx, np.int64), L


@pytest.mark.parametrize("deg,max_holders", [(0, 2), (1, 4), (2, 6), (3, 2), (3, 5)])
def test_consensus_matches_oracle(deg, max_holders):
    """z, u, w and the per-group residual sums against the oracle for every
    SH degree (plane count), the 1-2 / 3-4 / more-holder paths, with and
    without over-relaxation and residuals; single-holder duals and columns
    of no holder set keep their values."""
    rng = np.random.default_rng(32 + deg)
    K, G = 6, 2500
    A = 11 + 3 * (deg + 1) ** 2
    ptr, idx, L = _random_holders(rng, K, G, max_holders, unheld=0.02)
    x = rng.standard_normal((A, L)).astype(np.float32)
    u = (0.1 * rng.standard_normal((A, L))).astype(np.float32)
    zp = rng.standard_normal((A, G)).astype(np.float32)
    w0 = rng.standard_normal((A, L)).astype(np.float32)
    held = np.sort(idx)
    free = np.setdiff1d(np.arange(L), held)
    unheld_g = np.nonzero(np.diff(ptr) == 0)[0]
    single = idx[ptr[:-1][np.diff(ptr) == 1]]
    assert len(free) and len(unheld_g) and len(single)
    dptr, didx = torch.from_numpy(ptr).cuda(), torch.from_numpy(idx).cuda()
    for relax in (1.0, 1.6):
        for want_resid in (True, False):
            tx, tu = torch.from_numpy(x).cuda(), torch.from_numpy(u.copy()).cuda()
            tw, tz = torch.from_numpy(w0.copy()).cuda(), torch.from_numpy(zp.copy()).cuda()
            res = torch.zeros(10, device="cuda") if want_resid else None
            gs.consensus(tx, tu, tw, tz, dptr, didx, relax, res)
            rz, ru, rw = oracle.consensus(x, u, ptr, idx, G, relax=relax, z_prev=zp)
            gz, gu, gw = (t.cpu().numpy() for t in (tz, tu, tw))
            hg = np.diff(ptr) > 0
            np.testing.assert_allclose(gz[:, hg], rz[:, hg], rtol=1e-6, atol=1e-6)
            np.testing.assert_allclose(gu[:, held], ru[:, held], rtol=1e-6, atol=1e-6)
            np.testing.assert_allclose(gw[:, held], rw[:, held], rtol=1e-6, atol=1e-6)
            # untouched: columns of no holder, z of unheld ids, u of single holders (bitwise)
            assert np.array_equal(gu[:, free], u[:, free]) and np.array_equal(gw[:, free], w0[:, free])
            assert np.array_equal(gz[:, unheld_g], zp[:, unheld_g])
            assert np.array_equal(gu[:, single], u[:, single])
            if want_resid:
                rp, rd = oracle.residual_sums(x, rz, zp, ptr, idx, G)
                got = res.cpu().numpy().astype(np.float64)
                np.testing.assert_allclose(got[:5], rp, rtol=2e-5)
                np.testing.assert_allclose(got[5:], rd, rtol=2e-5)


def test_dual_rescale_matches_oracle():
    """u *= scale per group, w = z - u over held copies after a consensus
    (groups at scale 1 and zero duals untouched bitwise)."""
    rng = np.random.default_rng(40)
    K, G, deg = 4, 3000, 3
    A = 11 + 3 * (deg + 1) ** 2
    ptr, idx, L = _random_holders(rng, K, G, 3)
    x = rng.standard_normal((A, L)).astype(np.float32)
    u = (0.1 * rng.standard_normal((A, L))).astype(np.float32)
    u[:, idx[ptr[:-1][np.diff(ptr) == 1]]] = 0                  # single holders: duals stay zero
    zp = rng.standard_normal((A, G)).astype(np.float32)
    tx, tu = torch.from_numpy(x).cuda(), torch.from_numpy(u.copy()).cuda()
    tw, tz = torch.zeros_like(tu), torch.from_numpy(zp.copy()).cuda()
    dptr, didx = torch.from_numpy(ptr).cuda(), torch.from_numpy(idx).cuda()
    gs.consensus(tx, tu, tw, tz, dptr, didx, 1.0, None)
    u1, w1, z1 = tu.cpu().numpy(), tw.cpu().numpy(), tz.cpu().numpy()
    scale = (2.0, 0.5, 1.0, 4.0, 0.25)
    gs.dual_rescale(tu, tw, tz, dptr, didx, scale)
    ru, rw = oracle.rescale_duals(u1, z1, ptr, idx, G, scale)
    held = np.sort(idx)
    gu, gw = tu.cpu().numpy(), tw.cpu().numpy()
    np.testing.assert_allclose(gu[:, held], ru[:, held], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(gw[:, held], rw[:, held], rtol=1e-6, atol=1e-6)
    s_planes = np.asarray(oracle.penalty_groups(A)) == 2          # group s has scale 1
    assert np.array_equal(gu[s_planes], u1[s_planes]) and np.array_equal(gw[s_planes], w1[s_planes])
    zero = u1 == 0
    assert zero.sum() > 0 and np.array_equal(gw[zero], w1[zero])
    with pytest.raises(gs.GsError, match="scale"):
        gs.dual_rescale(tu, tw, tz, dptr, didx, (1.0, 0.0, 1.0, 1.0, 1.0))


def test_capacity_overflow_reported_then_grown(cfg1):
    cfg = gs.raster_cfg((16, 16))
    frame = make_frame(cfg1, cfg)
    params = torch.from_numpy(cfg1.params).cuda()
    buf = gs.Buffers(frame, 100)
    gs.project(params, frame, cfg, buf)
    gs.bin_sort(frame, cfg, buf)
    c = gs.read_counters(buf)
    assert c["status"] & gs.GS_STATUS_PAIR_OVERFLOW and c["pairs"] > 100
    gs.rasterize(params, frame, cfg, buf)
    assert buf.capacity >= c["pairs"]
    _bins_check(frame, buf)


def test_ragged_image_and_empty_frame():
    """A 100x70 image (partial tiles on both edges) and a frame whose
    Gaussians are all behind the camera."""
    s = scenes.config1()
    cam = scenes.look_at([0.0, 0.4, 2.5], [0, 0, 0], 100, 70, 90.0, 90.0)
    cfg = gs.raster_cfg((16, 16))
    p = s.params[:, :500].copy()
    frame = gs.Frame([cam], [gs.JobSpec(0, 0, 500, 1.0)], cfg)
    buf = gs.rasterize(torch.from_numpy(p).cuda(), frame, cfg)
    ref = oracle.render(p, cam)
    assert_image_close(frame.image(buf.rgb, 0).cpu().numpy().astype(np.float64), ref, ref["flags"])
    behind = p.copy()
    behind[2] += 10.0                       # all Gaussians behind the camera at z = 2.5
    b2 = gs.rasterize(torch.from_numpy(behind).cuda(), frame, cfg)
    assert gs.read_counters(b2)["pairs"] == 0
    assert torch.count_nonzero(b2.rgb).item() == 0
    assert torch.all(b2.T == 1).item()
    grad = torch.empty((p.shape[0], 500), device="cuda")
    gs.render_bwd(torch.from_numpy(behind).cuda(), frame, cfg, b2, grad, gs.LOSS_L1,
                  torch.rand(3 * 100 * 70, device="cuda"))
    assert torch.count_nonzero(grad).item() == 0


def test_f64_path_against_finite_differences():
    """FP64 instantiation of the same kernels: central differences h = 1e-6 of
    L = sum W * C on the 200-Gaussian, 64x64, SH-3 adjoint scene, on every
    one of its 59 x 200 = 11,800 parameters (coordinates whose keep/stop
    decisions flip inside [-h, h] are discarded and counted)."""
    from fd_batch import finite_differences
    s = scenes.config4a()
    cam = s.cams[0]
    cfg = gs.raster_cfg((16, 16))
    frame = gs.Frame([cam], [gs.JobSpec(0, 0, 200, 1.0)], cfg)
    p64 = torch.from_numpy(s.params.astype(np.float64)).cuda()
    rng = np.random.default_rng(41)
    Wt = torch.from_numpy(rng.standard_normal(3 * 64 * 64)).cuda()
    buf = gs.rasterize(p64, frame, cfg)
    grad = torch.empty_like(p64)
    gs.render_bwd(p64, frame, cfg, buf, grad, gs.LOSS_EXTERNAL, Wt)
    g = grad.cpu().numpy()
    # against the oracle's reverse mode (both FP64)
    g_ref = oracle.backward(s.params.astype(np.float64), cam, Wt.cpu().numpy().reshape(3, 64, 64))
    np.testing.assert_allclose(g, g_ref, rtol=1e-7, atol=1e-9 * np.abs(g_ref).max())
    coords = [(a, i) for a in range(59) for i in range(200)]
    print(f"\n[gpu] finite differences on {len(coords)} coordinates", flush=True)
    fd, noise, flipped = finite_differences(p64, cam, Wt, coords, cfg)
    ga = np.array([g[a, i] for a, i in coords])
    bad = (np.abs(fd - ga) > 1e-5 * np.abs(ga) + 1e-9 * np.abs(g).max() + noise) & ~flipped
    used = int((~flipped).sum())
    print(f"[gpu] {used} coordinates compared, {int(flipped.sum())} flipped", flush=True)
    assert used >= 0.9 * len(coords)
    assert (np.abs(ga[~flipped]) > 0).sum() > 5000
    assert not bad.any(), [(coords[k], fd[k], ga[k]) for k in np.nonzero(bad)[0][:10]]


def test_disjoint_and_shared_job_paths_agree(cfg1, gpu1):
    """Four views of one block (jobs share Gaussians: per-Gaussian accumulation
    over jobs) against the same four views on four disjoint copies of the
    block (one thread per record): the copies' gradients sum to the shared
    gradient, and each copy's image equals the shared-job image bit for bit."""
    cfg, frame, params, buf = gpu1
    n = params.shape[1]
    rep = params.repeat(1, 4).contiguous()
    jobs = [gs.JobSpec(v, v * n, (v + 1) * n, 0.25) for v in range(4)]
    f4 = gs.Frame(cfg1.cams, jobs, cfg)
    assert f4.jobs_disjoint == 1 and frame.jobs_disjoint == 0
    b4 = gs.rasterize(rep, f4, cfg)
    for a, b in zip(images(frame, buf), images(f4, b4)):
        np.testing.assert_array_equal(a, b)
    target = frame_target(frame, cfg1, range(4))
    g_shared = torch.empty_like(params)
    gs.render_bwd(params, frame, cfg, buf, g_shared, gs.LOSS_L1, target)
    g_copies = torch.empty_like(rep)
    gs.render_bwd(rep, f4, cfg, b4, g_copies, gs.LOSS_L1, target)
    summed = sum(g_copies[:, v * n:(v + 1) * n].double() for v in range(4))
    torch.testing.assert_close(summed, g_shared.double(), rtol=1e-5, atol=1e-9)
    # Gaussians outside every job get zero gradients
    f2 = gs.Frame(cfg1.cams, [gs.JobSpec(0, 0, n // 2, 1.0)], cfg)
    b2 = gs.rasterize(params, f2, cfg)
    g2 = torch.full_like(params, 7.0)
    gs.render_bwd(params, f2, cfg, b2, g2, gs.LOSS_L1, target[: 3 * 128 * 128])
    assert torch.count_nonzero(g2[:, n // 2:]).item() == 0
    assert torch.count_nonzero(g2[:, : n // 2]).item() > 0
