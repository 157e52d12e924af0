"""Adjoint at scale: 2M Gaussians (SH 3) in one 1920x1080 view, image and
gradients of the HIP path against the FP64 oracle on four 256x256 crops.

The loss is L = sum(W * C) with a seeded W ~ N(0, 1) on the crop's pixels and
zero elsewhere (and zero at pixels the oracle flags as within rounding of a
decision).  The oracle evaluates the crop's pixels against the Gaussians that
can reach them: every Gaussian that is culled, has opacity below alpha_min,
or whose conservative footprint (the alpha_min ellipse's bounding box grown
by 1% and 1 px, from the oracle's own FP64 projection) misses the crop has
alpha < alpha_min at every crop pixel, so dropping it changes no pixel; the
kept ones stay in ascending index order, which keeps the depth tie-break.
"""
import numpy as np
import pytest

import oracle
from paper_2405_13943_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2405_13943_amd import gs  # noqa: E402

# attribute groups of the planes: mean, rotation, log-scale, opacity, SH
GROUPS = {"u": [0, 1, 2], "q": [3, 4, 5, 6], "s": [7, 8, 9], "o": [10]}


def group_planes(A):
    return {**GROUPS, "f": list(range(11, A))}


CROPS = ((832, 412), (200, 150), (1100, 40), (1400, 300))
CROP = 256


@pytest.fixture(scope="module")
def scale():
    s = scenes.config4b()
    cam = s.cams[0]
    cfg = gs.raster_cfg((16, 16))
    params = torch.from_numpy(s.params).cuda()
    frame = gs.Frame([cam], [gs.JobSpec(0, 0, params.shape[1], 1.0)], cfg)
    buf = gs.rasterize(params, frame, cfg)
    assert gs.read_counters(buf)["status"] == 0
    pr = oracle.project(s.params, cam)
    return s, cam, cfg, params, frame, buf, pr


def crop_subset(pr, x0, y0):
    o, S, m = pr["opacity"], pr["cov2d"], pr["mean2d"]
    c = 2.0 * np.log(np.maximum(o * 255.0, 1.0))
    hx = np.sqrt(c * S[:, 0]) * 1.01 + 1.0
    hy = np.sqrt(c * S[:, 2]) * 1.01 + 1.0
    x1, y1 = x0 + CROP, y0 + CROP
    sel = pr["valid"] & (o * 255.0 >= 1.0) & (m[:, 0] + hx >= x0) & (m[:, 0] - hx <= x1) \
        & (m[:, 1] + hy >= y0) & (m[:, 1] - hy <= y1)
    return np.nonzero(sel)[0]


@pytest.mark.parametrize("crop", CROPS)
def test_image_and_gradient_on_crop(scale, crop):
    s, cam, cfg, params, frame, buf, pr = scale
    x0, y0 = crop
    W_, H_ = cam.width, cam.height
    idx = crop_subset(pr, x0, y0)
    assert 10_000 < len(idx) < 200_000
    sub = np.ascontiguousarray(s.params[:, idx])
    ys, xs = np.mgrid[y0:y0 + CROP, x0:x0 + CROP]
    pix = (ys * W_ + xs).ravel()
    ref = oracle.render(sub, cam, pixels=pix)
    ok = ref["flags"] == 0
    assert ok.mean() > 0.95
    # image on the crop, unflagged pixels: |d| <= 1e-4 |ref| + 1e-6
    img = frame.image(buf.rgb, 0).cpu().numpy().reshape(3, -1)[:, pix].astype(np.float64)
    d = np.abs(img - ref["rgb"])[:, ok]
    assert (d <= np.maximum(1e-4 * np.abs(ref["rgb"][:, ok]), ref["rgb_err"][:, ok]) + 1e-6).all(), d.max()
    Tg = buf.T[:W_ * H_].cpu().numpy()[pix].astype(np.float64)
    assert (np.abs(Tg - ref["T"])[ok] <= np.maximum(1e-4, ref["T_err"][ok]) * ref["T"][ok] + 1e-6).all()
    # gradient of sum(W * C)
    Wc = np.random.default_rng(x0 * 7 + y0).standard_normal((3, pix.size))
    Wc[:, ~ok] = 0.0
    g_ref = oracle.backward(sub, cam, Wc, pixels=pix)
    gin = np.zeros((3, H_ * W_), np.float32)
    gin[:, pix] = Wc.astype(np.float32)
    grad = torch.empty_like(params)
    gs.render_bwd(params, frame, cfg, buf, grad, gs.LOSS_EXTERNAL, torch.from_numpy(gin).reshape(-1).cuda())
    g = grad.cpu().numpy()
    gi = g[:, idx].astype(np.float64)
    for name, planes in group_planes(params.shape[0]).items():
        num = np.linalg.norm(gi[planes] - g_ref[planes])
        den = np.linalg.norm(g_ref[planes])
        assert den > 0, name
        assert num / den <= 1e-3, (name, num / den)
    # Gaussians that cannot reach the crop get exactly zero
    rest = np.ones(g.shape[1], bool)
    rest[idx] = False
    assert not g[:, rest].any()
