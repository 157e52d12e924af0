"""The training step at the benchmark's size and launch configuration: 500k
Gaussians (SH 3), one 1600x1066 view of the 40 m ring, the store in Z-order
of the means in 16-Gaussian chunks over 1024 strands, 16x16 tiles with the
wavefronts per tile chosen from the list lengths in both compositing passes.

Image, final transmittance and gradients are compared with the FP64 oracle on
256x256 crops (the oracle gets the Gaussians whose conservative footprint
meets the crop, as in the 2M-Gaussian adjoint test), and the fused backward +
Adam/ADMM call is compared bit for bit with the backward followed by the
optimiser at this size.
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

GROUPS = {"u": [0, 1, 2], "q": [3, 4, 5, 6], "s": [7, 8, 9], "o": [10]}
CROPS = ((700, 400), (1150, 600))
CROP = 256
LR, RHO = 1e-3, 1e-3


@pytest.fixture(scope="module")
def step():
    print("\n[gpu] scale scene: 500k Gaussians SH3, one 1600x1066 view, adaptive waves", flush=True)
    s = scenes.config2(n=500_000, n_cams=1)
    perm = gs.spatial_order(s.params[0:3], chunk=16, strands=1024)
    params_np = np.ascontiguousarray(s.params[:, perm])
    cam = s.cams[0]
    cfg = gs.raster_cfg((16, 16, -1))
    params = torch.from_numpy(params_np).cuda()
    frame = gs.Frame([cam], [gs.JobSpec(0, 0, params.shape[1], 1.0)], cfg)
    buf = gs.rasterize(params, frame, cfg)
    assert gs.read_counters(buf)["status"] == 0
    pr = oracle.project(params_np, cam)
    return params_np, cam, cfg, params, frame, buf, pr


def crop_subset(pr, x0, y0):
    o, S, m = pr["opacity"], pr["cov2d"], pr["mean2d"]
    c = 2.0 * np.log(np.maximum(o * 255.0, 1.0))
    hx = np.sqrt(c * S[:, 0]) * 1.01 + 1.0
    hy = np.sqrt(c * S[:, 2]) * 1.01 + 1.0
    x1, y1 = x0 + CROP, y0 + CROP
    sel = pr["valid"] & (o * 255.0 >= 1.0) & (m[:, 0] + hx >= x0) & (m[:, 0] - hx <= x1) \
        & (m[:, 1] + hy >= y0) & (m[:, 1] - hy <= y1)
    return np.nonzero(sel)[0]


def test_compositing_plan_at_scale(step):
    """The plan the timed step composites with: tiles grouped by wavefront
    count and longest list first inside each group."""
    from test_gpu_parity import plan_check
    params_np, cam, cfg, params, frame, buf, pr = step
    plan_check(frame, cfg, buf)


@pytest.mark.parametrize("crop", CROPS)
def test_image_and_gradient_on_crop(step, crop):
    params_np, cam, cfg, params, frame, buf, pr = step
    x0, y0 = crop
    W_, H_ = cam.width, cam.height
    idx = crop_subset(pr, x0, y0)
    assert 1_000 < len(idx) < 100_000
    sub = np.ascontiguousarray(params_np[:, idx])
    ys, xs = np.mgrid[y0:y0 + CROP, x0:x0 + CROP]
    pix = (ys * W_ + xs).ravel()
    ref = oracle.render(sub, cam, pixels=pix)
    ok = ref["flags"] == 0
    assert ok.mean() > 0.95
    img = frame.image(buf.rgb, 0).cpu().numpy().reshape(3, -1)[:, pix].astype(np.float64)
    d = np.abs(img - ref["rgb"])[:, ok]
    assert (d <= np.maximum(1e-4 * np.abs(ref["rgb"][:, ok]), ref["rgb_err"][:, ok]) + 1e-6).all(), d.max()
    Tg = buf.T[:W_ * H_].cpu().numpy()[pix].astype(np.float64)
    assert (np.abs(Tg - ref["T"])[ok] <= np.maximum(1e-4, ref["T_err"][ok]) * ref["T"][ok] + 1e-6).all()
    Wc = np.random.default_rng(x0 * 7 + y0).standard_normal((3, pix.size))
    Wc[:, ~ok] = 0.0
    g_ref = oracle.backward(sub, cam, Wc, pixels=pix)
    gin = np.zeros((3, H_ * W_), np.float32)
    gin[:, pix] = Wc.astype(np.float32)
    grad = torch.empty_like(params)
    gs.render_bwd(params, frame, cfg, buf, grad, gs.LOSS_EXTERNAL, torch.from_numpy(gin).reshape(-1).cuda())
    g = grad.cpu().numpy()
    gi = g[:, idx].astype(np.float64)
    for name, planes in {**GROUPS, "f": list(range(11, params.shape[0]))}.items():
        num = np.linalg.norm(gi[planes] - g_ref[planes])
        den = np.linalg.norm(g_ref[planes])
        assert den > 0, name
        assert num / den <= 1e-3, (name, num / den)
    rest = np.ones(g.shape[1], bool)
    rest[idx] = False
    assert not g[:, rest].any()


def test_fused_step_equals_backward_then_optimiser(step):
    """One local step with the L1 loss against a seeded target and the ADMM
    penalty: gs_render_bwd_adam against gs_render_bwd + gs_adam_admm, bit for
    bit on x, m and v of all 500k Gaussians."""
    params_np, cam, cfg, params, frame, buf, pr = step
    target = torch.from_numpy(scenes.rng(77).random(3 * cam.width * cam.height).astype(np.float32)).cuda()
    gen = torch.Generator(device="cuda").manual_seed(5)
    m0 = 1e-3 * torch.randn(params.shape, device="cuda", generator=gen)
    v0 = 1e-6 * torch.rand(params.shape, device="cuda", generator=gen)
    w = params + 1e-2 * torch.randn(params.shape, device="cuda", generator=gen)
    acfg = gs.adam_cfg([LR] * 5, [RHO] * 5, 3)
    x1, m1, v1 = params.clone(), m0.clone(), v0.clone()
    loss1 = torch.zeros(1, device="cuda")
    g = torch.empty_like(params)
    gs.render_bwd(x1, frame, cfg, buf, g, gs.LOSS_L1, target, loss1)
    gs.adam_admm(x1, g, m1, v1, w, None, acfg)
    x2, m2, v2 = params.clone(), m0.clone(), v0.clone()
    loss2 = torch.zeros(1, device="cuda")
    gs.render_bwd_adam(x2, frame, cfg, buf, m2, v2, w, None, acfg, gs.LOSS_L1, target, loss2)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2) and torch.equal(m1, m2) and torch.equal(v1, v2)
    assert not torch.equal(x1, params)
    torch.testing.assert_close(loss1, loss2, rtol=1e-6, atol=0)
