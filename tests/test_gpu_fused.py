"""gs_render_bwd_adam (backward with the optimiser fused into the projection
backward) against gs_render_bwd followed by gs_adam_admm: bit-identical
parameters and moments, and the same loss up to summation order."""
import numpy as np
import pytest

from paper_2405_13943_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2405_13943_amd import admm, gs  # noqa: E402

LR = (1e-3, 2e-3, 3e-3, 4e-3, 5e-3)
RHO = (0.5, 0.25, 0.125, 0.0625, 1.0)


def state(x, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    m = (torch.randn(x.shape, generator=g) * 1e-3).cuda()
    v = (torch.rand(x.shape, generator=g) * 1e-4).cuda()
    w = (x.cpu() + torch.randn(x.shape, generator=g) * 1e-2).cuda()
    mask = torch.rand(x.shape[1], generator=g).cuda()
    return m, v, w, mask


def both_paths(x, frame, cfg, target, w, mask, step, mode=gs.LOSS_L1, seed=0):
    """Run the two-call path and the fused path from the same state."""
    m0, v0, w0, k0 = state(x, seed)
    w_ = w0 if w else None
    k_ = k0 if mask else None
    acfg = gs.adam_cfg(LR, RHO, step)
    out = []
    for fused in (False, True):
        xs, ms, vs = x.clone(), m0.clone(), v0.clone()
        buf = gs.rasterize(xs, frame, cfg)
        loss = torch.zeros(frame.n_jobs, device="cuda")
        if fused:
            gs.render_bwd_adam(xs, frame, cfg, buf, ms, vs, w_, k_, acfg, mode, target, loss)
        else:
            g = torch.empty_like(xs)
            gs.render_bwd(xs, frame, cfg, buf, g, mode, target, loss)
            gs.adam_admm(xs, g, ms, vs, w_, k_, acfg)
        out.append((xs, ms, vs, loss))
    return out


def assert_same(a, b):
    """x, m, v bit for bit; the loss is a sum of per-wave float atomics whose
    order varies from run to run, so it agrees to rounding."""
    for ta, tb in zip(a[:3], b[:3]):
        assert torch.equal(ta, tb)
    torch.testing.assert_close(a[3], b[3], rtol=1e-6, atol=0)


@pytest.mark.parametrize("w,mask", [(False, False), (True, False), (True, True)])
def test_single_job_with_culled_gaussians(w, mask):
    s = scenes.config1()
    p = s.params.copy()
    p[scenes.MEAN + 2, :25] = 3.5          # behind camera 0 (at z = 3, looking down -z)
    x = torch.from_numpy(p).cuda()
    cfg = gs.raster_cfg((16, 16))
    frame = gs.Frame([s.cams[0]], [gs.JobSpec(0, 0, x.shape[1], 1.0)], cfg)
    target = torch.from_numpy(s.targets[0]).reshape(-1).cuda()
    a, b = both_paths(x, frame, cfg, target, w, mask, step=3)
    assert_same(a, b)
    assert not torch.equal(a[0], x)        # the step moved the parameters


def test_job_at_unaligned_column_with_uncovered_gaussians():
    """A job over Gaussians [3, n): its workgroups are not 16-byte aligned, so
    every one takes the per-Gaussian optimiser path, and the three Gaussians
    outside the job get the zero-gradient update of the uncovered kernel."""
    s = scenes.config1()
    x = torch.from_numpy(s.params).cuda()
    n = x.shape[1]
    cfg = gs.raster_cfg((16, 16))
    frame = gs.Frame([s.cams[1]], [gs.JobSpec(0, 3, n, 1.0)], cfg)
    assert frame.jobs_disjoint
    target = torch.from_numpy(s.targets[1]).reshape(-1).cuda()
    a, b = both_paths(x, frame, cfg, target, True, True, step=5, seed=3)
    assert_same(a, b)
    assert not torch.equal(a[0][:, :3], x[:, :3])   # the penalty moved the uncovered ones too


def test_disjoint_blocks_with_padding_columns():
    bs = scenes.block_scene(counts=(300, 400, 350), bounds=(-1.5, -0.5, 0.5, 1.5), n_cams=2, width=64, height=48,
                            y_range=(-0.5, 0.5), z_range=(-0.5, 0.5), logscale=(-3.5, 0.4), ring_radius=3.0,
                            ring_height=0.5, fx=60.0, sh_degree=1, seed=77)
    model = admm.BlockModel.from_global(bs.params_global, bs.local_gid)
    assert model.x.shape[1] > sum(len(g) for g in bs.local_gid)      # padding between blocks
    cfg = gs.raster_cfg((16, 16))
    cams = [bs.cams[k][1] for k in range(3)]
    jobs = [gs.JobSpec(k, *model.block(k), 1.0) for k in range(3)]
    frame = gs.Frame(cams, jobs, cfg)
    assert frame.jobs_disjoint
    dl = torch.randn(frame.n_pixels * 3, generator=torch.Generator().manual_seed(5)).cuda() * 1e-3
    a, b = both_paths(model.x, frame, cfg, dl, True, True, step=7, mode=gs.LOSS_EXTERNAL)
    assert_same(a, b)


def test_shared_gaussians_rejected():
    s = scenes.config1()
    x = torch.from_numpy(s.params).cuda()
    cfg = gs.raster_cfg((16, 16))
    frame = gs.Frame(s.cams, [gs.JobSpec(v, 0, x.shape[1], 0.25) for v in range(4)], cfg)
    assert not frame.jobs_disjoint
    buf = gs.rasterize(x, frame, cfg)
    m, v = torch.zeros_like(x), torch.zeros_like(x)
    target = torch.cat([torch.from_numpy(t).reshape(-1) for t in s.targets]).cuda()
    with pytest.raises(gs.GsError, match="share"):
        gs.render_bwd_adam(x, frame, cfg, buf, m, v, None, None, gs.adam_cfg(LR, RHO, 1), gs.LOSS_L1, target)
    assert np.isfinite(x.cpu().numpy()).all()
