"""Continuous-batching render server for the global model: every request
completes, latencies are reported, and each image is bit-identical whether
rendered inside a mixed batch or alone."""
import numpy as np
import pytest

from paper_2405_13943_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2405_13943_amd import gs, serve  # noqa: E402

RES = ((64, 48), (96, 64), (128, 96), (160, 120))


def small_model():
    p = scenes.gaussians(20_000, 3, 4242, [-5, -1, -5], [5, 1, 5], -3.0, 0.6)
    return torch.from_numpy(p).cuda()


def requests(n, seed):
    rng = scenes.rng(seed)
    cams = []
    for _ in range(n):
        w, h = RES[int(rng.integers(0, len(RES)))]
        th = rng.random() * 2 * np.pi
        cams.append(scenes.look_at([8 * np.cos(th), 2.0, 8 * np.sin(th)], [0, 0, 0], w, h))
    return cams


def test_mixed_batches_equal_alone_and_all_complete():
    params = small_model()
    cfg = gs.raster_cfg((16, 16))
    srv = serve.RenderServer(params, cfg, hbm_budget=2e9, n_slots=3, max_batch=8, resolutions=RES)
    n = 120
    cams = requests(n, 7)
    arrivals = scenes.poisson_arrivals(200.0, 10.0, 8)[:n]
    keep = list(range(0, n, 6))
    stats, reqs = srv.run_open_loop(cams, arrivals, keep=keep)
    assert stats["requests"] == n and all(r.done is not None for r in reqs)
    assert 0 < stats["p50_ms"] <= stats["p99_ms"]
    assert srv.idle()
    batched = [r for r in reqs if r.started is not None]
    assert len(batched) == n
    # continuous batching, not a serial queue: some launch held several
    # requests and several slots were on the GPU at once
    assert stats["largest_batch"] > 1 and stats["most_in_flight"] > 1, stats
    for rid in keep:
        alone = srv.render_alone(cams[rid])
        assert torch.equal(srv.kept[rid], alone), rid


def test_small_budget_queues_instead_of_failing():
    """An HBM budget that fits one view per slot still serves every request
    (they wait in the queue), with a batch size of one."""
    params = small_model()
    cfg = gs.raster_cfg((16, 16))
    probe = serve.RenderServer(params, cfg, hbm_budget=2e9, n_slots=1, max_batch=1, resolutions=RES)
    a = probe.slots[0].arena
    one_view = a.nbytes()
    assert one_view == serve.Arena.bytes_for(a.n_gauss, a.max_jobs, a.max_pixels, a.max_tiles, a.capacity)
    del probe
    srv = serve.RenderServer(params, cfg, hbm_budget=1.2 * one_view * 2, n_slots=2, max_batch=8, resolutions=RES)
    assert srv.max_batch == 1
    cams = requests(30, 9)
    arrivals = np.linspace(0.0, 0.01, 30)           # a burst
    stats, reqs = srv.run_open_loop(cams, arrivals, keep=[0, 29])
    assert stats["requests"] == 30
    assert torch.equal(srv.kept[29], srv.render_alone(cams[29]))


def test_spatial_order_serves_the_same_images():
    """The server's Z-ordered copy of the model is a permutation of the
    model's columns, and its images match the FP64 oracle on the model in
    its own order (1e-4 relative; pixels the oracle flags, e.g. two kept
    Gaussians at nearly the same depth, whose order follows the index, are
    left out), as do those of a server on the unpermuted model."""
    import oracle
    p = scenes.gaussians(1500, 3, 4343, [-5, -1, -5], [5, 1, 5], -2.5, 0.6)
    params = torch.from_numpy(p).cuda()
    cfg = gs.raster_cfg((16, 16))
    a = serve.RenderServer(params, cfg, hbm_budget=2e9, n_slots=1, max_batch=2, resolutions=RES)
    b = serve.RenderServer(params, cfg, hbm_budget=2e9, n_slots=1, max_batch=2, resolutions=RES, spatial_order=False)
    assert a.perm is not None and b.perm is None
    assert torch.equal(torch.sort(a.perm).values, torch.arange(params.shape[1], device=a.perm.device))
    assert torch.equal(a.params, params[:, a.perm])
    for cam in requests(3, 21):
        ref = oracle.render(p, cam)
        ok = ref["flags"] == 0
        assert ok.mean() > 0.95
        for srv in (a, b):
            img = srv.render_alone(cam).numpy().astype(np.float64)
            err = np.abs(img - ref["rgb"])
            bad = (err > 1e-4 * np.abs(ref["rgb"]) + 1e-6) & ok[None]
            assert not bad.any(), f"{bad.sum()} pixel-channels off"


def test_pair_overflow_is_retried_and_completes():
    """A pair budget far below what the views need (calibration headroom
    0.05): batches overflow on the device, the server raises its
    pairs-per-pixel estimate, re-admits smaller batches (growing an arena
    for a request that alone exceeds it) and every request completes with
    the image it has alone."""
    params = small_model()
    cfg = gs.raster_cfg((16, 16))
    srv = serve.RenderServer(params, cfg, hbm_budget=2e9, n_slots=2, max_batch=4, resolutions=RES,
                             pair_headroom=0.05)
    n = 24
    cams = requests(n, 13)
    arrivals = np.linspace(0.0, 0.005, n)
    keep = list(range(n))
    stats, reqs = srv.run_open_loop(cams, arrivals, keep=keep)
    assert stats["requests"] == n and all(r.done is not None for r in reqs)
    assert stats["retries"] >= 1
    assert all(r.tries <= srv.MAX_TRIES for r in reqs)
    for rid in keep:
        assert torch.equal(srv.kept[rid], srv.render_alone(cams[rid])), rid
