"""Batched K-block ADMM training (Alg. 2) and the autograd wrapper, on the
GPU, against the FP64 oracle and against per-block runs."""
import numpy as np
import pytest

import oracle
from paper_2405_13943_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2405_13943_amd import admm, gs, raster  # noqa: E402

F32 = lambda v: [float(np.float32(a)) for a in v]  # noqa: E731


def tiny_blocks():
    """Three x-slab blocks, 10% of each block's Gaussians shared with its
    neighbour, two 64x48 views per block."""
    return scenes.block_scene(counts=(300, 400, 350), bounds=(-1.5, -0.5, 0.5, 1.5), n_cams=2, width=64, height=48,
                              y_range=(-0.5, 0.5), z_range=(-0.5, 0.5), logscale=(-3.5, 0.4), ring_radius=3.0,
                              ring_height=0.5, fx=60.0, sh_degree=1, seed=77)


def targets_for(bs):
    return [[torch.from_numpy(t).reshape(-1).cuda() for t in scenes.target_images(900 + 10 * k, bs.cams[k])]
            for k in range(len(bs.cams))]


def make_trainer(bs, intv=2, rho=(1e-2,) * 5, relax=1.0, fused=True, strands=0):
    model = admm.BlockModel.from_global(bs.params_global, bs.local_gid, spatial_strands=strands)
    cfg = gs.raster_cfg((16, 16))
    return admm.AdmmTrainer(model, bs.cams, targets_for(bs), cfg, lr=(1e-3, 2e-3, 3e-3, 4e-3, 5e-3), rho=rho,
                            intv=intv, relax=relax, capacity=1 << 16, fused=fused)


@pytest.mark.parametrize("strands", [0, 4])
def test_batched_blocks_equal_single_block_runs(strands):
    """All blocks in one launch per stage give bit-identical images and
    gradients to rendering each block alone (store in the drawn order inside
    the holder groups, and in Z-order chunks over strands)."""
    bs = tiny_blocks()
    tr = make_trainer(bs, fused=False, strands=strands)
    views = [1, 0, 1]
    tr.local_step(views)
    f = tr.frame(views)
    imgs = [f.image(tr.buf.rgb, k).clone() for k in range(3)]
    g_all = tr.g.clone()
    x0 = admm.BlockModel.from_global(bs.params_global, bs.local_gid, spatial_strands=strands).x
    for k in range(3):
        a, b = tr.model.block(k)
        pk = x0[:, a:b].contiguous()
        fk = gs.Frame([bs.cams[k][views[k]]], [gs.JobSpec(0, 0, b - a, 1.0)], tr.cfg)
        bk = gs.rasterize(pk, fk, tr.cfg)
        assert torch.equal(fk.image(bk.rgb, 0), imgs[k])
        gk = torch.empty_like(pk)
        gs.render_bwd(pk, fk, tr.cfg, bk, gk, gs.LOSS_L1, tr.targets[k][views[k]])
        assert torch.equal(gk, g_all[:, a:b])


@pytest.mark.parametrize("strands", [0, 4])
def test_trainer_step_matches_oracle_composition(strands):
    """One trainer step (t = 0: local step for all blocks, then consensus)
    equals the oracle composed from the paper's pieces: per-block image
    gradient (FP64 render/backward), Adam on g + rho (x - w) with w = z - u
    and u = 0, then z = mean over holders, u = x - z, w = z - u.  Also with
    the store in Z-order chunks inside the holder groups."""
    bs = tiny_blocks()
    tr = make_trainer(bs, intv=1, strands=strands)
    x0 = tr.model.x.cpu().numpy().copy()
    tr.local_step()
    # the trainer's step (backward and optimiser fused) used the L1 gradient of
    # x0, recomputed here from the same records and bins
    f = tr.frame(tr.views_at(0))
    tgt = tr.target_buffer(tr.views_at(0))
    g_l1 = torch.empty_like(tr.model.x)
    gs.render_bwd(torch.from_numpy(x0).cuda(), f, tr.cfg, tr.buf, g_l1, gs.LOSS_L1, tgt)
    g_gpu = g_l1.cpu().numpy().astype(np.float64)
    # the L1 gradient is the kernels' external-gradient backward fed
    # dL/dC = sign(C - target) / 3HW of each block's own image (the kernels
    # themselves are checked against the FP64 oracle in test_gpu_parity)
    n_px = torch.tensor([3 * c.width * c.height for c in f.cams], device="cuda")
    dl = torch.cat([torch.sign(f.image(tr.buf.rgb, k) - f.image(tgt, k)).reshape(-1) / float(n_px[k])
                    for k in range(3)])
    x0_dev = torch.from_numpy(x0).cuda()
    g_ext = torch.empty_like(x0_dev)
    gs.render_bwd(x0_dev, f, tr.cfg, tr.buf, g_ext, gs.LOSS_EXTERNAL, dl)
    np.testing.assert_allclose(g_gpu, g_ext.cpu().numpy(), rtol=1e-6, atol=1e-12)
    # and that gradient matches the FP64 oracle where the oracle flags nothing
    for k in range(3):
        a, b = tr.model.block(k)
        cam = bs.cams[k][0]
        ref = oracle.render(x0[:, a:b], cam)
        dlk = f.image(dl, k).cpu().numpy().astype(np.float64)
        dlk[:, ref["flags"] != 0] = 0
        gk = torch.empty_like(x0_dev[:, a:b].contiguous())
        fk = gs.Frame([cam], [gs.JobSpec(0, 0, b - a, 1.0)], tr.cfg)
        bk = gs.rasterize(x0_dev[:, a:b].contiguous(), fk, tr.cfg)
        gs.render_bwd(x0_dev[:, a:b].contiguous(), fk, tr.cfg, bk, gk, gs.LOSS_EXTERNAL,
                      torch.from_numpy(dlk.astype(np.float32)).reshape(-1).cuda())
        g_ref = oracle.backward(x0[:, a:b], cam, dlk)
        num = np.linalg.norm(gk.cpu().numpy() - g_ref)
        assert num / np.linalg.norm(g_ref) < 1e-3, k
    # optimiser + consensus with the GPU's own gradient as input
    lr, rho = F32(tr.lr), F32(tr.rho)
    hp = dict(beta1=F32([0.9])[0], beta2=F32([0.999])[0], eps=F32([1e-8])[0])
    z = np.zeros_like(x0)
    rx, _, _ = oracle.adam_admm(x0, g_gpu.astype(np.float32), z, z, x0, lr, rho, 1, **hp)
    x1 = tr.model.x.cpu().numpy()
    np.testing.assert_allclose(x1, rx, rtol=0, atol=2e-6 * np.abs(x0).max() + 1e-7)
    tr.consensus()
    ptr, idx = tr.model.holder_ptr.cpu().numpy(), tr.model.holder_idx.cpu().numpy()
    rz, ru, rw = oracle.consensus(x1, np.zeros_like(x1), ptr, idx, len(ptr) - 1)
    np.testing.assert_allclose(tr.model.z.cpu().numpy(), rz, rtol=1e-6, atol=1e-7)
    # u = x - z and w = z - u cancel: FP32 bound from the magnitudes of the
    # terms, over the held columns (alignment padding between blocks belongs
    # to no holder set and is left alone by the consensus kernel)
    held = np.sort(idx)
    ulp = 2.0 ** -24
    mag = (np.abs(x1) + np.abs(rw + ru))[:, held]          # |x| + |z| for every local copy
    assert (np.abs(tr.u.cpu().numpy()[:, held] - ru[:, held]) <= 16 * ulp * mag).all()
    assert (np.abs(tr.w.cpu().numpy()[:, held] - rw[:, held]) <= 32 * ulp * mag).all()
    pad = np.setdiff1d(np.arange(x1.shape[1]), held)
    assert len(pad) > 0
    assert (tr.u.cpu().numpy()[:, pad] == 0).all()


def test_fused_and_unfused_trainers_agree():
    """Several steps with consensus: the fused trainer (gs_render_bwd_adam)
    and the two-call trainer end with bit-identical state."""
    bs = tiny_blocks()
    trs = [make_trainer(bs, intv=2, fused=f) for f in (True, False)]
    for tr in trs:
        for _ in range(5):
            tr.step()
    a, b = trs
    for name in ("m", "v", "u", "w"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name
    assert torch.equal(a.model.x, b.model.x) and torch.equal(a.model.z, b.model.z)


def test_trainer_loop_invariants_and_penalty():
    """Over several consensus rounds: after every consensus the holder mean of
    the duals is zero and w = z - u (supplementary B); shared copies stay
    closer together with a strong penalty than without one."""
    bs = tiny_blocks()
    spread = {}
    for rho in (0.0, 1.0):
        tr = make_trainer(bs, intv=3, rho=(rho,) * 5)
        for _ in range(9):
            tr.step()
        tr.consensus()
        ptr, idx = tr.model.holder_ptr.cpu().numpy(), tr.model.holder_idx.cpu().numpy()
        u, w, z, x = (a.cpu().numpy().astype(np.float64) for a in (tr.u, tr.w, tr.model.z, tr.model.x))
        shared = np.nonzero(np.diff(ptr) > 1)[0]
        assert len(shared) > 50
        for gid in shared[:200]:
            hs = idx[ptr[gid]:ptr[gid + 1]]
            np.testing.assert_allclose(u[:, hs].mean(axis=1), 0, atol=1e-6)
            np.testing.assert_allclose(w[:, hs], z[:, gid:gid + 1] - u[:, hs], atol=1e-6)
        spread[rho] = np.mean([np.abs(x[:, idx[ptr[g]:ptr[g + 1]]] - z[:, g:g + 1]).max() for g in shared])
        assert tr.check() == 0
    assert spread[1.0] < spread[0.0]


def test_adaptive_penalty_rounds_match_oracle():
    """Consensus rounds with the residual-balancing penalty and
    over-relaxation: each round's residual sums, rho decision and rescaled
    duals against the oracle fed the GPU's own x and previous z, u; no
    adjustment once the freeze iteration is passed (Sec. 3.3)."""
    bs = tiny_blocks()
    model = admm.BlockModel.from_global(bs.params_global, bs.local_gid)
    cfg = gs.raster_cfg((16, 16))
    ap = admm.AdaptivePenalty(mu=10.0, tau_inc=2.0, tau_dec=2.0, until=6)
    tr = admm.AdmmTrainer(model, bs.cams, targets_for(bs), cfg, lr=(1e-3, 2e-3, 3e-3, 4e-3, 5e-3),
                          rho=(1e-4, 1e-2, 1.0, 1e2, 1e-3), intv=2, relax=1.6, capacity=1 << 16, adaptive=ap)
    ptr, idx = model.holder_ptr.cpu().numpy(), model.holder_idx.cpu().numpy()
    G = len(ptr) - 1
    held = np.sort(idx)
    changed = 0
    for t in range(10):
        tr.local_step()
        if t % tr.intv:
            tr.t += 1
            continue
        x, u0, zp = (a.cpu().numpy().astype(np.float64) for a in (tr.model.x, tr.u, tr.model.z))
        rho0 = np.asarray(tr.rho, np.float64)
        n_hist = len(tr.history)
        tr.consensus()
        rz, ru, _ = oracle.consensus(x, u0, ptr, idx, G, relax=1.6, z_prev=zp)
        if t >= ap.until:
            assert len(tr.history) == n_hist and tuple(tr.rho) == tuple(np.float32(rho0))
            tr.t += 1
            continue
        _, res, rho1 = tr.history[-1]
        rp, rd = oracle.residual_sums(x, rz, zp, ptr, idx, G)
        np.testing.assert_allclose(res[:5], rp, rtol=1e-4)
        np.testing.assert_allclose(res[5:], rd, rtol=1e-4)
        want = oracle.adaptive_rho(rho0, rp, rd)
        np.testing.assert_allclose(rho1, want, rtol=1e-6)
        changed += int((np.asarray(rho1) != np.float32(rho0)).sum())
        ru2, rw2 = oracle.rescale_duals(ru, rz, ptr, idx, G, rho0 / np.asarray(rho1, np.float64))
        gu, gw = tr.u.cpu().numpy(), tr.w.cpu().numpy()
        mag = 1.0 + np.abs(x[:, held]) + np.abs(rz).max()         # FP32 cancellation scale of u and w
        assert (np.abs(gu[:, held] - ru2[:, held]) <= 1e-5 * mag).all()
        assert (np.abs(gw[:, held] - rw2[:, held]) <= 1e-5 * mag).all()
        tr.t += 1
    assert changed >= 3


def test_autograd_function_fp64_against_finite_differences():
    """GaussianRasterize in FP64 (200 Gaussians, SH 3, 64x64): backward
    through torch.autograd equals central differences h = 1e-6 of the
    forward on every one of the 11,800 parameters (coordinates whose
    keep/stop decisions flip inside [-h, h] are left out)."""
    from fd_batch import finite_differences
    s = scenes.config4a()
    cfg = gs.raster_cfg((16, 16))
    frame = gs.Frame(s.cams, [gs.JobSpec(0, 0, 200, 1.0)], cfg)
    p = torch.from_numpy(s.params.astype(np.float64)).cuda().requires_grad_(True)
    W = torch.from_numpy(np.random.default_rng(3).standard_normal(3 * 64 * 64)).cuda()
    out = raster.rasterize(p, frame, cfg)
    (W * out).sum().backward()
    g = p.grad.cpu().numpy()
    coords = [(a, i) for a in range(59) for i in range(200)]
    fd, noise, flipped = finite_differences(p.detach(), s.cams[0], W, coords, cfg)
    ga = np.array([g[a, i] for a, i in coords])
    bad = (np.abs(fd - ga) > 1e-5 * np.abs(ga) + 1e-9 * np.abs(g).max() + noise) & ~flipped
    assert (~flipped).sum() >= 0.9 * len(coords)
    assert not bad.any(), [(coords[k], fd[k], ga[k]) for k in np.nonzero(bad)[0][:10]]


@pytest.mark.parametrize("groups", [2, 3])
def test_streamed_groups_equal_one_launch_per_stage(groups):
    """Blocks in contiguous groups, each group's local steps on a stream of
    its own, consensus after both: the store, optimiser state, duals,
    targets and global model are bit-identical to one launch per stage over
    all blocks, over five steps with two consensus rounds."""
    bs = tiny_blocks()
    ref = make_trainer(bs, intv=2)
    model = admm.BlockModel.from_global(bs.params_global, bs.local_gid)
    tr = admm.StreamedAdmmTrainer(model, bs.cams, targets_for(bs), gs.raster_cfg((16, 16)), groups=groups,
                                  lr=(1e-3, 2e-3, 3e-3, 4e-3, 5e-3), rho=(1e-2,) * 5, intv=2, capacity=1 << 16)
    assert len(tr.subs) == groups
    for _ in range(5):
        ref.step()
        tr.step()
    tr.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(ref.model.x, tr.model.x)
    assert torch.equal(ref.m, tr.full.m) and torch.equal(ref.v, tr.full.v)
    assert torch.equal(ref.u, tr.full.u) and torch.equal(ref.w, tr.full.w)
    assert torch.equal(ref.model.z, tr.model.z)


def test_autotuner_picks_a_candidate_and_caches(tmp_path):
    bs = tiny_blocks()
    model = admm.BlockModel.from_global(bs.params_global, bs.local_gid)
    tg = targets_for(bs)
    trainers = {}

    def run(tile):
        if tile not in trainers:
            trainers[tile] = admm.AdmmTrainer(model, bs.cams, tg, gs.raster_cfg(tile), capacity=1 << 16)
        trainers[tile].local_step([0, 0, 0])

    path = str(tmp_path / "tune.json")
    best = admm.autotune_tile(run, "tiny-3blocks", path, reps=2)
    assert best in admm.TILES
    # libgs timed every candidate and wrote them to the cache file
    import json
    ent = json.load(open(path))["tiny-3blocks"]
    assert tuple(ent["tile"]) == best
    assert len(ent["ms"]) == len(admm.TILES) and all(v > 0 for v in ent["ms"].values())
    assert ent["ms"]["x".join(map(str, best))] == min(ent["ms"].values())
    assert admm.autotune_tile(lambda t: (_ for _ in ()).throw(AssertionError), "tiny-3blocks", path) == best


def test_trainer_on_alg1_blocks():
    """Blocks made by Alg. 1 (K = 3, overlap 1.4) from a small uneven scene:
    the batched frame renders each block as its own render, the holder CSR
    covers every Gaussian the grouping assigned, and after steps with
    consensus the duals of shared Gaussians average to zero."""
    si = scenes.split_input(n=3000, n_grid=3, width=64, height=48)
    model, boxes, groups = admm.BlockModel.from_split(si.params_global, 3)
    cams = admm.split_cameras(boxes, si.cams)
    assert all(len(c) > 0 for c in cams)
    ptr = model.holder_ptr.cpu().numpy()
    cnt = np.diff(ptr)
    assert cnt.sum() == sum(len(g) for g in groups) and (cnt >= 1).all() and (cnt > 1).sum() > 100
    targets = [[torch.from_numpy(t).reshape(-1).cuda() for t in scenes.target_images(970 + 10 * k, cams[k])]
               for k in range(3)]
    cfg = gs.raster_cfg((16, 16))
    tr = admm.AdmmTrainer(model, cams, targets, cfg, lr=(1e-3, 2e-3, 3e-3, 4e-3, 5e-3), rho=(1e-2,) * 5, intv=2,
                          capacity=1 << 18, relax=1.6, adaptive=admm.AdaptivePenalty(until=10))
    views = [0, 0, 0]
    f = tr.frame(views)
    buf = gs.Buffers(f, 1 << 18)
    gs.rasterize(model.x, f, cfg, buf)
    for k in range(3):
        a, b = model.block(k)
        fk = gs.Frame([cams[k][0]], [gs.JobSpec(0, 0, b - a, 1.0)], cfg)
        bk = gs.rasterize(model.x[:, a:b].contiguous(), fk, cfg)
        assert torch.equal(f.image(buf.rgb, k), fk.image(bk.rgb, 0))
    for _ in range(5):
        tr.step()
    assert tr.check() == 0
    idx = model.holder_idx.cpu().numpy()
    u = tr.u.cpu().numpy().astype(np.float64)
    x = model.x.cpu().numpy().astype(np.float64)
    for g in np.nonzero(cnt > 1)[0][:300]:
        hs = idx[ptr[g]:ptr[g + 1]]
        # FP32 rounding of u = x - z at the copies' magnitude (means reach ~50)
        tol = 8 * 2.0 ** -24 * (1.0 + np.abs(x[:, hs]).max(axis=1))
        assert (np.abs(u[:, hs].mean(axis=1)) <= tol).all(), g
    assert len(tr.history) >= 2
