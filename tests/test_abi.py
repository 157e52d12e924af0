"""The C-ABI library loads, exports every symbol include/gs.h declares, its
struct layouts agree with the binding, and host-side logic (planning,
argument validation) works without a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs.h")


@pytest.fixture(scope="module")
def gs():
    from paper_2405_13943_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_2405_13943_amd import gs as g
    return g


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(gs):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(gs.lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", gs._build.LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (gs_[a-z0-9_]+)", out))
    assert set(names) <= exported, set(names) - exported


def test_struct_layouts_match_header(gs, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "gs.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gs_params), sizeof(gs_camera), sizeof(gs_job),
         sizeof(gs_frame), sizeof(gs_raster_cfg), sizeof(gs_bins), sizeof(gs_adam_cfg));
  printf("%zu %zu %zu %zu %zu %zu\\n", offsetof(gs_job, g0), offsetof(gs_job, loss_weight), offsetof(gs_frame, jobs_disjoint),
         offsetof(gs_raster_cfg, bg), offsetof(gs_adam_cfg, step), offsetof(gs_raster_cfg, bwd_waves));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    sizes, offs = [list(map(int, l.split())) for l in subprocess.run([str(exe)], capture_output=True,
                                                                    text=True).stdout.splitlines()]
    S = ctypes.sizeof
    assert sizes == [S(gs.GsParams), S(gs.GsCamera), S(gs.GsJob), S(gs.GsFrame), S(gs.GsRasterCfg), S(gs.GsBins),
                     S(gs.GsAdamCfg)]
    assert offs == [gs.GsJob.g0.offset, gs.GsJob.loss_weight.offset, gs.GsFrame.jobs_disjoint.offset,
                    gs.GsRasterCfg.bg.offset, gs.GsAdamCfg.step.offset, gs.GsRasterCfg.bwd_waves.offset]


def test_frame_plan_host_only(gs):
    from paper_2405_13943_amd import scenes
    s = scenes.config1()
    cfg = gs.raster_cfg((16, 16))
    cams = (gs.GsCamera * 4)(*[gs.camera_struct(c) for c in s.cams])
    jobs = (gs.GsJob * 4)()
    for i in range(4):
        jobs[i].cam, jobs[i].g0, jobs[i].g1 = i, 0, 2000
    nr, npx, nt, gm, dj = gs.c_i64(), gs.c_i64(), gs.c_i32(), gs.c_i64(), gs.c_i32()
    rc = gs.lib.gs_frame_plan(cams, 4, jobs, 4, ctypes.byref(cfg), ctypes.byref(nr), ctypes.byref(npx),
                              ctypes.byref(nt), ctypes.byref(gm), ctypes.byref(dj))
    assert rc == 0
    assert (nr.value, npx.value, nt.value, gm.value, dj.value) == (8000, 4 * 128 * 128, 4 * 64, 2000, 0)
    assert [jobs[i].tile0 for i in range(4)] == [0, 64, 128, 192]
    assert [jobs[i].px0 for i in range(4)] == [0, 16384, 32768, 49152]
    assert [jobs[i].rec0 for i in range(4)] == [0, 2000, 4000, 6000]
    # ragged image: 100x70 with 16x16 tiles -> 7 x 5 tiles
    c2 = scenes.look_at([0, 0, 3], [0, 0, 0], 100, 70, 80.0, 80.0)
    cams2 = (gs.GsCamera * 1)(gs.camera_struct(c2))
    jobs2 = (gs.GsJob * 1)()
    jobs2[0].cam, jobs2[0].g0, jobs2[0].g1 = 0, 5, 9
    assert gs.lib.gs_frame_plan(cams2, 1, jobs2, 1, ctypes.byref(cfg), ctypes.byref(nr), ctypes.byref(npx),
                                ctypes.byref(nt), ctypes.byref(gm), ctypes.byref(dj)) == 0
    assert (jobs2[0].tiles_x, jobs2[0].tiles_y, nr.value, gm.value, dj.value) == (7, 5, 4, 9, 1)
    # disjoint blocks: [0, 3), [3, 7); overlapping: [0, 3), [2, 5)
    jobs3 = (gs.GsJob * 2)()
    for k, (a, b) in enumerate([(0, 3), (3, 7)]):
        jobs3[k].cam, jobs3[k].g0, jobs3[k].g1 = 0, a, b
    gs.lib.gs_frame_plan(cams2, 1, jobs3, 2, ctypes.byref(cfg), ctypes.byref(nr), ctypes.byref(npx),
                         ctypes.byref(nt), ctypes.byref(gm), ctypes.byref(dj))
    assert dj.value == 1 and jobs3[1].rec0 == 3 and jobs3[1].tile0 == 35
    jobs3[1].g0 = 2
    gs.lib.gs_frame_plan(cams2, 1, jobs3, 2, ctypes.byref(cfg), ctypes.byref(nr), ctypes.byref(npx),
                         ctypes.byref(nt), ctypes.byref(gm), ctypes.byref(dj))
    assert dj.value == 0


def test_invalid_arguments_rejected_without_launch(gs):
    cfg = gs.raster_cfg()
    f = gs.GsFrame()
    bad = gs.GsParams(None, -1, 0, 0, 0)
    assert gs.lib.gs_project(ctypes.byref(bad), ctypes.byref(f), ctypes.byref(cfg), None, None, None, None) == gs.GS_E_INVALID
    assert "negative" in gs.lib.gs_last_error().decode()
    deg4 = gs.GsParams(None, 0, 0, 4, 0)
    assert gs.lib.gs_project(ctypes.byref(deg4), ctypes.byref(f), ctypes.byref(cfg), None, None, None, None) == gs.GS_E_INVALID
    cfg_bad = gs.raster_cfg((12, 12))
    ok = gs.GsParams(None, 0, 0, 0, 0)
    assert gs.lib.gs_project(ctypes.byref(ok), ctypes.byref(f), ctypes.byref(cfg_bad), None, None, None, None) == gs.GS_E_INVALID
    for tile in [(8, 8, 2), (16, 8, 4), (16, 16, 3), (32, 8, 8), (16, 16, 2, 3), (8, 8, 1, 2), (16, 16, 2, -2)]:
        c = gs.raster_cfg(tile)
        assert gs.lib.gs_project(ctypes.byref(ok), ctypes.byref(f), ctypes.byref(c), None, None, None, None) == gs.GS_E_INVALID
    for tile in [(16, 16, 4), (32, 8, 2), (16, 8, 2), (16, 16, 2, 1), (32, 8, 4, 2), (16, 16, 2, -1), (8, 8, -1, -1)]:
        c = gs.raster_cfg(tile)
        assert gs.lib.gs_project(ctypes.byref(ok), ctypes.byref(f), ctypes.byref(c), None, None, None, None) == gs.GS_OK
    # jobs reaching past the parameter planes
    f2 = gs.GsFrame(1, 1, 1, 1, 10, 10, 11, 1, 0)
    p10 = gs.GsParams(1, 10, 10, 0, 0)
    assert gs.lib.gs_project(ctypes.byref(p10), ctypes.byref(f2), ctypes.byref(cfg), 1, 1, None, None) == gs.GS_E_INVALID
    # backward workspace too small
    bins = gs.GsBins(1, 1, 1, 1, 1000, 1)
    rc = gs.lib.gs_render_bwd(ctypes.byref(p10), ctypes.byref(gs.GsFrame(1, 1, 1, 1, 10, 10, 10, 1, 0)), ctypes.byref(cfg),
                              1, 1, ctypes.byref(bins), 1, 1, 0, 1, None, ctypes.byref(p10), 1, 8, None)
    assert rc == gs.GS_E_CAPACITY
    # Adam with mismatched planes, bad step
    a = gs.GsParams(1, 10, 10, 0, 0)
    b = gs.GsParams(1, 11, 11, 0, 0)
    acfg = gs.adam_cfg([1e-3] * 5, [0] * 5, 1)
    assert gs.lib.gs_adam_admm(ctypes.byref(a), ctypes.byref(b), ctypes.byref(a), ctypes.byref(a), None, None,
                               ctypes.byref(acfg), None, None) == gs.GS_E_INVALID
    acfg0 = gs.adam_cfg([1e-3] * 5, [0] * 5, 0)
    assert gs.lib.gs_adam_admm(ctypes.byref(a), ctypes.byref(a), ctypes.byref(a), ctypes.byref(a), None, None,
                               ctypes.byref(acfg0), None, None) == gs.GS_E_INVALID
    # consensus relaxation outside (0, 2)
    assert gs.lib.gs_consensus(ctypes.byref(a), ctypes.byref(a), ctypes.byref(a), ctypes.byref(a), 1, 1,
                               2.5, None, None) == gs.GS_E_INVALID

    # fused backward + Adam: shared Gaussians unsupported, bad planes, small workspace
    fr_shared = gs.GsFrame(1, 1, 2, 2, 20, 20, 10, 0, 0)
    rc = gs.lib.gs_render_bwd_adam(ctypes.byref(p10), ctypes.byref(fr_shared), ctypes.byref(cfg), 1, 1,
                                   ctypes.byref(bins), 1, 1, 0, 1, None, ctypes.byref(p10), ctypes.byref(p10), None, None,
                                   ctypes.byref(acfg), 1, 1 << 20, None)
    assert rc == gs.GS_E_UNSUPPORTED and "share" in gs.lib.gs_last_error().decode()
    fr_disj = gs.GsFrame(1, 1, 1, 1, 10, 10, 10, 1, 0)
    rc = gs.lib.gs_render_bwd_adam(ctypes.byref(p10), ctypes.byref(fr_disj), ctypes.byref(cfg), 1, 1,
                                   ctypes.byref(bins), 1, 1, 0, 1, None, ctypes.byref(b), ctypes.byref(p10), None, None,
                                   ctypes.byref(acfg), 1, 1 << 20, None)
    assert rc == gs.GS_E_INVALID
    rc = gs.lib.gs_render_bwd_adam(ctypes.byref(p10), ctypes.byref(fr_disj), ctypes.byref(cfg), 1, 1,
                                   ctypes.byref(bins), 1, 1, 0, 1, None, ctypes.byref(p10), ctypes.byref(p10), None, None,
                                   ctypes.byref(acfg), 1, 8, None)
    assert rc == gs.GS_E_CAPACITY


def test_bin_sort_noalloc_size_limit_host_only(gs):
    """Binning with the static workspace refuses a frame whose workspace
    exceeds the array (16 bytes per pair of capacity: 5 Mi pairs need more
    than 64 MiB) with GS_E_CAPACITY, on the host, before touching a device;
    bad arguments are refused as by gs_bin_sort."""
    assert gs.lib.gs_bin_sort_noalloc_max_bytes() == 64 << 20
    cfg = gs.raster_cfg()
    fr = gs.GsFrame(1, 1, 1, 1, 1000, 4096, 1000, 1, 0)
    big = gs.GsBins(1, 1, 1, 1, 5 << 20, 1)
    assert gs.lib.gs_bin_sort_workspace_size(1000, 5 << 20, 1) > 64 << 20
    rc = gs.lib.gs_bin_sort_noalloc(ctypes.byref(fr), ctypes.byref(cfg), 1, ctypes.byref(big), None)
    assert rc == gs.GS_E_CAPACITY and "static scratch" in gs.lib.gs_last_error().decode()
    assert gs.lib.gs_bin_sort_noalloc(ctypes.byref(fr), ctypes.byref(cfg), None, ctypes.byref(big), None) == gs.GS_E_INVALID
    assert gs.lib.gs_bin_sort_noalloc(ctypes.byref(fr), ctypes.byref(cfg), 1, None, None) == gs.GS_E_INVALID


def test_autotune_cache_host_only(gs, tmp_path):
    """gs_autotune answers a cached workload key from the JSON cache without
    calling the step (no device work), rejects invalid candidates and
    arguments, and gs_set_tune_cache rejects a malformed file."""
    import json
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"blocks-4": {"tile": [32, 8, -1, -1], "ms": {"32x8x-1x-1": 8.5, "16x16x-1x-1": 9.0},
                                             "when": "x"},
                                "other": {"tile": [8, 8, 1, 1], "ms": {}}}))
    gs.set_tune_cache(str(path))
    calls = []
    cands = [(16, 16, -1, -1), (32, 8, -1, -1)]
    best, ms = gs.autotune("blocks-4", cands, lambda t: calls.append(t), reps=2)
    assert best == (32, 8, -1, -1) and ms == 8.5 and not calls
    best, ms = gs.autotune("other", cands, lambda t: calls.append(t))
    assert best == (8, 8, 1, 1) and ms == -1.0 and not calls
    with pytest.raises(gs.GsError, match="not a valid launch shape"):
        gs.autotune("blocks-4", [(12, 12, 1, 1)], lambda t: calls.append(t))
    with pytest.raises(gs.GsError, match="at least one"):
        gs.autotune("blocks-4", cands, lambda t: calls.append(t), reps=0)
    bad = tmp_path / "bad.json"
    bad.write_text('{"k": {"tile": [16, 16]}}')
    with pytest.raises(gs.GsError, match="malformed"):
        gs.set_tune_cache(str(bad))
    gs.set_tune_cache(None)
    assert not calls


def test_profile_registry_host_only(gs):
    """Selecting kernels to time launches nothing; kernels never launched
    report zero."""
    gs.profile_set(["k_render_bwd", "k_project_bwd_adam"])
    assert gs.profile_get("k_render_bwd") == (0.0, 0)
    gs.profile_set("*")
    gs.profile_set(None)
    assert gs.profile_get("k_emit") == (0.0, 0)
    assert gs.lib.gs_profile_get(None, None, None) == gs.GS_E_INVALID
    # pausing keeps the selection; recording resumes on enable or on a new set
    gs.profile_set(["k_render_bwd"])
    gs.profile_enable(False)
    gs.profile_enable(True)
    assert gs.profile_get("k_render_bwd") == (0.0, 0)
    gs.profile_enable(False)
    gs.profile_set(None)


def test_workspace_sizes_grow_with_inputs(gs):
    a = gs.lib.gs_bin_sort_workspace_size(1000, 10000, 64)
    b = gs.lib.gs_bin_sort_workspace_size(2000, 20000, 64)
    assert 0 < a < b
    assert gs.lib.gs_render_bwd_workspace_size(1000, 0) == 1000 * 9 * 4 * 4   # 4 wavefronts per tile at most
    assert gs.lib.gs_render_bwd_workspace_size(1000, 1) == 1000 * 9 * 8 * 4


def test_penalty_update_host_only_matches_oracle(gs):
    """gs_penalty_update (host code, no device work) takes the oracle's
    decisions on random residual sums, including exact ties at the mu
    boundary, and rejects invalid hyper-parameters."""
    import oracle
    rng = np.random.default_rng(3)
    for trial in range(200):
        rho = np.float32(10.0 ** rng.uniform(-4, 4, 5))
        rp = np.float32(10.0 ** rng.uniform(-6, 6, 5))
        rd = np.float32(10.0 ** rng.uniform(-6, 6, 5))
        if trial % 7 == 0:
            rp[:] = 0
        mu, ti, td = (10.0, 2.0, 2.0) if trial % 2 else (5.0, 3.0, 1.5)
        new, scale = gs.penalty_update(np.concatenate([rp, rd]), rho, mu, ti, td)
        want = oracle.adaptive_rho(rho.astype(np.float64), rp.astype(np.float64), rd.astype(np.float64), mu, ti, td)
        assert np.array_equal(np.float32(new), np.float32(want)), trial
        np.testing.assert_array_equal(np.float32(scale), rho / np.float32(want))
    # ||r|| = mu ||s|| exactly: no change
    new, scale = gs.penalty_update([100.0] * 5 + [1.0] * 5, [1.0] * 5, mu=10.0)
    assert new == (1.0,) * 5 and scale == (1.0,) * 5
    for bad in (dict(mu=1.0), dict(tau_inc=0.5), dict(tau_dec=float("nan"))):
        with pytest.raises(gs.GsError, match="penalty"):
            gs.penalty_update([1.0] * 10, [1.0] * 5, **bad)
    with pytest.raises(gs.GsError, match="residual"):
        gs.penalty_update([-1.0] + [1.0] * 9, [1.0] * 5)
    with pytest.raises(gs.GsError, match="rho"):
        gs.penalty_update([1.0] * 10, [0.0] + [1.0] * 4)


def test_ssim_entry_host_checks(gs):
    """Workspace size and argument checks of gs_ssim_loss_grad, no launch."""
    assert gs.lib.gs_ssim_workspace_size(1000) == 1000 * 3 * 3 * 4
    assert gs.lib.gs_ssim_workspace_size(0) == 0
    f = gs.GsFrame()
    cfg = gs.raster_cfg()
    call = lambda lam: gs.lib.gs_ssim_loss_grad(ctypes.byref(f), ctypes.byref(cfg), None, None, lam, None, None,  # noqa: E731
                                                None, 0, None)
    assert call(-0.5) == gs.GS_E_INVALID and "lambda" in gs.lib.gs_last_error().decode()
    assert call(float("inf")) == gs.GS_E_INVALID
    assert call(0.2) == gs.GS_OK                   # empty frame: nothing to do
    f.n_pixels = 10
    assert call(0.2) == gs.GS_E_INVALID            # null images


def _morton_ref(means, bits):
    """Z-order by brute force: quantise, interleave bit by bit, sort by
    (code, index)."""
    m = np.asarray(means, np.float64)
    lo, hi = m.min(1), m.max(1)
    cells = 1 << bits
    q = np.clip(np.floor((m - lo[:, None]) / np.maximum(hi - lo, 1e-30)[:, None] * cells), 0, cells - 1)
    q = q.astype(np.int64)
    codes = []
    for i in range(m.shape[1]):
        c = 0
        for b in range(bits):
            for a in range(3):
                c |= ((int(q[a, i]) >> b) & 1) << (3 * b + a)
        codes.append((c, i))
    return [i for _, i in sorted(codes)]


def test_spatial_order(gs):
    """gs_spatial_order against a brute-force Z-order, a hand-worked 1-bit
    case (octants x + 2y + 4z, ties by index), and argument checks."""
    r = np.random.default_rng(2)
    means = (r.random((3, 700)) * [[100], [20], [100]] - [[50], [10], [50]]).astype(np.float32)
    for bits in (1, 3, 10):
        assert gs.spatial_order(means, bits).tolist() == _morton_ref(means, bits)
    pts = np.array([[1, 0, 1, 0, 1], [1, 1, 0, 0, 1], [0, 0, 0, 0, 1]], np.float32)
    # octant codes: 3, 2, 1, 0, 7
    assert gs.spatial_order(pts, 1).tolist() == [3, 2, 1, 0, 4]
    with pytest.raises(gs.GsError, match="bits"):
        gs.spatial_order(means, 0)
    bad = means.copy()
    bad[1, 5] = np.inf
    with pytest.raises(gs.GsError, match="finite"):
        gs.spatial_order(bad)


def test_spatial_order_strands(gs):
    """Chunks of the Z-order dealt over strands: strand s takes chunks s,
    s + k, ...; the tail shorter than a chunk stays last."""
    r = np.random.default_rng(4)
    means = r.random((3, 1000)).astype(np.float32)
    z = gs.spatial_order(means, 10)
    got = gs.spatial_order(means, 10, chunk=16, strands=5)
    chunks = z[:992].reshape(62, 16)
    want = np.concatenate([chunks[s::5].reshape(-1) for s in range(5)] + [z[992:]])
    assert np.array_equal(got, want)
    assert np.array_equal(np.sort(got), np.arange(1000))
    assert np.array_equal(gs.spatial_order(means, 10, chunk=16, strands=1), z)
    with pytest.raises(gs.GsError, match="strands"):
        gs.spatial_order(means, 10, chunk=16, strands=0)


def test_spatial_order_degenerate_clouds(gs):
    """Equal means (a zero-extent box on every axis) keep the index order; a
    single Gaussian and an empty store are permutations too; a flat cloud
    (zero extent on one axis) orders by the other two."""
    same = np.ones((3, 50), np.float32)
    assert gs.spatial_order(same).tolist() == list(range(50))
    assert gs.spatial_order(np.zeros((3, 1), np.float32)).tolist() == [0]
    assert gs.spatial_order(np.zeros((3, 0), np.float32)).tolist() == []
    r = np.random.default_rng(9)
    flat = r.random((3, 300)).astype(np.float32)
    flat[1] = 2.0
    assert gs.spatial_order(flat, 6).tolist() == _morton_ref(flat, 6)
