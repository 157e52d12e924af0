"""gs_bin_sort_noalloc (binning with the library's static workspace) against
gs_bin_sort (caller workspace) through the C ABI: the same bins, bit for bit,
on two calls in a row, the second with a smaller frame.

Bins are integer work: the sorted record ids, the tile ranges, the first
pair of each visible record and the counters must be identical.  The
compositing plan's tile groups must hold the same tiles (the order inside a
group is not fixed)."""
import numpy as np
import pytest

from paper_2405_13943_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2405_13943_amd import gs  # noqa: E402


def _snapshot(frame, buf):
    torch.cuda.synchronize()
    c = gs.read_counters(buf)
    meta = buf.meta.view(-1, gs.META_WORDS).cpu().numpy().view(np.uint32)
    vis = (meta[:, 1] & 0xFFFFFF) > 0
    order = buf.tile_order.cpu().numpy().view(np.uint32)
    n4, n2 = int(order[0]), int(order[1])
    groups = (order[4:4 + n4], order[4 + n4:4 + n4 + n2], order[4 + n4 + n2:4 + frame.n_tiles])
    return {
        "counters": c,
        "vals": buf.vals[:c["pairs"]].cpu().numpy().copy(),
        "ranges": buf.ranges.cpu().numpy().copy(),
        "pair_off": buf.pair_off.cpu().numpy()[:frame.n_records][vis].copy(),
        "group_sizes": order[:3].copy(),
        "groups": [np.sort(g) for g in groups],
    }


def _compare(frame, cfg, buf):
    """Bins of gs_bin_sort, then of gs_bin_sort_noalloc, from the same records."""
    buf.counters.zero_()
    gs.bin_sort(frame, cfg, buf)
    ref = _snapshot(frame, buf)
    assert ref["counters"]["status"] == 0 and ref["counters"]["pairs"] > 0
    # spoil the outputs so that nothing is left over from the first call
    buf.vals.fill_(-1)
    buf.ranges.fill_(-1)
    buf.pair_off.fill_(-1)
    buf.tile_order.fill_(-1)
    buf.counters.zero_()
    gs.bin_sort_noalloc(frame, cfg, buf)
    got = _snapshot(frame, buf)
    assert got["counters"] == ref["counters"]
    np.testing.assert_array_equal(got["vals"], ref["vals"])
    np.testing.assert_array_equal(got["ranges"], ref["ranges"])
    np.testing.assert_array_equal(got["pair_off"], ref["pair_off"])
    np.testing.assert_array_equal(got["group_sizes"], ref["group_sizes"])
    for a, b in zip(got["groups"], ref["groups"]):
        np.testing.assert_array_equal(a, b)
    return ref["counters"]["pairs"]


def test_noalloc_bins_equal_workspace_bins_two_calls():
    max_bytes = gs.lib.gs_bin_sort_noalloc_max_bytes()
    assert max_bytes == 64 << 20
    # call 1: two 1600x1066 views of a 200k-Gaussian SH3 scene, 16x16 tiles, adaptive plan
    print("\n[gpu] noalloc call 1: 200k Gaussians SH3, 2 x 1600x1066, 16x16", flush=True)
    sc = scenes.config2(n=200_000, n_cams=8, width=1600, height=1066)
    params = torch.from_numpy(sc.params).cuda()
    cfg = gs.raster_cfg((16, 16), fwd_waves=-1, bwd_waves=-1)
    n = params.shape[1]
    frame = gs.Frame(sc.cams, [gs.JobSpec(0, 0, n, 0.5), gs.JobSpec(3, 0, n, 0.5)], cfg)
    buf = gs.Buffers(frame, 1 << 20)
    need = gs.lib.gs_bin_sort_workspace_size(frame.n_records, buf.capacity, frame.n_tiles)
    assert need <= max_bytes
    gs.project(params, frame, cfg, buf)
    p1 = _compare(frame, cfg, buf)
    # call 2: a smaller frame (20k Gaussians, one 640x480 view, 8x8 tiles)
    print("[gpu] noalloc call 2: 20k Gaussians SH3, 640x480, 8x8", flush=True)
    sc2 = scenes.config2(n=20_000, n_cams=4, width=640, height=480)
    params2 = torch.from_numpy(sc2.params).cuda()
    cfg2 = gs.raster_cfg((8, 8), fwd_waves=-1, bwd_waves=-1)
    frame2 = gs.Frame(sc2.cams, [gs.JobSpec(1, 0, params2.shape[1], 1.0)], cfg2)
    buf2 = gs.Buffers(frame2, 1 << 16)
    gs.project(params2, frame2, cfg2, buf2)
    p2 = _compare(frame2, cfg2, buf2)
    assert p2 < p1

