"""The edge-case scene (scenes.edge_cases) makes every clamp and cull rule of
the rasterizer act, away from its threshold, according to the FP64 oracle;
the GPU parity test on it (test_gpu_edge_cases) relies on this."""
import numpy as np

import oracle
from paper_2405_13943_amd import scenes

BG = (0.2, 0.5, 0.9)


def test_edge_scene_rules_act():
    p, cam = scenes.edge_cases()
    cfg = oracle.RasterConfig(bg=BG)
    pr = oracle.project(p, cam, cfg)
    r = oracle.render(p, cam, cfg)
    # pixels near a decision threshold: a handful at most
    assert np.count_nonzero(r["flags"]) <= 4
    # colour clamp: 60 all channels, 61 red only, both well below zero
    assert pr["valid"][60] and (pr["rgb"][60] == 0).all()
    assert pr["rgb"][61][0] == 0 and (pr["rgb"][61][1:] > 0.05).all()
    assert pr["colour_gap"][60] > 0.1 and pr["colour_gap"][61] > 0.05
    # alpha clamp: some pixel centres of 62 and 63 have o G > 0.99
    ys, xs = np.mgrid[0:cam.height, 0:cam.width] + 0.5
    for i in (62, 63):
        d0, d1 = xs - pr["mean2d"][i][0], ys - pr["mean2d"][i][1]
        a, b, c = pr["conic"][i]
        al = pr["opacity"][i] * np.exp(-0.5 * (a * d0 * d0 + 2 * b * d0 * d1 + c * d1 * d1))
        assert (al > 0.991).sum() >= 2, i
    # Jacobian clamp beyond 1.3x the half field of view, and the Gaussian
    # still changes the image
    lim = 1.3 * (cam.width / 2) / cam.fx
    for i, ax in ((64, 0), (65, 1)):
        t = pr["tcam"][i]
        assert abs(t[ax] / t[2]) > 1.05 * lim and pr["clip_gap"][i] > 0.05
        q = p.copy()
        q[10, i] = -30.0
        assert np.abs(oracle.render(q, cam, cfg)["rgb"] - r["rgb"]).max() > 0.05, i
    # just past the near plane (kept, visible), and before it (culled)
    assert pr["valid"][66] and 0.2 < pr["tcam"][66][2] < 0.25
    q = p.copy()
    q[10, 66] = -30.0
    assert np.abs(oracle.render(q, cam, cfg)["rgb"] - r["rgb"]).max() > 0.05
    assert not pr["valid"][67] and pr["tcam"][67][2] < 0.2
    # the background shows where the transmittance stays high
    assert r["T"].max() > 0.5
    # all depths distinct
    z = pr["tcam"][:, 2]
    assert len(np.unique(z)) == len(z)
