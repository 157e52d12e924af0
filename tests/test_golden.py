"""The FP64 oracle against hand-worked examples stored under tests/golden/.

Each fixture holds its inputs, the values worked out by hand from the
equation it cites, and that derivation; none of the expected values comes
from code.  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2405_13943_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
Y00 = 0.5 / math.sqrt(math.pi)


def fixtures(kind):
    out = []
    for name in sorted(os.listdir(GOLDEN)):
        if name.endswith(".json"):
            with open(os.path.join(GOLDEN, name)) as fh:
                d = json.load(fh)
            if d["kind"] == kind:
                out.append(pytest.param(d, id=name[:-5]))
    return out


def test_every_fixture_cites_and_derives():
    names = [n for n in os.listdir(GOLDEN) if n.endswith(".json")]
    assert names
    for n in names:
        with open(os.path.join(GOLDEN, n)) as fh:
            d = json.load(fh)
        assert d["cite"] and d["derivation"] and d["expected"], n


def centred_gaussian(cam, px, depth_offset, opacity, colour, distance):
    """One SH-0 Gaussian whose mean projects exactly onto the centre of
    pixel px (so its alpha there is its opacity)."""
    f, d = cam.fx, distance - depth_offset
    p = np.zeros((scenes.n_attr(0), 1))
    p[0, 0] = (px[0] + 0.5 - cam.cx) * d / f
    p[1, 0] = -(px[1] + 0.5 - cam.cy) * d / f
    p[2, 0] = depth_offset
    p[3:7, 0] = [1, 0, 0, 0]
    p[7:10, 0] = math.log(0.02)
    p[10, 0] = math.log(opacity / (1 - opacity))
    p[11:14, 0] = (np.asarray(colour) - 0.5) / Y00
    return p


@pytest.mark.parametrize("fx", fixtures("compositing"))
def test_compositing_fixture(fx):
    c = fx["camera"]
    cam = scenes.look_at([0.0, 0.0, c["distance"]], [0, 0, 0], c["width"], c["height"], c["f"], c["f"])
    px = fx["pixel"]
    layers = [centred_gaussian(cam, px, L["depth_offset"], L["opacity"], L["colour"], c["distance"])
              for L in fx["layers"]]
    pix = [px[1] * c["width"] + px[0]]
    e = fx["expected"]
    for params in (np.concatenate(layers, axis=1), np.concatenate(layers[::-1], axis=1)):
        r = oracle.render(params, cam, pixels=pix)
        np.testing.assert_allclose(r["rgb"][:, 0], e["rgb"], rtol=fx["rtol"])
        np.testing.assert_allclose(r["T"][0], e["T"], rtol=fx["rtol"])
        assert r["n"][0] == e["n_contrib"]


@pytest.mark.parametrize("fx", fixtures("consensus"))
def test_consensus_fixture(fx):
    A = scenes.n_attr(fx["sh_degree"])
    x = np.concatenate([v * np.ones((A, 1)) for v in fx["copies"]], axis=1)
    k = len(fx["copies"])
    ptr, idx = np.array([0, k]), np.arange(k)
    z_prev = fx["z_prev"] * np.ones((A, 1))
    z, u, _ = oracle.consensus(x, np.zeros_like(x), ptr, idx, 1, z_prev=z_prev)
    e = fx["expected"]
    np.testing.assert_array_equal(z, e["z"])
    np.testing.assert_array_equal(u, np.ones((A, 1)) * np.asarray(e["u"])[None, :])
    rp, rd = oracle.residual_sums(x, z, z_prev, ptr, idx, 1)
    np.testing.assert_array_equal(rp, e["primal"])
    np.testing.assert_array_equal(rd, e["dual"])


@pytest.mark.parametrize("fx", fixtures("adam"))
def test_adam_fixture(fx):
    A = scenes.n_attr(fx["sh_degree"])
    one = np.ones((A, 1))
    z = np.zeros((A, 1))
    x1, m1, v1 = oracle.adam_admm(fx["x"] * one, fx["g"] * one, z, z, fx["w"] * one, [fx["lr"]] * 5,
                                  [fx["rho"]] * 5, fx["step"], beta1=fx["beta1"], beta2=fx["beta2"], eps=fx["eps"])
    e = fx["expected"]
    np.testing.assert_allclose(x1, e["x"], rtol=fx["rtol"])
    np.testing.assert_allclose(m1, e["m"], rtol=fx["rtol"])
    np.testing.assert_allclose(v1, e["v"], rtol=fx["rtol"])


@pytest.mark.parametrize("fx", fixtures("l1"))
def test_l1_fixture(fx):
    from oracle.raster import l1_loss_and_grad
    C, t = np.asarray(fx["C"]), np.asarray(fx["target"])
    e = fx["expected"]
    for w in fx["weights"]:
        L, g = l1_loss_and_grad(C, t, w)
        assert abs(L - w * e["sum_abs"] / e["n"]) < 1e-15
        np.testing.assert_array_equal(g, w * np.asarray(e["sign"], dtype=np.float64) / e["n"])
