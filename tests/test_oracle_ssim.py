"""Pins of the D-SSIM oracle (the lambda * L_ssim term of Eq. 3): library
filters, a direct window sum, closed forms and invariants of the SSIM
definition, central differences and autograd of an independent form."""
import numpy as np
import pytest

from oracle import l1_loss_and_grad, ssim

nd = pytest.importorskip("scipy.ndimage")


def _img(seed, shape):
    return np.random.default_rng(seed).random(shape)


@pytest.mark.parametrize("shape", [(40, 33), (7, 5), (3, 12)])
def test_blur_is_the_truncated_gaussian_filter(shape):
    """Separable zero-padded blur = SciPy's Gaussian filter with the same
    radius (5 = truncate x sigma) and zero boundary, and a direct sum of the
    11 x 11 window at a few pixels (including corners)."""
    x = _img(1, shape)
    got = ssim.blur(x)
    ref = nd.gaussian_filter(x, ssim.SIGMA, truncate=5.0 / ssim.SIGMA, mode="constant", cval=0.0)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)
    r = np.arange(11) - 5
    w2 = np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / (2 * 1.5 ** 2))
    w2 /= w2.sum()
    H, W = shape
    for (i, j) in [(0, 0), (H - 1, W - 1), (H // 2, W // 3)]:
        acc = 0.0
        for a in range(11):
            for b in range(11):
                ii, jj = i + a - 5, j + b - 5
                if 0 <= ii < H and 0 <= jj < W:
                    acc += w2[a, b] * x[ii, jj]
        assert abs(got[i, j] - acc) < 1e-13


def test_identical_images_score_one():
    x = _img(2, (30, 25))
    np.testing.assert_allclose(ssim.ssim_map(x, x), 1.0, atol=1e-12)
    assert abs(ssim.dssim_loss(np.stack([x, x]), np.stack([x, x]))) < 1e-12


def test_constant_images_closed_form():
    """Constant images a, b: where the window fits, sigma terms vanish and
    SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.3, 0.8
    s = ssim.ssim_map(np.full((20, 24), a), np.full((20, 24), b))
    want = (2 * a * b + ssim.C1) / (a * a + b * b + ssim.C1)
    np.testing.assert_allclose(s[5:-5, 5:-5], want, rtol=1e-12)
    assert not np.allclose(s[0, 0], want)          # the zero padding reaches the corner


def test_symmetric_in_its_arguments():
    x, y = _img(3, (17, 19)), _img(4, (17, 19))
    np.testing.assert_allclose(ssim.ssim_map(x, y), ssim.ssim_map(y, x), rtol=1e-13)


@pytest.mark.parametrize("shape", [(2, 7, 6), (3, 13, 16)])
def test_gradient_central_differences(shape):
    """Every pixel of small images (windows wider than the image included)."""
    x, y = _img(5, shape), _img(6, shape)
    g = ssim.dssim_grad(x, y)
    h = 1e-6
    idx = list(np.ndindex(*shape))
    if len(idx) > 120:
        idx = [idx[i] for i in np.random.default_rng(7).choice(len(idx), 120, replace=False)]
    for t in idx:
        xp, xm = x.copy(), x.copy()
        xp[t] += h
        xm[t] -= h
        fd = (ssim.dssim_loss(xp, y) - ssim.dssim_loss(xm, y)) / (2 * h)
        assert abs(fd - g[t]) <= 1e-7 * max(1.0, abs(g).max()) + 1e-6 * abs(fd), (t, fd, g[t])


def test_gradient_matches_autograd_of_a_convolution_form():
    """torch conv2d form of the same definition (2D window, padding 5), FP64."""
    torch = pytest.importorskip("torch")
    x, y = _img(8, (3, 21, 18)), _img(9, (3, 21, 18))
    g1 = ssim.window_1d()
    w2 = torch.tensor(np.outer(g1, g1))[None, None]
    tx = torch.tensor(x, requires_grad=True)
    ty = torch.tensor(y)

    def conv(a):
        return torch.nn.functional.conv2d(a[:, None], w2, padding=5)[:, 0]
    mx, my = conv(tx), conv(ty)
    vx, vy, cxy = conv(tx * tx) - mx * mx, conv(ty * ty) - my * my, conv(tx * ty) - mx * my
    s = ((2 * mx * my + ssim.C1) * (2 * cxy + ssim.C2)) / ((mx * mx + my * my + ssim.C1) * (vx + vy + ssim.C2))
    loss = 1 - s.mean()
    loss.backward()
    assert abs(loss.item() - ssim.dssim_loss(x, y)) < 1e-12
    np.testing.assert_allclose(ssim.dssim_grad(x, y), tx.grad.numpy(), rtol=1e-9, atol=1e-15)


def test_gradient_vanishes_at_the_target():
    x = _img(10, (2, 15, 14))
    np.testing.assert_allclose(ssim.dssim_grad(x, x), 0.0, atol=1e-15)


def test_loss_without_ssim_is_the_l1_term():
    x, y = _img(11, (3, 9, 8)), _img(12, (3, 9, 8))
    l, g = ssim.loss_and_grad(x, y, 0.0, weight=0.5)
    l1, g1 = l1_loss_and_grad(x, y, 0.5)
    assert l == l1
    np.testing.assert_array_equal(g, g1)
    l2, g2 = ssim.loss_and_grad(x, y, 0.2, weight=0.5)
    assert abs(l2 - (l1 + 0.5 * 0.2 * ssim.dssim_loss(x, y))) < 1e-15
    np.testing.assert_allclose(g2, g1 + 0.1 * ssim.dssim_grad(x, y), rtol=1e-14, atol=1e-18)
