"""FP64 oracle of the structural-similarity term of the training loss
(test infrastructure).

Eq. 3 adds lambda * L_ssim to the photometric term.  Read as the D-SSIM of
the 3D Gaussian splatting recipe the paper builds on: L_ssim = 1 - mean SSIM,
with SSIM as defined by Wang et al. (the paper's SSIM metric citation):

    SSIM(p) = (2 mu_x mu_y + C1)(2 sigma_xy + C2)
              / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2))

mu, sigma^2 and sigma_xy are local moments under an 11 x 11 Gaussian window
of standard deviation 1.5 normalised to sum 1, C1 = (0.01 L)^2 and
C2 = (0.03 L)^2 with dynamic range L = 1.  Readings: the window is centred on
every pixel of the image and zero outside it (a zero-padded "same"
correlation, as in the splatting recipe; Wang et al. keep only windows that
fit), every colour channel is a separate image, and the mean runs over all
pixels and channels.

The gradient is the chain rule written out: with A1 = 2 mu_x mu_y + C1,
A2 = 2 sigma_xy + C2, B1 = mu_x^2 + mu_y^2 + C1, B2 = sigma_x^2 + sigma_y^2
+ C2 and the moments taken as functions of the window sums mu_x, E[x^2],
E[xy],

    dS/dE[x^2] = -S / B2,   dS/dE[xy] = 2 A1 / (B1 B2),
    dS/dmu_x  = 2 mu_y A2 / (B1 B2) - 2 mu_x S / B1
                - 2 mu_x dS/dE[x^2] - mu_y dS/dE[xy],

and dS(p)/dx(q) = G(p - q) (dS/dmu_x + 2 x(q) dS/dE[x^2] + y(q) dS/dE[xy]),
so the image gradient is a zero-padded correlation of the three maps.
Pinned by the not-gpu tests (identity and constant-image closed forms, the
blur against SciPy's Gaussian filter and a direct window sum, the gradient
against central differences and against torch autograd of an independent
convolution form).
"""
from __future__ import annotations

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window_1d():
    """Normalised 1D Gaussian taps; the 2D window is their outer product."""
    r = np.arange(WINDOW, dtype=np.float64) - WINDOW // 2
    g = np.exp(-r * r / (2.0 * SIGMA * SIGMA))
    return g / g.sum()


def blur(img):
    """Zero-padded 'same' correlation of a 2D image with the window, one
    axis at a time (sum of shifted copies; the window is symmetric)."""
    g = window_1d()
    h = WINDOW // 2
    a = np.asarray(img, np.float64)
    H, W = a.shape
    rows = np.zeros_like(a)
    for k in range(WINDOW):
        d = k - h                      # out[:, c] += g[k] * a[:, c + d]
        lo, hi = max(0, -d), min(W, W - d)
        if lo < hi:
            rows[:, lo:hi] += g[k] * a[:, lo + d:hi + d]
    out = np.zeros_like(a)
    for k in range(WINDOW):
        d = k - h
        lo, hi = max(0, -d), min(H, H - d)
        if lo < hi:
            out[lo:hi, :] += g[k] * rows[lo + d:hi + d, :]
    return out


def ssim_map(x, y):
    """Per-pixel SSIM of two 2D images (one channel)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def dssim_loss(img, target):
    """L_ssim = 1 - mean SSIM over the channels and pixels of [C][H][W] images."""
    img = np.asarray(img, np.float64)
    target = np.asarray(target, np.float64)
    return 1.0 - np.mean([ssim_map(img[c], target[c]).mean() for c in range(img.shape[0])])


def dssim_grad(img, target):
    """d L_ssim / d img for [C][H][W] images (the chain rule above)."""
    img = np.asarray(img, np.float64)
    target = np.asarray(target, np.float64)
    n = img.size
    out = np.zeros_like(img)
    for c in range(img.shape[0]):
        x, y = img[c], target[c]
        mx, my = blur(x), blur(y)
        sxx = blur(x * x) - mx * mx
        syy = blur(y * y) - my * my
        sxy = blur(x * y) - mx * my
        a1, a2 = 2 * mx * my + C1, 2 * sxy + C2
        b1, b2 = mx * mx + my * my + C1, sxx + syy + C2
        s = a1 * a2 / (b1 * b2)
        d_xx = -s / b2
        d_xy = 2 * a1 / (b1 * b2)
        d_mu = 2 * my * a2 / (b1 * b2) - 2 * mx * s / b1 - 2 * mx * d_xx - my * d_xy
        # L = 1 - sum(S) / n  ->  dL/dS = -1/n
        out[c] = -(blur(d_mu) + 2 * x * blur(d_xx) + y * blur(d_xy)) / n
    return out


def loss_and_grad(img, target, lam, weight=1.0):
    """Eq. 3 for one view: weight * (mean |C - target| + lam * L_ssim) and its
    gradient (sign(0) = 0 for the L1 part)."""
    img = np.asarray(img, np.float64)
    target = np.asarray(target, np.float64)
    d = img - target
    n = img.size
    l1 = np.abs(d).sum() / n
    loss = weight * (l1 + lam * dssim_loss(img, target))
    grad = weight * (np.sign(d) / n + lam * dssim_grad(img, target))
    return loss, grad
