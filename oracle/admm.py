"""FP64 oracle for the optimiser with the ADMM penalty and for the consensus
step (test infrastructure).

Follows the scaled-form block ADMM of Eq. 8a-c and its per-attribute form in
the supplementary (detailed Eq. 8, Sec. C), the training loop of Alg. 2 and
the dual initialisation u = 0 (Sec. "More Implementation Details").

The x-update of Eq. 8a is an argmin that the paper solves inexactly by
training steps; read as textbook Adam (Kingma & Ba, with bias correction) on
the gradient of loss + (rho_a / 2) ||x - z + u||^2, i.e. the image gradient
plus rho_a (x - w) with w = z - u.
"""
from __future__ import annotations

import numpy as np

GROUPS = ("p", "q", "s", "f", "o")   # mean, rotation, scale, SH features, opacity


def penalty_groups(n_planes: int) -> np.ndarray:
    """Attribute group (index into GROUPS) of each parameter plane:
    planes 0-2 mean (p), 3-6 quaternion (q), 7-9 log-scale (s),
    10 opacity logit (o), 11.. SH coefficients (f)."""
    g = np.empty(n_planes, np.int64)
    g[0:3] = 0
    g[3:7] = 1
    g[7:10] = 2
    g[10] = 4
    g[11:] = 3
    return g


def adam_admm(x, g, m, v, w, lr, rho, step, beta1=0.9, beta2=0.999, eps=1e-8, mask=None):
    """One Adam step on x with the ADMM penalty gradient rho_a (x - w) added.

    x, g, m, v, w: [A][N] arrays (w = z - u; None means no penalty).
    lr, rho: per-group values in GROUPS order.  step: 1-based step counter.
    mask: optional [N] array of 0/1 selecting which Gaussians get the penalty.
    Returns new (x, m, v) in FP64."""
    x = np.asarray(x, np.float64)
    g = np.asarray(g, np.float64)
    m = np.asarray(m, np.float64)
    v = np.asarray(v, np.float64)
    grp = penalty_groups(x.shape[0])
    lr_p = np.asarray(lr, np.float64)[grp][:, None]
    rho_p = np.asarray(rho, np.float64)[grp][:, None]
    gp = g.copy()
    if w is not None:
        pen = rho_p * (x - np.asarray(w, np.float64))
        if mask is not None:
            pen = pen * np.asarray(mask, np.float64)[None, :]
        gp = gp + pen
    m1 = beta1 * m + (1 - beta1) * gp
    v1 = beta2 * v + (1 - beta2) * gp * gp
    mhat = m1 / (1 - beta1 ** step)
    vhat = v1 / (1 - beta2 ** step)
    x1 = x - lr_p * mhat / (np.sqrt(vhat) + eps)
    return x1, m1, v1


def consensus(x_local, u_local, holder_ptr, holder_idx, n_global, relax=1.0, z_prev=None):
    """Consensus step of Eq. 8b-c / Alg. 2 over Gaussians held by several blocks.

    For each global id with holder local indices H (ascending block order):
        xh_k = relax * x_k + (1 - relax) * z_prev      (over-relaxation, Sec. 3.3)
        z    = (1/|H|) sum_k xh_k                      (Eq. 8b, simplified form)
        u_k  = u_k + xh_k - z                          (Eq. 8c)
        w_k  = z - u_k
    The mean runs over the blocks that hold the Gaussian.  Returns (z [A][G],
    u_local, w_local) in FP64."""
    x = np.asarray(x_local, np.float64)
    u = np.array(u_local, np.float64, copy=True)
    A = x.shape[0]
    z = np.zeros((A, n_global))
    w = np.zeros_like(x)
    for gid in range(n_global):
        hs = holder_idx[holder_ptr[gid]:holder_ptr[gid + 1]]
        if len(hs) == 0:
            continue
        xs = x[:, hs]
        if relax != 1.0:
            xs = relax * xs + (1 - relax) * np.asarray(z_prev, np.float64)[:, gid:gid + 1]
        acc = np.zeros(A)
        for j in range(xs.shape[1]):       # ascending block order
            acc = acc + xs[:, j]
        zg = acc / len(hs)
        z[:, gid] = zg
        for j, h in enumerate(hs):
            u[:, h] = u[:, h] + xs[:, j] - zg
            w[:, h] = zg - u[:, h]
    return z, u, w


def consensus_full(x_local, u_local, holder_ptr, holder_idx, n_global):
    """Unsimplified z-update (supplementary Sec. B): z = mean over holders of
    (x_k + u_k).  Equal to the simplified form once the duals average to zero."""
    x = np.asarray(x_local, np.float64)
    u = np.asarray(u_local, np.float64)
    z = np.zeros((x.shape[0], n_global))
    for gid in range(n_global):
        hs = holder_idx[holder_ptr[gid]:holder_ptr[gid + 1]]
        if len(hs):
            z[:, gid] = (x[:, hs] + u[:, hs]).mean(axis=1)
    return z


def unscaled_lagrangian(f, x, z, y, rho):
    """Augmented Lagrangian of Eq. 5: sum_i f_i + y_i^T (x_i - z) + rho/2 ||x_i - z||^2."""
    return sum(fi + yi @ (xi - z) + 0.5 * rho * (xi - z) @ (xi - z) for fi, xi, yi in zip(f, x, y))


def scaled_lagrangian(f, x, z, u, rho):
    """Scaled form of Eq. 7: sum_i f_i + rho/2 ||x_i - z + u_i||^2 - rho/2 ||u_i||^2."""
    return sum(fi + 0.5 * rho * (xi - z + ui) @ (xi - z + ui) - 0.5 * rho * ui @ ui
               for fi, xi, ui in zip(f, x, u))


def residual_sums(x_local, z_new, z_prev, holder_ptr, holder_idx, n_global):
    """Squared residual sums per attribute group (Sec. 3.3), over the local
    copies of every Gaussian held by at least one block:

        primal  sum_k ||x_k - z||^2            (r = x_i - z, one term per copy)
        dual    sum_k ||z - z_prev||^2         (s = rho (z - z_prev), one term
                                                per copy, without the rho^2)

    Reading: the dual residual is counted once per holding block, as the
    primal one is (the consensus form of the residuals in the cited Boyd et
    al. survey).  Returns (primal[5], dual[5]) in GROUPS order, FP64."""
    x = np.asarray(x_local, np.float64)
    zn = np.asarray(z_new, np.float64)
    zp = np.asarray(z_prev, np.float64)
    grp = penalty_groups(x.shape[0])
    rp = np.zeros(5)
    rd = np.zeros(5)
    for gid in range(n_global):
        hs = holder_idx[holder_ptr[gid]:holder_ptr[gid + 1]]
        if len(hs) == 0:
            continue
        dp = ((x[:, hs] - zn[:, gid:gid + 1]) ** 2).sum(axis=1)
        dd = len(hs) * (zn[:, gid] - zp[:, gid]) ** 2
        np.add.at(rp, grp, dp)
        np.add.at(rd, grp, dd)
    return rp, rd


def adaptive_rho(rho, primal_sq, dual_sq, mu=10.0, tau_inc=2.0, tau_dec=2.0):
    """Penalty update of Sec. 3.3 per attribute group:

        rho * tau_inc   when ||r|| > mu ||s||
        rho / tau_dec   when ||s|| > mu ||r||
        rho             otherwise

    with ||r|| = sqrt(primal_sq) and ||s|| = rho * sqrt(dual_sq).  The paper's
    third branch reads "=" where "otherwise" is meant.  Returns the new rho
    (FP64 array of 5)."""
    rho = np.asarray(rho, np.float64)
    r = np.sqrt(np.asarray(primal_sq, np.float64))
    s = rho * np.sqrt(np.asarray(dual_sq, np.float64))
    out = rho.copy()
    inc = r > mu * s
    dec = ~inc & (s > mu * r)
    out[inc] = rho[inc] * tau_inc
    out[dec] = rho[dec] / tau_dec
    return out


def rescale_duals(u_local, z_global, holder_ptr, holder_idx, n_global, scale):
    """Scaled duals after a penalty change: u = y / rho, so keeping y fixed
    while rho becomes rho' multiplies u by rho / rho' (per group, ``scale``);
    the consensus targets follow, w = z - u.  The paper does not spell this
    step out; it is the rule of the scaled form (supplementary A).  Columns
    held by no Gaussian are left as they are (u) or zero (w).  Returns
    (u, w) in FP64."""
    u = np.array(u_local, np.float64, copy=True)
    z = np.asarray(z_global, np.float64)
    grp = penalty_groups(u.shape[0])
    sc = np.asarray(scale, np.float64)[grp][:, None]
    w = np.zeros_like(u)
    for gid in range(n_global):
        hs = holder_idx[holder_ptr[gid]:holder_ptr[gid + 1]]
        if len(hs) == 0:
            continue
        u[:, hs] = u[:, hs] * sc
        w[:, hs] = z[:, gid:gid + 1] - u[:, hs]
    return u, w
