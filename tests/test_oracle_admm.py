"""Pins of the optimiser, consensus and binning oracles (P7-P13): closed forms,
a library optimiser, textbook consensus-ADMM convergence and brute force."""
import numpy as np
import pytest

import oracle
from oracle.admm import penalty_groups


def _state(A=14, N=50, seed=0):
    r = np.random.default_rng(seed)
    return (r.standard_normal((A, N)), r.standard_normal((A, N)), r.standard_normal((A, N)))


LR = (1e-3, 2e-3, 3e-3, 4e-3, 5e-3)
RHO = (1e4, 1e4, 1e4, 1e3, 1e4)


def test_first_adam_step_closed_form():
    """From zero moments the first step is -lr g' / (|g'| + eps) with
    g' = g + rho (x - w) (P7)."""
    x, g, w = _state()
    z = np.zeros_like(x)
    x1, m1, v1 = oracle.adam_admm(x, g, z, z, w, LR, RHO, step=1)
    grp = penalty_groups(x.shape[0])
    gp = g + np.asarray(RHO)[grp][:, None] * (x - w)
    lr = np.asarray(LR)[grp][:, None]
    np.testing.assert_allclose(x1, x - lr * gp / (np.abs(gp) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * gp, rtol=1e-12)
    np.testing.assert_allclose(v1, 0.001 * gp * gp, rtol=1e-12)


def test_adam_matches_torch_optimizer():
    """Without the penalty the update is torch.optim.Adam; with it, torch.optim.Adam
    fed the penalised gradient (library routine, several steps)."""
    torch = pytest.importorskip("torch")
    x0, _, w = _state(A=14, N=30, seed=3)
    r = np.random.default_rng(9)
    grads = [r.standard_normal(x0.shape) for _ in range(5)]
    grp = penalty_groups(14)
    for rho in ((0.0,) * 5, RHO):
        params = [torch.tensor(x0[grp == k], dtype=torch.float64, requires_grad=True) for k in range(5)]
        opt = torch.optim.Adam([{"params": [params[k]], "lr": LR[k]} for k in range(5)],
                               betas=(0.9, 0.999), eps=1e-8)
        x, m, v = x0.copy(), np.zeros_like(x0), np.zeros_like(x0)
        for t, g in enumerate(grads, start=1):
            x, m, v = oracle.adam_admm(x, g, m, v, w, LR, rho, step=t)
            opt.zero_grad()
            for k in range(5):
                sel = grp == k
                pen = rho[k] * (params[k].detach().numpy() - w[sel])
                params[k].grad = torch.tensor(g[sel] + pen, dtype=torch.float64)
            opt.step()
        for k in range(5):
            np.testing.assert_allclose(x[grp == k], params[k].detach().numpy(), rtol=1e-10, atol=1e-12)


def test_penalty_alone_pulls_to_consensus_target():
    """With zero image gradient, Adam on rho/2 ||x - w||^2 converges to x = w (P8)."""
    x, _, w = _state(N=20, seed=4)
    m, v = np.zeros_like(x), np.zeros_like(x)
    for t in range(1, 6001):
        x, m, v = oracle.adam_admm(x, np.zeros_like(x), m, v, w, (1e-2,) * 5, (1.0,) * 5, step=t)
    assert np.abs(x - w).max() < 1e-3


def test_mask_restricts_penalty():
    x, g, w = _state(N=10, seed=5)
    z = np.zeros_like(x)
    mask = (np.arange(10) % 2).astype(np.float64)
    x1, _, _ = oracle.adam_admm(x, g, z, z, w, LR, RHO, step=1, mask=mask)
    x0, _, _ = oracle.adam_admm(x, g, z, z, None, LR, RHO, step=1)
    np.testing.assert_array_equal(x1[:, mask == 0], x0[:, mask == 0])
    assert not np.allclose(x1[:, mask == 1], x0[:, mask == 1])


def _holders(K=3, G=40, seed=6):
    """Random holder sets: each global id held by 1..K blocks, locals laid out
    block by block in ascending global id."""
    r = np.random.default_rng(seed)
    held = [sorted(r.choice(K, r.integers(1, K + 1), replace=False)) for _ in range(G)]
    local_of = {}
    locs = []
    for k in range(K):
        for g in range(G):
            if k in held[g]:
                local_of[(g, k)] = len(locs)
                locs.append(g)
    ptr = np.zeros(G + 1, np.int64)
    idx = []
    for g in range(G):
        idx += [local_of[(g, k)] for k in held[g]]
        ptr[g + 1] = len(idx)
    return np.asarray(idx, np.int64), ptr, np.asarray(locs), held


def test_consensus_toy_problem_converges_to_holder_mean():
    """Consensus ADMM on f_k(x) = 1/2 ||x - a_k||^2 with the exact x-update
    x = (a_k + rho (z - u)) / (1 + rho) converges to the mean of a_k over the
    blocks that hold each variable (Boyd et al., consensus ADMM) (P9)."""
    idx, ptr, locs, held = _holders()
    L, A, rho = len(locs), 5, 0.7
    a = np.random.default_rng(7).standard_normal((A, L))
    z = np.zeros((A, len(ptr) - 1))
    u = np.zeros((A, L))
    for _ in range(300):
        x = (a + rho * (z[:, locs] - u)) / (1 + rho)
        z, u, _ = oracle.consensus(x, u, ptr, idx, len(ptr) - 1)
    ref = np.stack([a[:, idx[ptr[g]:ptr[g + 1]]].mean(axis=1) for g in range(len(ptr) - 1)], axis=1)
    np.testing.assert_allclose(z, ref, atol=1e-9)


def test_duals_average_to_zero_and_full_form_agrees():
    """After each consensus the holder-mean of u is zero (supplementary B),
    so the simplified z equals the full form mean(x + u) (P10)."""
    idx, ptr, locs, _ = _holders(seed=8)
    L, A = len(locs), 4
    r = np.random.default_rng(9)
    u = np.zeros((A, L))
    for _ in range(5):
        x = r.standard_normal((A, L))
        zf = oracle.consensus_full(x, u, ptr, idx, len(ptr) - 1)
        z, u, w = oracle.consensus(x, u, ptr, idx, len(ptr) - 1)
        np.testing.assert_allclose(z, zf, atol=1e-12)
        for g in range(len(ptr) - 1):
            hs = idx[ptr[g]:ptr[g + 1]]
            np.testing.assert_allclose(u[:, hs].mean(axis=1), 0, atol=1e-12)
        np.testing.assert_allclose(w, z[:, locs] - u, atol=1e-15)


def test_identical_copies_are_a_fixed_point():
    """Identical local copies give z = x and leave u unchanged (P11); a
    Gaussian held by one block gets z = x, u = 0."""
    idx, ptr, locs, _ = _holders(seed=10)
    A = 3
    zg = np.random.default_rng(11).standard_normal((A, len(ptr) - 1))
    x = zg[:, locs]
    u0 = np.zeros_like(x)
    z, u, w = oracle.consensus(x, u0, ptr, idx, len(ptr) - 1)
    np.testing.assert_allclose(z, zg, atol=1e-15)
    np.testing.assert_allclose(u, 0, atol=1e-15)


def test_over_relaxation_reduces_to_plain_at_one():
    idx, ptr, locs, _ = _holders(seed=12)
    r = np.random.default_rng(13)
    x = r.standard_normal((3, len(locs)))
    u = r.standard_normal((3, len(locs)))
    zp = r.standard_normal((3, len(ptr) - 1))
    a = oracle.consensus(x, u, ptr, idx, len(ptr) - 1, relax=1.0, z_prev=zp)
    b = oracle.consensus(x, u, ptr, idx, len(ptr) - 1)
    for p, q in zip(a, b):
        np.testing.assert_array_equal(p, q)
    # relax = alpha: xh = alpha x + (1 - alpha) z_prev (Sec. 3.3, sign typo read as +)
    c = oracle.consensus(x, u, ptr, idx, len(ptr) - 1, relax=1.6, z_prev=zp)
    xh = 1.6 * x + (1 - 1.6) * zp[:, locs]
    d = oracle.consensus(xh, u, ptr, idx, len(ptr) - 1)
    for p, q in zip(c, d):
        np.testing.assert_allclose(p, q, atol=1e-14)


def test_scaled_and_unscaled_lagrangian_agree():
    """Eq. 5 equals Eq. 7 with u = y / rho (supplementary A, with the
    completed square read as ||r + y/rho||^2) (P13)."""
    r = np.random.default_rng(14)
    rho = 2.5
    x = r.standard_normal((4, 6))
    z = r.standard_normal(6)
    y = r.standard_normal((4, 6))
    f = r.standard_normal(4)
    a = oracle.unscaled_lagrangian(f, x, z, y, rho)
    b = oracle.scaled_lagrangian(f, x, z, y / rho, rho)
    assert abs(a - b) < 1e-12 * max(1, abs(a))


def test_bin_reference_brute_force():
    """Each tile's list holds exactly the records whose rectangle covers it,
    ordered by (depth bits, record index) (P12)."""
    r = np.random.default_rng(15)
    R = 300
    tiles_x, tiles_y = [5, 3], [4, 6]
    base = [0, 20]
    job = r.integers(0, 2, R)
    rects = np.zeros((R, 4), np.int64)
    for i in range(R):
        tx, ty = tiles_x[job[i]], tiles_y[job[i]]
        x0, y0 = r.integers(0, tx), r.integers(0, ty)
        rects[i] = [x0, y0, min(tx - 1, x0 + r.integers(-1, 3)), min(ty - 1, y0 + r.integers(0, 3))]
    depth = r.integers(1, 50, R).astype(np.uint32)          # many ties
    vals, ranges = oracle.bin_reference(rects, depth, base, tiles_x, job, 38)
    for t in range(38):
        j = 0 if t < 20 else 1
        lt = t - base[j]
        tx, ty = lt % tiles_x[j], lt // tiles_x[j]
        want = [i for i in range(R) if job[i] == j and rects[i, 0] <= tx <= rects[i, 2]
                and rects[i, 1] <= ty <= rects[i, 3]]
        want.sort(key=lambda i: (int(depth[i]), i))
        got = list(vals[ranges[t, 0]:ranges[t, 1]])
        assert got == want, t
