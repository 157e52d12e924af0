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


def test_residual_sums_worked_example():
    """One Gaussian held by two blocks, every plane of copy a at 1 and of
    copy b at 3, previous z at 0: z = 2, each plane adds (1-2)^2 + (3-2)^2 = 2
    to the primal sum and 2 copies x (2-0)^2 = 8 to the dual sum (Sec. 3.3).
    Planes per group (p, q, s, f, o) at SH degree 1: means 3, rotation 4,
    scales 3, SH colour 3 x 4 = 12, opacity 1."""
    A = 14 + 9
    x = np.concatenate([np.ones((A, 1)), 3 * np.ones((A, 1))], axis=1)
    ptr, idx = np.array([0, 2]), np.array([0, 1])
    z, _, _ = oracle.consensus(x, np.zeros_like(x), ptr, idx, 1)
    np.testing.assert_array_equal(z, 2.0)
    rp, rd = oracle.residual_sums(x, z, np.zeros((A, 1)), ptr, idx, 1)
    np.testing.assert_array_equal(rp, [6, 8, 6, 24, 2])
    np.testing.assert_array_equal(rd, [24, 32, 24, 96, 8])


def test_primal_residual_is_the_dual_increment():
    """Without relaxation the u-update adds x - z to every copy, so the
    primal sum equals sum ||u_new - u_old||^2 (Eq. 8c); at the holder mean it
    also equals sum ||x||^2 - |H| ||z||^2 (variance split)."""
    idx, ptr, locs, _ = _holders(seed=20)
    r = np.random.default_rng(21)
    A, L, G = 14, len(locs), len(ptr) - 1
    x = r.standard_normal((A, L))
    u0 = r.standard_normal((A, L))
    zp = r.standard_normal((A, G))
    z, u1, _ = oracle.consensus(x, u0, ptr, idx, G)
    rp, rd = oracle.residual_sums(x, z, zp, ptr, idx, G)
    grp = penalty_groups(A)
    want = np.array([((u1 - u0)[grp == k] ** 2).sum() for k in range(5)])
    np.testing.assert_allclose(rp, want, rtol=1e-12)
    cnt = np.diff(ptr)
    split = np.array([(x[grp == k] ** 2).sum() - (cnt * (z[grp == k] ** 2)).sum() for k in range(5)])
    np.testing.assert_allclose(rp, split, rtol=1e-10)
    # dual: every local copy sees the move of its own z
    dz = (z - zp)[:, locs]
    np.testing.assert_allclose(rd, [(dz[grp == k] ** 2).sum() for k in range(5)], rtol=1e-12)


def test_adaptive_rho_branches():
    """rho grows by tau_inc when ||r|| > mu ||s||, shrinks by tau_dec when
    ||s|| > mu ||r|| (||s|| carries the factor rho), stays otherwise (Sec. 3.3)."""
    rho = np.array([1.0, 1.0, 2.0, 0.5, 1.0])
    # ||r|| = 11, ||s|| = 1           -> inc
    # ||r|| = 1,  ||s|| = 11          -> dec
    # ||r|| = 4,  ||s|| = 2 * 2 = 4   -> keep
    # ||r|| = 0,  ||s|| = 0           -> keep
    # ||r|| = 9,  ||s|| = 1 (mu = 10) -> keep
    new = oracle.adaptive_rho(rho, [121, 1, 16, 0, 81], [1, 121, 4, 0, 1], mu=10, tau_inc=2, tau_dec=4)
    np.testing.assert_array_equal(new, [2.0, 0.25, 2.0, 0.5, 1.0])
    # equal residual sums: the factor rho in s decides (||r|| = 1, ||s|| = rho)
    np.testing.assert_array_equal(oracle.adaptive_rho([0.01] * 5, [1] * 5, [1] * 5), [0.02] * 5)
    np.testing.assert_array_equal(oracle.adaptive_rho([100.0] * 5, [1] * 5, [1] * 5), [50.0] * 5)


def test_dual_rescale_keeps_the_unscaled_x_update():
    """After rho -> rho', the scaled x-update with u' = u rho / rho' is the
    unscaled one of Eq. 5 with y = rho u held fixed: on f = 1/2 ||x - a||^2,
    argmin f + y (x - z) + rho'/2 ||x - z||^2 = (a - y + rho' z) / (1 + rho')."""
    idx, ptr, locs, _ = _holders(seed=22)
    r = np.random.default_rng(23)
    A, L, G = 14, len(locs), len(ptr) - 1
    a = r.standard_normal((A, L))
    u = r.standard_normal((A, L))
    z = r.standard_normal((A, G))
    grp = penalty_groups(A)
    rho = np.array([0.5, 1.0, 2.0, 4.0, 8.0])
    rho_new = np.array([1.0, 0.5, 2.0, 1.0, 16.0])
    u2, w2 = oracle.rescale_duals(u, z, ptr, idx, G, rho / rho_new)
    rn = rho_new[grp][:, None]
    scaled = (a + rn * w2) / (1 + rn)                       # w = z - u
    y = rho[grp][:, None] * u
    unscaled = (a - y + rn * z[:, locs]) / (1 + rn)
    np.testing.assert_allclose(scaled, unscaled, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(w2, z[:, locs] - u2, atol=1e-15)


def _toy_run(rho0, adaptive, iters=400, seed=24, tol=1e-8):
    idx, ptr, locs, _ = _holders(K=4, G=60, seed=seed)
    A, L, G = 14, len(locs), len(ptr) - 1
    grp = penalty_groups(A)
    a = np.random.default_rng(seed + 1).standard_normal((A, L)) * 3
    ref = np.stack([a[:, idx[ptr[g]:ptr[g + 1]]].mean(axis=1) for g in range(G)], axis=1)
    rho = np.full(5, rho0)
    z = np.zeros((A, G))
    u = np.zeros((A, L))
    for t in range(1, iters + 1):
        rn = rho[grp][:, None]
        x = (a + rn * (z[:, locs] - u)) / (1 + rn)
        z_prev = z
        z, u, _ = oracle.consensus(x, u, ptr, idx, G)
        if np.abs(z - ref).max() < tol:
            return t, z, ref
        if adaptive and t <= 100:
            rp, rd = oracle.residual_sums(x, z, z_prev, ptr, idx, G)
            new = oracle.adaptive_rho(rho, rp, rd)
            u, _ = oracle.rescale_duals(u, z, ptr, idx, G, rho / new)
            rho = new
    return iters, z, ref


@pytest.mark.parametrize("rho0", [1e3, 1e5])
def test_adaptive_penalty_recovers_from_a_poor_initial_rho(rho0):
    """Consensus ADMM on the quadratic toy problem converges to the holder
    mean with the residual-balancing penalty (frozen after 100 iterations
    here) and does so in far fewer iterations than with the poor fixed rho
    it started from (Sec. 3.3, the scheme of Boyd et al.).  On this problem
    z moves by the factor rho / (1 + rho) per iteration, so a large rho is the
    poor start."""
    t_ad, z, ref = _toy_run(rho0, True)
    np.testing.assert_allclose(z, ref, atol=1e-8)
    t_fx, _, _ = _toy_run(rho0, False)
    assert t_ad < 150 and t_fx == 400, (t_ad, t_fx)


def test_adaptive_penalty_keeps_a_good_rho_converging():
    """From a small rho the toy problem is solved in a few iterations with or
    without adaptation; adaptation must not spoil that."""
    t_ad, z, ref = _toy_run(1e-3, True)
    np.testing.assert_allclose(z, ref, atol=1e-8)
    assert t_ad < 20
