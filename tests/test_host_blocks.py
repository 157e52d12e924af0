"""Host-side block bookkeeping of the K-block trainer (no GPU): the holder
grouped numbering of the global ids and the block store built on it."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")

from paper_2405_13943_amd import admm  # noqa: E402


def _blocks(seed, K=4, G=500):
    r = np.random.default_rng(seed)
    held = [sorted(r.choice(K, r.integers(0 if g % 17 == 0 else 1, 4), replace=False)) for g in range(G)]
    return [np.array([g for g in range(G) if k in held[g]], np.int64) for k in range(K)], held


@pytest.mark.parametrize("seed", [0, 1])
def test_holder_order_groups_holder_sets(seed):
    local_gid, held = _blocks(seed)
    G = len(held)
    perm, inv = admm.holder_order(local_gid, G)
    assert np.array_equal(np.sort(perm), np.arange(G)) and np.array_equal(perm[inv], np.arange(G))
    sets = [tuple(held[i]) for i in perm]
    # every holder set forms one run of consecutive new ids, unheld ids last
    runs = [sets[0]] + [b for a, b in zip(sets, sets[1:]) if a != b]
    assert len(runs) == len(set(runs))
    assert all(len(s) > 0 for s in sets[:sum(1 for h in held if h)]) and all(not s for s in sets[sum(1 for h in held if h):])
    # original order kept inside a group
    for s in set(sets):
        ids = perm[[i for i, t in enumerate(sets) if t == s]]
        assert np.all(np.diff(ids) > 0)


def test_block_model_store_order_and_round_trip():
    """Every block's copies are stored in ascending new id, the holder CSR
    points at copies of the right Gaussian, the consensus of identical
    copies returns z, and global_params restores the caller's order."""
    local_gid, held = _blocks(2)
    G, A = len(held), 14
    params = np.random.default_rng(3).standard_normal((A, G)).astype(np.float32)
    model = admm.BlockModel.from_global(params, local_gid, device="cpu")
    x = model.x.numpy().astype(np.float64)
    z = model.z.numpy().astype(np.float64)
    ptr, idx = model.holder_ptr.numpy(), model.holder_idx.numpy()
    for k in range(model.K):
        a, b = model.block(k)
        assert np.array_equal(model.local_gid[k], np.sort(model.local_gid[k])) and b - a == len(local_gid[k])
        np.testing.assert_array_equal(x[:, a:b], z[:, model.local_gid[k]])
    for g in range(G):
        hs = idx[ptr[g]:ptr[g + 1]]
        assert len(hs) == len(held[model.perm[g]])
        assert np.all(x[:, hs] == z[:, g:g + 1])
    zc, uc, _ = oracle.consensus(x, np.zeros_like(x), ptr, idx, G)
    held_new = np.diff(ptr) > 0
    np.testing.assert_array_equal(zc[:, held_new], z[:, held_new])
    np.testing.assert_array_equal(model.global_params().numpy(), params)
    plain = admm.BlockModel.from_global(params, local_gid, device="cpu", group_holders=False)
    np.testing.assert_array_equal(plain.global_params().numpy(), params)


def test_holder_groups_ordered_inside_by_rank():
    """A rank inside the holder groups reorders each group and nothing else:
    the groups keep their places and sizes."""
    r = np.random.default_rng(8)
    G = 400
    local_gid = [np.sort(r.choice(G, 150, replace=False)), np.sort(r.choice(G, 220, replace=False))]
    perm0, _ = admm.holder_order(local_gid, G)
    rank = r.permutation(G)
    perm1, inv1 = admm.holder_order(local_gid, G, within=rank)
    mask = np.zeros(G, np.int64)
    for k, g in enumerate(local_gid):
        mask[g] |= 1 << k
    assert np.array_equal(mask[perm0], mask[perm1])            # same group at every position
    for m in np.unique(mask):
        ids = perm1[mask[perm1] == m]
        assert np.all(np.diff(rank[ids]) > 0)                  # rank order inside the group
    assert np.array_equal(inv1[perm1], np.arange(G))
