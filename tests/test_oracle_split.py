"""Pins of the scene-splitting oracle (Alg. 1 and the overlap expansion):
worked examples by hand, balance and partition invariants, brute force."""
import numpy as np
import pytest

from oracle import split


def test_worked_example_two_cells():
    """Six points on a 4 x 1 ground rectangle: the longer ground axis is x,
    the three smallest x go left, the boxes are re-tightened."""
    pts = [(0.0, 0, 0.0), (3.0, 0, 1.0), (1.0, 5, 0.5), (4.0, 0, 0.0), (2.0, 0, 1.0), (0.5, 0, 0.2)]
    cells = split.split_cells(pts, 2)
    assert [ids for _, ids in cells] == [[0, 2, 5], [1, 3, 4]]
    assert cells[0][0] == [0.0, 0.0, 0.0, 1.0, 5.0, 0.5]
    assert cells[1][0] == [2.0, 0.0, 0.0, 4.0, 0.0, 1.0]
    # odd count: floor(n / 2) points in the first half
    odd = split.split_cells([(float(x), 0.0, 0.0) for x in [3, 0, 4, 1, 2]], 2)
    assert [ids for _, ids in odd] == [[1, 3], [0, 2, 4]]


def test_vertical_axis_is_never_split():
    """A tall thin column (y up) still splits along the longer ground axis."""
    r = np.random.default_rng(0)
    pts = np.stack([r.random(50), 100 * r.random(50), 3 * r.random(50)], 1)
    cells = split.split_cells(pts, 2)
    za = [max(pts[i][2] for i in ids) for _, ids in cells]
    zb = [min(pts[i][2] for i in ids) for _, ids in cells]
    assert za[0] <= zb[1]                   # cut along z (extent 3 > 1)


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 8])
def test_partition_and_balance(K):
    """The cells partition the points; with the median split the block
    sizes differ by at most one point per round of halving."""
    r = np.random.default_rng(K)
    pts = np.concatenate([r.normal([0, 0, 0], [5, 1, 2], (150, 3)), r.normal([20, 0, 5], [2, 1, 2], (50, 3))])
    cells = split.split_cells(pts, K)
    assert len(cells) == K
    ids = sorted(i for _, c in cells for i in c)
    assert ids == list(range(len(pts)))
    sizes = [len(c) for _, c in cells]
    rounds = int(np.ceil(np.log2(K))) if K > 1 else 0
    if K == 2 ** rounds:
        assert max(sizes) - min(sizes) <= rounds
    for box, c in cells:                    # boxes are tight
        assert box == split.tight_box([tuple(p) for p in pts], c)


def test_expansion_worked_example_and_containment():
    box = [0.0, 0.0, 0.0, 2.0, 4.0, 6.0]
    assert split.expand_box(box, 1.5) == [-0.5, -1.0, -1.5, 2.5, 5.0, 7.5]
    r = np.random.default_rng(3)
    pts = r.random((120, 3)) * [10, 1, 10]
    cells = split.split_cells(pts, 4)
    boxes = [b for b, _ in cells]
    g1 = split.group(boxes, 1.0, pts)
    for (_, c), g in zip(cells, g1):        # s = 1: each block holds its own cell
        assert set(c) <= set(g)
    g14 = split.group(boxes, 1.4, pts)
    assert sum(map(len, g14)) > sum(map(len, g1))
    for a, b in zip(g1, g14):
        assert set(a) <= set(b)


def test_group_brute_force():
    r = np.random.default_rng(4)
    pts = r.random((40, 3))
    boxes = [[0.1, 0.0, 0.2, 0.5, 1.0, 0.6], [0.4, 0.2, 0.0, 0.9, 0.8, 1.0]]
    got = split.group(boxes, 1.2, pts)
    for box, g in zip(boxes, got):
        c = (np.array(box[:3]) + np.array(box[3:])) / 2
        h = (np.array(box[3:]) - np.array(box[:3])) / 2 * 1.2
        want = [i for i in range(40) if np.all(np.abs(pts[i] - c) <= h + 1e-15)]
        assert g == want


def test_rounds_split_every_cell_first_in_first_out():
    """K = 4 from 8 points on a line: round one cuts at the middle, round two
    cuts each half, cells in the order the algorithm appends them."""
    pts = [(float(x), 0.0, 0.0) for x in [7, 1, 5, 3, 0, 6, 2, 4]]
    cells = split.split_cells(pts, 4)
    assert [[pts[i][0] for i in c] for _, c in cells] == [[1.0, 0.0], [3.0, 2.0], [5.0, 4.0], [7.0, 6.0]]
    three = split.split_cells(pts, 3)
    assert [sorted(pts[i][0] for i in c) for _, c in three] == [[4.0, 5.0, 6.0, 7.0], [0.0, 1.0], [2.0, 3.0]]


def test_single_point_cells_wait_their_turn():
    """Three points on the x axis, K = 3 (worked by hand).  Round 1 cuts
    {0, 1, 2} at the median: {0} and {1, 2}.  Round 2 takes {0} first; it
    cannot be cut, so it is appended again unchanged; then {1, 2} is cut
    into {1} and {2}.  Cells in order: {0}, {1}, {2}."""
    pts = [[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [2.0, 0.0, 0.0]]
    cells = split.split_cells(pts, 3)
    assert [ids for _, ids in cells] == [[0], [1], [2]]
    assert [box for box, _ in cells] == [[0.0, 0, 0, 0.0, 0, 0], [1.0, 0, 0, 1.0, 0, 0], [2.0, 0, 0, 2.0, 0, 0]]
    # five points, K = 5.  Round 1: {0,1} {2,3,4}.  Round 2: {2,3,4} {0} {1},
    # then {0} {1} {2} {3,4}.  Round 3: {0}, {1} and {2} are appended again
    # in turn, leaving {3,4} {0} {1} {2}; the cut of {3,4} gives the order
    # {0} {1} {2} {3} {4}
    pts5 = [[float(i), 0.0, 0.0] for i in range(5)]
    got = [ids for _, ids in split.split_cells(pts5, 5)]
    assert got == [[0], [1], [2], [3], [4]]
    # six points, K = 5: round 2 leaves {0} {1,2} {3} {4,5}; round 3 appends
    # {0} again, then cuts {1,2}: {3} {4,5} {0} {1} {2}
    pts6 = [[float(i), 0.0, 0.0] for i in range(6)]
    assert [ids for _, ids in split.split_cells(pts6, 5)] == [[3], [4, 5], [0], [1], [2]]
