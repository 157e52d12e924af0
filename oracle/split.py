"""Oracle of the recursive scene splitting (Alg. 1) and the overlap
expansion that creates shared Gaussians (Sec. 3.2, scene splitting)
(test infrastructure).  Plain Python over small inputs, FP64.

Alg. 1, as read here:
  * the scene box is the tight axis-aligned box of all points;
  * rounds: while there are fewer than K cells, take the current cells in
    order (first in, first out); each is removed, split in two along its
    longer ground axis, its points grouped into the two halves, and the two
    re-tightened boxes appended;
  * readings where the paper is silent: the split puts the floor(n/2) points
    with the smallest (coordinate, point id) in the first half (the median
    split, so that blocks hold similar numbers of points, the paper's
    balance constraint); the "longer axis" is the longer of the ground
    axes (the paper assumes one axis is aligned with the ground and splits
    the ground plane), ties to the lower axis index; when K is not a power
    of two the last round stops as soon as there are K cells; a cell of a
    single point cannot be cut in two non-empty halves, so its turn takes
    it out and appends it again unchanged (K <= n still ends with K cells,
    since some cell holds two points while there are fewer than n cells).
Overlap (Sec. 3.2): every cell box is scaled by s about its centre and a
point (or a camera centre) belongs to every block whose scaled box covers it
(inclusive bounds), so points near a cut are shared by both sides.  The
scaled box is computed as each side moved out by (s - 1) / 2 of the extent.
"""
from __future__ import annotations

import numpy as np


def tight_box(pts, ids):
    """[lo xyz, hi xyz] of the given points (FP64)."""
    lo = [min(pts[i][a] for i in ids) for a in range(3)]
    hi = [max(pts[i][a] for i in ids) for a in range(3)]
    return lo + hi


def split_cells(points, K, ground_axes=(0, 2)):
    """Alg. 1: returns the K cells as (box, point ids) in the order the
    algorithm leaves them."""
    pts = [tuple(float(v) for v in p) for p in np.asarray(points, np.float64)]
    n = len(pts)
    if K < 1 or K > n:
        raise ValueError("need 1 <= K <= number of points")
    all_ids = list(range(n))
    cells = [(tight_box(pts, all_ids), all_ids)]
    while len(cells) < K:
        current = list(cells)                 # this round's cells, first in first out
        while current and len(cells) < K:
            box, ids = current.pop(0)
            cells.remove((box, ids))
            if len(ids) < 2:
                cells.append((box, ids))
                continue
            ext = {a: box[3 + a] - box[a] for a in ground_axes}
            axis = max(ground_axes, key=lambda a: (ext[a], -a))
            order = sorted(ids, key=lambda i: (pts[i][axis], i))
            half = len(order) // 2
            first, second = sorted(order[:half]), sorted(order[half:])
            cells.append((tight_box(pts, first), first))
            cells.append((tight_box(pts, second), second))
    return cells


def expand_box(box, s):
    """Box scaled by s about its centre, written as each side moved out by
    (s - 1) / 2 of the extent (the same box; exact at s = 1, so a block
    always covers its own cell)."""
    lo, hi = box[:3], box[3:]
    g = [(s - 1.0) / 2.0 * (hi[a] - lo[a]) for a in range(3)]
    return [lo[a] - g[a] for a in range(3)] + [hi[a] + g[a] for a in range(3)]


def group(boxes, s, points, axes=(0, 1, 2)):
    """Per block, the ascending ids of the points its scaled box covers on
    the given axes (all three for points; the ground axes for camera
    centres, which sit above the point cloud: the paper assigns views by
    their ground-plane cell)."""
    pts = np.asarray(points, np.float64)
    out = []
    for box in boxes:
        e = expand_box(box, s)
        out.append([i for i in range(len(pts))
                    if all(e[a] <= pts[i][a] <= e[3 + a] for a in axes)])
    return out
