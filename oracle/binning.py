"""Tile-binning reference (test infrastructure).

The paper does not describe tiling; the rasterizer's result is the per-pixel
definition in ``orc.c``.  Binning is an acceleration, and its integer output
is checked bit for bit against this reference: given each record's integer
tile rectangle and the FP32 bit pattern of its depth, emit one
(tile, depth-bits) key per covered tile in record order, stable-sort by key,
and cut the sorted list into per-tile ranges.
"""
from __future__ import annotations

import numpy as np


def bin_reference(rects, depth_bits, tile_base, tiles_x, job_of_record, n_tiles_total):
    """rects: [R][4] int (tx0, ty0, tx1, ty1) inclusive, empty when tx0 > tx1;
    depth_bits: [R] uint32; tile_base/tiles_x: per job; job_of_record: [R].

    Returns (values [P] uint32 record ids in sorted order,
             ranges [n_tiles_total][2] uint32 start/end)."""
    keys, vals = [], []
    for r in range(len(rects)):
        x0, y0, x1, y1 = (int(v) for v in rects[r])
        if x0 > x1 or y0 > y1:
            continue
        j = int(job_of_record[r])
        for ty in range(y0, y1 + 1):
            for tx in range(x0, x1 + 1):
                tile = int(tile_base[j]) + ty * int(tiles_x[j]) + tx
                keys.append((tile << 32) | int(depth_bits[r]))
                vals.append(r)
    keys = np.asarray(keys, np.uint64)
    vals = np.asarray(vals, np.uint32)
    order = np.argsort(keys, kind="stable")
    keys, vals = keys[order], vals[order]
    ranges = np.zeros((n_tiles_total, 2), np.uint32)
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    for i in range(len(tiles)):
        t = tiles[i]
        if i == 0 or tiles[i - 1] != t:
            ranges[t, 0] = i
        if i == len(tiles) - 1 or tiles[i + 1] != t:
            ranges[t, 1] = i + 1
    return vals, ranges
