"""Tile binning and the (tile, depth) order (oracle).

The index-mapping subsection of PocketGS says a GPU sort produces the
permutation pi from sorted index i to canonical index pi(i), and rendering
and backpropagation walk the sorted view.  The paper does not give the key;
the reading here:

  * a Gaussian overlaps every tile of its inclusive rectangle (projection.py);
  * tile_global = view_offset + ty * TX + tx (row-major);
  * key = tile_global * 2^32 + bits(float32 depth); depth > 0.2 so the float
    bits order like the values;
  * order = lexicographic (tile, depth bits, canonical id): a stable sort of
    pairs emitted in canonical order, each Gaussian's tiles in row-major order;
  * per-tile ranges [start, end) into the sorted list; an empty tile has [0, 0).

`bin_and_sort` builds the pairs with plain loops and orders them with
numpy.lexsort (a library sort is one step, as the definition allows).
"""

from __future__ import annotations

import numpy as np


def depth_bits(depth32: np.ndarray) -> np.ndarray:
    return np.asarray(depth32, np.float32).view(np.uint32).astype(np.uint64)


def emit_pairs(proj: dict, view_offset: int = 0):
    """Unsorted (keys, values) in emission order: canonical id ascending, then
    the Gaussian's tiles row-major."""
    TX, _ = proj["tiles"]
    rect = proj["rect"]
    vis = proj["visible"]
    dbits = depth_bits(proj["depth32"])
    keys, vals = [], []
    for g in np.nonzero(vis)[0]:
        x0, y0, x1, y1 = (int(t) for t in rect[g])
        for ty in range(y0, y1 + 1):
            for tx in range(x0, x1 + 1):
                tile = view_offset + ty * TX + tx
                keys.append((np.uint64(tile) << np.uint64(32)) | dbits[g])
                vals.append(g)
    return np.asarray(keys, np.uint64), np.asarray(vals, np.uint32)


def stable_sort_pairs(keys: np.ndarray, vals: np.ndarray):
    """Stable sort by the 64-bit key (ties keep emission order)."""
    order = np.argsort(keys, kind="stable")
    return keys[order], vals[order]


def bin_and_sort(proj: dict, view_offset: int = 0, n_tiles: int | None = None):
    """Returns dict(keys, values, ranges (n_tiles, 2), num_pairs)."""
    TX, TY = proj["tiles"]
    if n_tiles is None:
        n_tiles = view_offset + TX * TY
    keys, vals = emit_pairs(proj, view_offset)
    if keys.size:
        tile = (keys >> np.uint64(32)).astype(np.int64)
        dep = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
        order = np.lexsort((vals.astype(np.int64), dep, tile))
        keys, vals = keys[order], vals[order]
    ranges = np.zeros((n_tiles, 2), np.int64)
    if keys.size:
        tile = (keys >> np.uint64(32)).astype(np.int64)
        starts = np.searchsorted(tile, np.arange(n_tiles), side="left")
        ends = np.searchsorted(tile, np.arange(n_tiles), side="right")
        nonempty = ends > starts
        ranges[:, 0] = np.where(nonempty, starts, 0)
        ranges[:, 1] = np.where(nonempty, ends, 0)
    return dict(keys=keys, values=vals, ranges=ranges, num_pairs=int(keys.size))


def tile_lists(bins: dict):
    """List of per-tile canonical-id arrays in sorted order."""
    return [bins["values"][s:e] for s, e in bins["ranges"]]
