"""Tile/depth keys and the reference sort order (oracle; test infrastructure only).

Sec. III-A: Gaussians are sorted by depth and composited front to back. With
the image cut into tiles, every (Gaussian, tile) pair whose 3-sigma pixel
rectangle touches the tile gets a 64-bit key

    key = (tile_id << 32) | bits(t_z)          tile_id = ty * tiles_x + tx

(t_z > 0 after culling, so the IEEE bits of t_z order like t_z), and the
Gaussian index as value. Pairs are enumerated in Gaussian-index order, tiles
row-major inside each rectangle. The reference order sorts by key, then by
index: (tile, depth bits, index), a total order.
"""
from __future__ import annotations

import numpy as np

from .project import ScreenRecords


def tile_grid(width: int, height: int, tile_w: int, tile_h: int):
    return (width + tile_w - 1) // tile_w, (height + tile_h - 1) // tile_h


def make_pairs(rec: ScreenRecords, width: int, height: int, tile_w: int, tile_h: int):
    """Unsorted (key uint64, value uint32) pairs in emission order."""
    tiles_x, _ = tile_grid(width, height, tile_w, tile_h)
    idx = np.nonzero(rec.visible)[0]
    keys = []
    vals = []
    zbits = rec.z.astype(np.float32).view(np.uint32)
    for g in idx:
        tx0, tx1, ty0, ty1 = rec.tile_rect[g]
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                tid = ty * tiles_x + tx
                keys.append((np.uint64(tid) << np.uint64(32)) | np.uint64(zbits[g]))
                vals.append(g)
    return np.array(keys, dtype=np.uint64), np.array(vals, dtype=np.uint32)


def make_pairs_fast(rec: ScreenRecords, width: int, height: int, tile_w: int, tile_h: int):
    """Same pairs as ``make_pairs``, built with array ops (for large scenes)."""
    tiles_x, _ = tile_grid(width, height, tile_w, tile_h)
    idx = np.nonzero(rec.visible)[0]
    tr = rec.tile_rect[idx]
    wx = tr[:, 1] - tr[:, 0] + 1
    wy = tr[:, 3] - tr[:, 2] + 1
    cnt = wx * wy
    total = int(cnt.sum())
    owner = np.repeat(np.arange(idx.size), cnt)
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    local = np.arange(total) - start[owner]
    ty = tr[owner, 2] + local // wx[owner]
    tx = tr[owner, 0] + local % wx[owner]
    tid = (ty * tiles_x + tx).astype(np.uint64)
    zbits = rec.z.astype(np.float32).view(np.uint32)[idx][owner].astype(np.uint64)
    keys = (tid << np.uint64(32)) | zbits
    return keys, idx[owner].astype(np.uint32)


def sort_pairs(keys: np.ndarray, vals: np.ndarray):
    """Reference order: ascending key, ties by ascending value."""
    order = np.lexsort((vals, keys))
    return keys[order], vals[order]


def tile_ranges(sorted_keys: np.ndarray, n_tiles: int) -> np.ndarray:
    """[n_tiles, 2] half-open ranges of each tile in the sorted pair list."""
    tid = (sorted_keys >> np.uint64(32)).astype(np.int64)
    starts = np.searchsorted(tid, np.arange(n_tiles), side="left")
    ends = np.searchsorted(tid, np.arange(n_tiles), side="right")
    return np.stack([starts, ends], 1)
