"""Submap retrieval around a prior pose (oracle; test infrastructure only).

Sec. III-B2 and Sec. III-C1: the map is stored in a 2D voxel grid, each cell
keyed by its integer coordinates; cells whose centre lies within a radius of
the prior camera position (in x, y) are retrieved, with all their Gaussians.
The paper answers the radius query with a KD-tree over cell centres; the plain
definition of that query is the brute-force distance test below.

Cell of a Gaussian: (floor(x / cell), floor(y / cell)); centre ((ix + 0.5) cell,
(iy + 0.5) cell); kept iff (cx - px)^2 + (cy - py)^2 <= r^2. Float64.

Order of the returned submap (the submap index that breaks depth ties): the
map keeps its Gaussians by fine 3D voxel (Sec. IV uses 1 m voxels), so the
kept Gaussians are listed by the Morton code of their voxel
(v = floor(coord / voxel) + 2^20, clamped to [0, 2^21 - 1], x bit b -> code
bit 3b, y -> 3b + 1, z -> 3b + 2; a non-finite coordinate counts as 0), ties
by ascending map index. voxel <= 0 lists them by ascending map index.
"""
from __future__ import annotations

import numpy as np

_OFF = 1 << 20
_MAXV = (1 << 21) - 1


def cell_ids(means: np.ndarray, cell: float) -> np.ndarray:
    m = np.asarray(means, dtype=np.float64)
    return np.floor(m[:, :2] / cell).astype(np.int64)


def voxel_morton(means: np.ndarray, voxel: float) -> np.ndarray:
    """Morton code (uint64) of each Gaussian's 3D voxel, bit by bit."""
    m = np.asarray(means, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        f = np.floor(m / voxel) + _OFF
    v = np.where(np.isfinite(f), np.clip(f, 0, _MAXV), 0).astype(np.uint64)
    code = np.zeros(m.shape[0], dtype=np.uint64)
    for b in range(21):
        for a in range(3):
            bit = (v[:, a] >> np.uint64(b)) & np.uint64(1)
            code |= bit << np.uint64(3 * b + a)
    return code


def crop_indices(means: np.ndarray, cell: float, center_xy, radius: float, voxel: float = 1.0) -> np.ndarray:
    ids = cell_ids(means, cell)
    centre = (ids.astype(np.float64) + 0.5) * cell
    d2 = (centre[:, 0] - center_xy[0]) ** 2 + (centre[:, 1] - center_xy[1]) ** 2
    keep = np.nonzero(d2 <= radius * radius)[0].astype(np.int64)
    if voxel <= 0 or keep.size == 0:
        return keep
    code = voxel_morton(np.asarray(means)[keep], voxel)
    return keep[np.lexsort((keep, code))]
