"""Submap retrieval around a prior pose (oracle; test infrastructure only).

Sec. III-B2 and Sec. III-C1: the map is stored in a 2D voxel grid, each cell
keyed by its integer coordinates; cells whose centre lies within a radius of
the prior camera position (in x, y) are retrieved, with all their Gaussians.
The paper answers the radius query with a KD-tree over cell centres; the plain
definition of that query is the brute-force distance test below.

Cell of a Gaussian: (floor(x / cell), floor(y / cell)); centre ((ix + 0.5) cell,
(iy + 0.5) cell); kept iff (cx - px)^2 + (cy - py)^2 <= r^2. Float64. The
result lists the kept Gaussians' indices in ascending order.
"""
from __future__ import annotations

import numpy as np


def cell_ids(means: np.ndarray, cell: float) -> np.ndarray:
    m = np.asarray(means, dtype=np.float64)
    return np.floor(m[:, :2] / cell).astype(np.int64)


def crop_indices(means: np.ndarray, cell: float, center_xy, radius: float) -> np.ndarray:
    ids = cell_ids(means, cell)
    centre = (ids.astype(np.float64) + 0.5) * cell
    d2 = (centre[:, 0] - center_xy[0]) ** 2 + (centre[:, 1] - center_xy[1]) ** 2
    return np.nonzero(d2 <= radius * radius)[0].astype(np.int64)
