"""Brute-force candidate search (oracle; test infrastructure only).

Sec. III-C1: render the submap at every candidate pose, score each render
against the query with NCC (Eq. 10) and keep the most similar. Ties go to the
lowest candidate index. ``render_pose`` chains the other oracle modules for
one pose: covariance, projection (Eq. 3-4), keys and sort, compositing
(Eq. 1, 2, 5).
"""
from __future__ import annotations

import numpy as np

from . import blend, gaussians, keys, project


def argmax(scores: np.ndarray) -> int:
    return int(np.argmax(np.asarray(scores)))  # first maximum = lowest index


def topk(scores: np.ndarray, k: int) -> np.ndarray:
    s = np.asarray(scores, dtype=np.float64)
    order = np.lexsort((np.arange(s.size), -s))
    return order[:k]


def prepare(g):
    """(means, cov6, opacity, rgb) of a Gaussians set, float32."""
    return (np.asarray(g.means, np.float32), gaussians.covariance(g.scales, g.quats),
            np.asarray(g.opacity, np.float32), np.asarray(g.rgb, np.float32))


def render_pose(prep, pose, cam, tile=(16, 16), with_pairs=False):
    mu, cov6, op, rgb = prep
    tw, th = tile
    rec = project.preprocess(mu, cov6, op, rgb, pose, cam.width, cam.height,
                             cam.fx, cam.fy, cam.cx, cam.cy, tw, th)
    k, v = keys.make_pairs_fast(rec, cam.width, cam.height, tw, th)
    ks, vs = keys.sort_pairs(k, v)
    tx, ty = keys.tile_grid(cam.width, cam.height, tw, th)
    rng = keys.tile_ranges(ks, tx * ty)
    out = blend.render_tiled(rec, vs, rng, cam.width, cam.height, tw, th)
    if with_pairs:
        return out, rec, ks, vs, rng
    return out
