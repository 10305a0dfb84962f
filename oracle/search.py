"""Brute-force candidate search (oracle; test infrastructure only).

Sec. III-C1: render the submap at every candidate pose, score each render
against the query with NCC (Eq. 10) and keep the most similar. Ties go to the
lowest candidate index. ``render_pose`` chains the other oracle modules for
one pose: covariance, projection (Eq. 3-4), keys and sort, compositing
(Eq. 1, 2, 5).

``early_stop_search`` is the random-order variant of Sec. IV (initial
relocalisation): candidates are scored in a given random order, in batches,
and the search stops after the first batch whose best score reaches the
threshold, or once a fixed share of the candidates has been scored. Reading:
the paper's stop test on NCC is garbled ("dropped below" for a similarity);
it is read as "the best NCC so far reaches the threshold". Its second test,
on feature matches of a later stage, is outside this path.
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


def early_stop_search(scores, order, batch: int, max_eval: int, threshold: float):
    """Score candidates order[0], order[1], ... in batches of ``batch``; stop after
    the first batch whose best score is >= threshold, or once ``max_eval``
    candidates are scored. Returns (best candidate, its score, number scored);
    ties go to the lowest candidate index among those scored."""
    scores = np.asarray(scores, dtype=np.float64)
    order = [int(i) for i in order]
    best, best_score, n = -1, -np.inf, 0
    while n < max_eval:
        for c in order[n:min(n + batch, max_eval)]:
            if scores[c] > best_score or (scores[c] == best_score and c < best):
                best, best_score = c, scores[c]
        n = min(n + batch, max_eval)
        if best_score >= threshold:
            break
    return best, float(best_score), n
