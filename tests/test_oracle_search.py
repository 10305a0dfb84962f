"""Pins of the search oracle (Sec. III-C1 and the random-order early stop of Sec. IV)."""
import numpy as np
import pytest

import workloads as W
from oracle import search


def test_argmax_and_topk_ties_go_to_lowest_index():
    s = np.array([0.2, 0.9, 0.5, 0.9, -1.0])
    assert search.argmax(s) == 1
    assert list(search.topk(s, 3)) == [1, 3, 2]


def test_early_stop_without_stop_is_the_argmax():
    rng = np.random.default_rng(5)
    s = rng.uniform(-1, 1, 37)
    order = rng.permutation(37)
    best, score, n = search.early_stop_search(s, order, batch=5, max_eval=37, threshold=np.inf)
    assert (best, n) == (search.argmax(s), 37) and score == s.max()


def test_early_stop_hand_example():
    # order visits 3, 0, 4 | 1, 2 ; the threshold 0.8 is first reached by candidate 1 (0.85)
    s = [0.10, 0.85, 0.95, 0.30, 0.20]
    assert search.early_stop_search(s, [3, 0, 4, 1, 2], batch=3, max_eval=5, threshold=0.8) == (2, 0.95, 5)
    # a batch of 2 stops after the batch holding candidate 1: 3, 0 | 4, 1
    assert search.early_stop_search(s, [3, 0, 4, 1, 2], batch=2, max_eval=5, threshold=0.8) == (1, 0.85, 4)
    # the scored share caps the search: only 3 and 0 are scored
    assert search.early_stop_search(s, [3, 0, 4, 1, 2], batch=2, max_eval=2, threshold=0.8) == (3, 0.30, 2)


@pytest.mark.parametrize("seed", range(6))
def test_early_stop_matches_closed_form(seed):
    """Brute force against the definition: the search ends with the batch that holds
    the first candidate (in visiting order) whose score reaches the threshold."""
    rng = np.random.default_rng(seed)
    P = int(rng.integers(1, 60))
    s = np.round(rng.uniform(0, 1, P), 2)  # ties on purpose
    order = rng.permutation(P)
    batch = int(rng.integers(1, 9))
    max_eval = int(rng.integers(1, P + 1))
    thr = float(rng.uniform(0.5, 1.1))
    best, score, n = search.early_stop_search(s, order, batch, max_eval, thr)
    hit = [k for k in range(max_eval) if s[order[k]] >= thr]
    n_ref = min(max_eval, (hit[0] // batch + 1) * batch) if hit else max_eval
    seen = order[:n_ref]
    best_ref = min(c for c in seen if s[c] == s[seen].max())
    assert (best, n) == (best_ref, n_ref) and score == s[best_ref]


# Sec. IV, Fig. 2: NCC between the query and renders around the true pose
# peaks at the true pose and falls off with the x and yaw error.
FIG2_DX = [-2.0, -1.0, -0.5, -0.25, 0.0, 0.25, 0.5, 1.0, 2.0]       # metres
FIG2_DYAW = [-10.0, -6.0, -3.0, -1.5, 0.0, 1.5, 3.0, 6.0, 10.0]     # degrees


def fig2_sweeps(scene):
    """(x sweep poses, yaw sweep poses) through the hidden pose."""
    hx, hy, hyaw = scene.hidden_offset
    xs = W.offset_poses(scene, [(hx + d, hy, hyaw) for d in FIG2_DX])
    ys = W.offset_poses(scene, [(hx, hy, hyaw + d) for d in FIG2_DYAW])
    return xs, ys


def check_fig2_profile(scores, offsets):
    """The peak is at offset 0, clear of its neighbours; within +-3 steps of the
    peak the scores fall strictly with |offset|; all others stay below the peak."""
    s = np.asarray(scores, np.float64)
    c = offsets.index(0.0)
    assert int(np.argmax(s)) == c, s
    assert s[c] - max(s[c - 1], s[c + 1]) > 0.05, s
    for k in range(1, 4):
        assert s[c - k] < s[c - k + 1] and s[c + k] < s[c + k - 1], s
    assert np.all(np.delete(s, c) < s[c])


def test_fig2_ncc_peaks_at_the_true_pose_config0():
    from oracle import ncc as oncc
    sc = W.config0()
    prep = search.prepare(sc.gaussians)
    query = search.render_pose(prep, sc.hidden_pose, sc.camera).rgb + sc.query_noise
    xs, ys = fig2_sweeps(sc)
    for poses, offs in ((xs, FIG2_DX), (ys, FIG2_DYAW)):
        s = oncc.ncc(query, np.stack([search.render_pose(prep, p, sc.camera).rgb for p in poses]))
        check_fig2_profile(s, offs)
