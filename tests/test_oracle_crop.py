"""Pins for the oracle's voxel-grid radius crop (Sec. III-B2, Sec. III-C1)."""
import numpy as np
from scipy.spatial import cKDTree

import workloads as W
from oracle import crop


def test_matches_scipy_kdtree_over_cell_centres():
    rng = np.random.default_rng(0)
    means = rng.uniform([-50, -30, 0], [150, 30, 5], size=(20000, 3)).astype(np.float32)
    for (cx, cy, r, cell) in [(10, 0, 25, 10), (100, -5, 50, 10), (0, 0, 7.5, 2.5)]:
        got = crop.crop_indices(means, cell, (cx, cy), r, voxel=0.0)
        ids = np.floor(means[:, :2].astype(np.float64) / cell).astype(np.int64)
        cells, inv = np.unique(ids, axis=0, return_inverse=True)
        centres = (cells + 0.5) * cell
        keep_cells = cKDTree(centres).query_ball_point([cx, cy], r + 1e-9)
        ref = np.nonzero(np.isin(inv.ravel(), keep_cells))[0]
        assert np.array_equal(got, ref)
        assert np.all(np.diff(got) > 0)


def test_hand_example():
    means = np.array([[5, 5, 0], [15, 5, 0], [26, 1, 0], [5, -3, 0], [-1, 2, 0]], np.float32)
    # cells (0,0) (1,0) (2,0) (0,-1) (-1,0); centres (5,5) (15,5) (25,5) (5,-5) (-5,5)
    # prior (5, 0), radius 10: distances 5, 11.18, 20.6, 5, 11.18
    assert crop.crop_indices(means, 10.0, (5.0, 0.0), 10.0, voxel=0.0).tolist() == [0, 3]


def test_config1_crop_size():
    sc = W.config1()
    idx = crop.crop_indices(sc.gaussians.means, sc.crop_cell, sc.prior_center[:2], sc.crop_radius,
                            sc.crop_voxel)
    # 10 m cells with centres within 50 m of (100, 0): x cells 50..150 on both sides of y = 0
    m = sc.gaussians.means[idx].astype(np.float64)
    assert m[:, 0].min() >= 50 and m[:, 0].max() < 150
    assert idx.size == 500143


def test_voxel_order_hand_example():
    """Morton order of 1 m voxels, x bit first: (0,0,0) < (1,0,0) < (0,1,0) < (1,1,0)
    < (0,0,1) < (1,0,1) < (2,0,0); ties (same voxel) by ascending index."""
    v = np.array([[2, 0, 0], [0, 0, 1], [1, 1, 0], [0, 1, 0], [1, 0, 0], [0, 0, 0], [1, 0, 1],
                  [0, 0, 0]], np.float64)
    means = (v + 0.25).astype(np.float32)
    got = crop.crop_indices(means, 10.0, (0.0, 0.0), 100.0, voxel=1.0).tolist()
    assert got == [5, 7, 4, 3, 2, 1, 6, 0]
    # negative coordinates sort below positive ones along each axis (offset 2^20)
    m2 = np.array([[0.5, 0.5, 0.5], [-0.5, 0.5, 0.5]], np.float32)
    assert crop.crop_indices(m2, 10.0, (0.0, 0.0), 100.0, voxel=1.0).tolist() == [1, 0]


def test_voxel_order_is_a_permutation_of_the_selection():
    sc = W.config1(n=200_000)
    a = crop.crop_indices(sc.gaussians.means, 10.0, (100.0, 0.0), 50.0, voxel=1.0)
    b = crop.crop_indices(sc.gaussians.means, 10.0, (100.0, 0.0), 50.0, voxel=0.0)
    assert np.array_equal(np.sort(a), b) and not np.array_equal(a, b)
