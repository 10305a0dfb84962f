"""Pins for the oracle's tile/depth keys and reference order (Sec. III-A)."""
import numpy as np

import workloads as W
from oracle import gaussians, keys, project


def _rec(scene, p):
    cam = scene.camera
    cov6 = gaussians.covariance(scene.gaussians.scales, scene.gaussians.quats)
    return project.preprocess(scene.gaussians.means, cov6, scene.gaussians.opacity,
                              scene.gaussians.rgb, scene.poses[p], cam.width, cam.height,
                              cam.fx, cam.fy, cam.cx, cam.cy, 16, 16)


def test_fast_pairs_equal_loop_pairs():
    sc = W.tiny_scene(3, n=200)
    rec = _rec(sc, 0)
    k1, v1 = keys.make_pairs(rec, sc.camera.width, sc.camera.height, 16, 16)
    k2, v2 = keys.make_pairs_fast(rec, sc.camera.width, sc.camera.height, 16, 16)
    assert k1.size > 100
    assert np.array_equal(k1, k2) and np.array_equal(v1, v2)


def test_key_bit_layout_and_order_against_python_sort():
    sc = W.tiny_scene(4, n=150)
    rec = _rec(sc, 1)
    k, v = keys.make_pairs(rec, sc.camera.width, sc.camera.height, 16, 16)
    ks, vs = keys.sort_pairs(k, v)
    tiles_x = (sc.camera.width + 15) // 16
    # brute force: python tuples (tile, depth as float, index)
    tup = []
    for g in np.nonzero(rec.visible)[0]:
        tx0, tx1, ty0, ty1 = rec.tile_rect[g]
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                tup.append((ty * tiles_x + tx, float(rec.z[g]), int(g)))
    tup.sort()
    assert [t[2] for t in tup] == vs.tolist()
    assert [t[0] for t in tup] == (ks >> np.uint64(32)).astype(np.int64).tolist()
    zb = (ks & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    assert np.array_equal(zb.astype(np.float64), np.array([t[1] for t in tup]))


def test_positive_float_bits_are_monotone():
    z = np.sort(np.random.default_rng(0).uniform(0.2, 500, 10000).astype(np.float32))
    assert np.all(np.diff(z.view(np.uint32).astype(np.int64)) >= 0)


def test_equal_depth_ties_break_by_index():
    keys_ = np.array([5, 5, 5, 3], np.uint64)
    vals = np.array([9, 2, 7, 4], np.uint32)
    ks, vs = keys.sort_pairs(keys_, vals)
    assert ks.tolist() == [3, 5, 5, 5] and vs.tolist() == [4, 2, 7, 9]


def test_ranges_cover_sorted_list():
    sc = W.config0()
    rec = _rec(sc, 0)
    k, v = keys.make_pairs_fast(rec, sc.camera.width, sc.camera.height, 16, 16)
    ks, vs = keys.sort_pairs(k, v)
    rng = keys.tile_ranges(ks, 8 * 6)
    assert rng[0, 0] == 0 and rng[-1, 1] == ks.size
    assert np.all(rng[1:, 0] == rng[:-1, 1])
    tid = (ks >> np.uint64(32)).astype(np.int64)
    for t in range(48):
        assert np.all(tid[rng[t, 0]:rng[t, 1]] == t)
    # counts per Gaussian add up to the pair total
    assert rec.n_tiles.sum() == ks.size
