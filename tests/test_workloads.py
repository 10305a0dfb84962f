"""Seeded generators are deterministic and have the documented shapes."""
import numpy as np

import workloads as W

# SHA-256 of the generated Gaussian arrays (seeded numpy default_rng / PCG64)
DIGEST0 = "19cbe4ff6ab6d5ad50a4418c09f14dd5bbfd1c3172975fc0e3afbc9c13d52fea"
DIGEST1 = "ba9b1f8c22e68f18672953aef0f1e0e7d9028a4f60945ffe5bafd2cea6af5d67"


def test_config0_shapes_and_ranges():
    s = W.config0()
    g = s.gaussians
    assert g.n == 4096 and s.poses.shape == (16, 3, 4) and s.query_noise.shape == (3, 96, 128)
    assert all(a.dtype == np.float32 for a in g.arrays())
    assert g.means[:, 0].min() >= -10 and g.means[:, 2].max() <= 5
    assert np.all(g.scales > 0) and np.all((g.opacity > 0) & (g.opacity < 1))
    # poses are rigid: R R^T = I
    r = s.poses[:, :, :3].astype(np.float64)
    assert np.abs(np.einsum("pij,pkj->pik", r, r) - np.eye(3)).max() < 1e-6


def test_config1_shapes():
    s = W.config1()
    g = s.gaussians
    assert g.n == 1_000_000 and s.poses.shape == (64, 3, 4)
    assert s.camera == W.Camera(1408, 376, 552.0, 552.0, 704.0, 188.0)
    ground = g.means[:600_000]
    assert abs(float(ground[:, 2].std()) - 0.05) < 0.002
    fac = g.means[600_000:]
    assert np.all(np.abs(np.abs(fac[:, 1]) - 8) < 0.5)


def test_generators_are_deterministic():
    a = W.config0()
    b = W.config0()
    assert W.digest(*a.gaussians.arrays(), a.poses, a.hidden_pose, a.query_noise) == \
        W.digest(*b.gaussians.arrays(), b.poses, b.hidden_pose, b.query_noise)
    assert W.digest(*a.gaussians.arrays()) == DIGEST0

    assert W.digest(*W.config1().gaussians.arrays()) == DIGEST1


def test_autotune_buckets_and_variants():
    from paper_2403_11367_amd import autotune
    assert [autotune.size_bucket(n) for n in (1, 2, 3, 175195, 262144, 262145, 956309)] == \
        [1, 2, 4, 262144, 262144, 524288, 1048576]
    v = autotune.variants()
    assert len(v) == len(autotune.TILES) * len(autotune.CHUNKS) * len(autotune.BLOCKS_PER_CU) * len(autotune.POSE_GROUPS)
    assert {(x["tile_w"], x["tile_h"]) for x in v} == {(16, 16), (32, 8), (8, 32)}
