"""Pins for the oracle's covariance and projection (Sec. III-A, Eq. 3-4).

Each check compares the oracle with something other than itself: a library
rotation routine, eigenvalues, finite differences of the projection, closed
forms for special cases, and a hand-derived worked example.
"""
import json
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import workloads as W
from oracle import gaussians, project

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_quats(n, seed):
    return np.random.default_rng(seed).normal(size=(n, 4)).astype(np.float32)


def test_rotation_orthonormal_det1():
    q = _rand_quats(500, 1)
    r = gaussians.quat_to_rot(gaussians.normalise_quat(q)).astype(np.float64)
    eye = np.einsum("nij,nkj->nik", r, r)
    assert np.abs(eye - np.eye(3)).max() < 2e-6
    assert np.abs(np.linalg.det(r) - 1.0).max() < 2e-6


def test_rotation_matches_scipy():
    q = _rand_quats(300, 2)
    r = gaussians.quat_to_rot(gaussians.normalise_quat(q)).astype(np.float64)
    # scipy takes scalar-last (x, y, z, w)
    ref = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], 1).astype(np.float64)).as_matrix()
    assert np.abs(r - ref).max() < 2e-6


def test_rotation_about_z_closed_form():
    th = np.linspace(-3, 3, 13)
    q = np.stack([np.cos(th / 2), 0 * th, 0 * th, np.sin(th / 2)], 1).astype(np.float32)
    r = gaussians.quat_to_rot(gaussians.normalise_quat(q)).astype(np.float64)
    for k, t in enumerate(th):
        ref = np.array([[np.cos(t), -np.sin(t), 0], [np.sin(t), np.cos(t), 0], [0, 0, 1]])
        assert np.abs(r[k] - ref).max() < 1e-6


def test_quaternion_scale_invariance():
    q = _rand_quats(100, 3)
    r1 = gaussians.quat_to_rot(gaussians.normalise_quat(q))
    r2 = gaussians.quat_to_rot(gaussians.normalise_quat(np.float32(3.7) * q))
    assert np.abs(r1.astype(np.float64) - r2).max() < 2e-6


def test_covariance_eigenvalues_are_squared_scales():
    rng = np.random.default_rng(4)
    s = np.exp(rng.normal(-1.0, 0.5, size=(300, 3))).astype(np.float32)
    q = _rand_quats(300, 5)
    c = gaussians.full_cov(gaussians.covariance(s, q)).astype(np.float64)
    ev = np.linalg.eigvalsh(c)
    ref = np.sort(s.astype(np.float64) ** 2, axis=1)
    assert np.abs(ev - ref).max() / ref.max() < 1e-5


def _proj64(pt, pose, fx, fy, cx, cy):
    t = pose[:, :3] @ pt + pose[:, 3]
    return np.array([fx * t[0] / t[2] + cx, fy * t[1] / t[2] + cy])


def test_covariance_matches_library_rotation():
    """Sigma = R diag(s^2) R^T with R from scipy (fp64 matmul), not R^T diag(s^2) R."""
    rng = np.random.default_rng(8)
    s = np.exp(rng.normal(-1.0, 0.5, size=(200, 3))).astype(np.float32)
    q = _rand_quats(200, 9)
    got = gaussians.full_cov(gaussians.covariance(s, q)).astype(np.float64)
    R = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], 1).astype(np.float64)).as_matrix()
    ref = np.einsum("nij,nj,nkj->nik", R, s.astype(np.float64) ** 2, R)
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-5


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_screen_cov_matches_finite_difference_jacobian(seed):
    """Sigma2D = J_w Sigma J_w^T + eps I with J_w = d m / d mu (Eq. 4, world coordinates)
    taken by central differences in fp64, for anisotropic rotated Gaussians and a
    rotated pose."""
    sc = W.config0()
    cam = sc.camera
    pose = sc.poses[5 + seed].astype(np.float64)
    rng = np.random.default_rng(seed)
    n = 40
    # points in front of the camera, inside the field of view (clamp inactive)
    depth = rng.uniform(3, 20, n)
    xs = rng.uniform(-0.5, 0.5, n) * depth
    ys = rng.uniform(-0.4, 0.4, n) * depth
    cam_pts = np.stack([xs, ys, depth], 1)
    world = ((cam_pts - pose[:, 3]) @ pose[:, :3]).astype(np.float32)  # R^T (p - t)
    scales = np.exp(rng.normal(-2.0, 0.5, size=(n, 3))).astype(np.float32)
    cov6 = gaussians.covariance(scales, _rand_quats(n, 20 + seed))
    cov = gaussians.full_cov(cov6).astype(np.float64)
    p32 = pose.astype(np.float32)
    rec = project.preprocess(world, cov6, np.full(n, 0.5, np.float32), np.zeros((n, 3), np.float32),
                             p32, cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)
    assert rec.visible.all()
    p64 = p32.astype(np.float64)
    h = 1e-5
    for k in range(n):
        pt = world[k].astype(np.float64)
        J = np.zeros((2, 3))
        for d in range(3):
            e = np.zeros(3)
            e[d] = h
            J[:, d] = (_proj64(pt + e, p64, cam.fx, cam.fy, cam.cx, cam.cy)
                       - _proj64(pt - e, p64, cam.fx, cam.fy, cam.cx, cam.cy)) / (2 * h)
        ref = J @ cov[k] @ J.T + 0.3 * np.eye(2)
        got = np.array([[rec.cov2d[k, 0], rec.cov2d[k, 1]], [rec.cov2d[k, 1], rec.cov2d[k, 2]]], np.float64)
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
        uv = _proj64(pt, p64, cam.fx, cam.fy, cam.cx, cam.cy)
        assert abs(rec.u[k] - uv[0]) < 1e-3 and abs(rec.v[k] - uv[1]) < 1e-3


def test_axis_aligned_on_axis_closed_form():
    pose = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float32)
    rng = np.random.default_rng(7)
    for _ in range(20):
        z = rng.uniform(1, 30)
        sx, sy, sz = rng.uniform(0.05, 0.5, 3)
        cov6 = np.array([[sx * sx, 0, 0, sy * sy, 0, sz * sz]], np.float32)
        rec = project.preprocess(np.array([[0, 0, z]], np.float32), cov6, np.array([0.5], np.float32),
                                 np.zeros((1, 3), np.float32), pose, 200, 100, 150.0, 160.0, 100.0, 50.0)
        a_ref = (150.0 * np.float32(sx * sx) ** 0.5 / np.float32(z)) ** 2 + 0.3
        c_ref = (160.0 * np.float32(sy * sy) ** 0.5 / np.float32(z)) ** 2 + 0.3
        assert rec.visible[0]
        assert abs(rec.cov2d[0, 0] - a_ref) < 1e-5 * a_ref
        assert abs(rec.cov2d[0, 2] - c_ref) < 1e-5 * c_ref
        assert rec.cov2d[0, 1] == 0.0
        assert rec.u[0] == 100.0 and rec.v[0] == 50.0


def test_golden_single_gaussian_geometry():
    gd = json.load(open(os.path.join(GOLDEN, "single_gaussian_onaxis.json")))
    c = gd["camera"]
    g = gd["gaussian"]
    cov6 = gaussians.covariance(np.array([g["scale"]], np.float32), np.array([g["quat_wxyz"]], np.float32))
    rec = project.preprocess(np.array([g["mean"]], np.float32), cov6, np.array([g["opacity"]], np.float32),
                             np.array([g["rgb"]], np.float32), np.array(gd["pose"], np.float32),
                             c["width"], c["height"], c["fx"], c["fy"], c["cx"], c["cy"])
    e = gd["expect"]
    assert rec.visible[0]
    np.testing.assert_allclose(rec.cov2d[0], e["cov2d_abc"], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(rec.conic[0], e["conic"], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose([rec.rx[0], rec.ry[0]], [e["rx"], e["ry"]], rtol=1e-6)
    assert [rec.u[0], rec.v[0]] == e["uv"] and rec.z[0] == e["z"]
    assert rec.rect[0].tolist() == e["rect"]
    assert rec.tile_rect[0].tolist() == e["tile_rect"]


def test_conic_is_inverse_and_rect_is_pixel_bbox_of_ellipse():
    sc = W.config0()
    cam = sc.camera
    mu = sc.gaussians.means
    cov6 = gaussians.covariance(sc.gaussians.scales, sc.gaussians.quats)
    rec = project.preprocess(mu, cov6, sc.gaussians.opacity, sc.gaussians.rgb, sc.poses[3],
                             cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)
    vis = np.nonzero(rec.visible)[0]
    assert vis.size > 1000
    a, b, c = [rec.cov2d[vis, k].astype(np.float64) for k in range(3)]
    A, B, C = [rec.conic[vis, k].astype(np.float64) for k in range(3)]
    assert np.abs(A * a + B * b - 1).max() < 1e-5
    assert np.abs(A * b + B * c).max() < 1e-5 * np.maximum(1, np.abs(B * c)).max()
    # brute force over pixels: every pixel centre with d^2 <= 9 (a hair inside) is in the rect
    ii, jj = np.meshgrid(np.arange(cam.width) + 0.5, np.arange(cam.height) + 0.5, indexing="xy")
    for g in vis[:300]:
        dx = ii - rec.u[g]
        dy = jj - rec.v[g]
        d2 = rec.conic[g, 0] * dx * dx + 2 * rec.conic[g, 1] * dx * dy + rec.conic[g, 2] * dy * dy
        inside = d2 <= 9.0 - 1e-4
        js, is_ = np.nonzero(inside)
        i0, i1, j0, j1 = rec.rect[g]
        assert ((is_ >= i0) & (is_ <= i1) & (js >= j0) & (js <= j1)).all()
        # and the rect is the pixel range of |x - u| <= rx, |y - v| <= ry
        for (lo, hi, c, r, n_) in ((i0, i1, rec.u[g], rec.rx[g], cam.width), (j0, j1, rec.v[g], rec.ry[g], cam.height)):
            dist = np.abs(np.arange(n_) + 0.5 - np.float64(c)) - np.float64(r)
            if np.abs(dist).min() < 1e-4:
                continue  # a pixel centre sits on the box edge: float rounding decides
            cols = np.nonzero(dist <= 0)[0]
            assert cols.min() == lo and cols.max() == hi


def test_culling_rules():
    pose = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float32)
    mu = np.array([[0, 0, 0.19], [0, 0, 0.2], [0, 0, 0.21], [np.nan, 0, 5], [100, 0, 5],
                   [0, 0, -5], [0, 0, 5]], np.float32)
    n = mu.shape[0]
    cov6 = np.tile(np.array([[0.01, 0, 0, 0.01, 0, 0.01]], np.float32), (n, 1))
    rec = project.preprocess(mu, cov6, np.full(n, 0.5, np.float32), np.zeros((n, 3), np.float32), pose,
                             64, 48, 50.0, 50.0, 32.0, 24.0)
    # near plane: strictly greater than 0.2; NaN culled; far off-screen culled; behind culled
    assert rec.visible.tolist() == [False, False, True, False, False, False, True]


def test_non_finite_parameters_are_culled_and_counted():
    # the same on-axis Gaussian 7 times, then one non-finite entry in each of
    # opacity, a colour channel, a covariance entry and the mean (the first copy
    # stays clean)
    pose = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float32)
    n = 7
    mu = np.tile(np.array([[0.0, 0.0, 5.0]], np.float32), (n, 1))
    cov6 = np.tile(np.array([[0.01, 0, 0, 0.01, 0, 0.01]], np.float32), (n, 1))
    op = np.full(n, 0.5, np.float32)
    rgb = np.full((n, 3), 0.5, np.float32)
    op[1], op[2] = np.nan, np.inf
    rgb[3, 1] = -np.inf
    cov6[4, 3] = np.inf
    mu[5, 0] = np.nan
    rgb[6, 2] = np.nan
    bad = project.nonfinite(mu, cov6, op, rgb)
    assert bad.tolist() == [False] + [True] * 6
    rec = project.preprocess(mu, cov6, op, rgb, pose, 64, 48, 50.0, 50.0, 32.0, 24.0)
    assert rec.visible.tolist() == [True] + [False] * 6


def test_jacobian_clamp_outside_fov():
    """A Gaussian far to the side: J uses x/z clamped to 1.3 * (W/2)/fx, u does not."""
    pose = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float32)
    z = np.float32(4.0)
    x = np.float32(20.0)  # x/z = 5, far beyond 1.3 * 32/50 = 0.832
    s2 = np.float32(0.25)
    cov6 = np.array([[s2, 0, 0, s2, 0, s2]], np.float32)
    rec = project.preprocess(np.array([[x, 0, z]], np.float32), cov6, np.array([0.5], np.float32),
                             np.zeros((1, 3), np.float32), pose, 64, 48, 50.0, 50.0, 32.0, 24.0)
    lim = 1.3 * 32 / 50
    J = np.array([[50 / 4.0, 0, -50 * lim / 4.0], [0, 50 / 4.0, 0]])
    ref = 0.25 * J @ J.T + 0.3 * np.eye(2)
    assert abs(rec.cov2d[0, 0] - ref[0, 0]) < 1e-4 * ref[0, 0]
    assert abs(rec.u[0] - (50 * 5 + 32)) < 1e-4
    assert not rec.visible[0]  # its 3-sigma box misses the 64-pixel-wide image
