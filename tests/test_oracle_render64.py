"""Pins of the float64 gradient-check renderer: its images equal the float32
pipeline's oracle (pinned elsewhere by closed forms and brute force) to float32
accuracy, and its central differences reproduce closed-form gradients of a
single Gaussian."""
import numpy as np

import workloads as W
from oracle import render64 as R
from oracle import search


def test_images_match_the_float32_oracle_on_config0():
    sc = W.config0()
    p = R.as_params(sc.gaussians)
    pr = search.prepare(sc.gaussians)
    ref = search.render_pose(pr, sc.poses[5], sc.camera)
    rng = np.random.default_rng(0)
    pix = np.stack([rng.integers(0, sc.camera.width, 300), rng.integers(0, sc.camera.height, 300)], 1)
    rgb, dep, _, marg = R.render(p, sc.poses[5], sc.camera, pixels=pix)
    ok = ~marg & ~ref.flag[pix[:, 1], pix[:, 0]]
    assert ok.sum() > 250
    assert np.abs(rgb[ok] - ref.rgb[:, pix[ok, 1], pix[ok, 0]].T).max() < 2e-4
    assert np.abs(dep[ok] - ref.depth[pix[ok, 1], pix[ok, 0]]).max() < 2e-3


def _one_gaussian(logit=0.0, scale=-1.0):
    g = W.Gaussians(means=np.array([[0.2, 5.0, -0.1]], np.float32), scales=np.full((1, 3), np.exp(scale), np.float32),
                    quats=np.array([[0.9, 0.1, -0.3, 0.2]], np.float32),
                    opacity=np.array([1 / (1 + np.exp(-logit))], np.float32), rgb=np.array([[0.3, 0.6, 0.9]], np.float32))
    cam = W.Camera(48, 40, 40.0, 40.0, 24.0, 20.0)
    pose = W.pose_from_center(np.zeros(3), W.AXES_ALONG_Y)
    return R.as_params(g), cam, pose


def test_single_gaussian_colour_and_logit_gradients_closed_form():
    p, cam, pose = _one_gaussian(logit=-0.5)
    rng = np.random.default_rng(3)
    w_rgb = rng.normal(size=(1, 3, cam.height, cam.width))
    w_d = rng.normal(size=(1, cam.height, cam.width))
    scr = R.project(p, pose, cam)
    i, j = np.meshgrid(np.arange(cam.width) + 0.5, np.arange(cam.height) + 0.5, indexing="xy")
    dx, dy = i - scr.u[0], j - scr.v[0]
    A, B, C = scr.conic[0]
    d2 = A * dx * dx + 2 * B * dx * dy + C * dy * dy
    a = scr.opacity[0] * np.exp(-0.5 * d2)
    take = (d2 <= R.CUTOFF) & (a >= R.ALPHA_MIN)
    assert take.sum() > 20 and a.max() < R.ALPHA_MAX
    alpha = np.where(take, a, 0.0)
    for c in range(3):  # dL/dc = sum w alpha (T = 1 in front of the only Gaussian)
        g, stable = R.fd_gradient(p, [pose], cam, w_rgb, w_d, 0, 4, c, 1e-6)
        assert stable and abs(g - (w_rgb[0, c] * alpha).sum()) < 1e-7 * max(1, abs(g))
    # dL/dlogit = sum (w . c + w_d z) alpha (1 - o)
    closed = ((np.tensordot(scr.rgb[0], w_rgb[0], 1) + w_d[0] * scr.z[0]) * alpha * (1 - scr.opacity[0])).sum()
    g, stable = R.fd_gradient(p, [pose], cam, w_rgb, w_d, 0, 3, 0, 1e-6)
    assert stable and abs(g - closed) < 1e-6 * max(1, abs(closed))


def test_stencil_that_changes_the_contributing_set_is_unstable():
    p, cam, pose = _one_gaussian(logit=-0.5)
    rng = np.random.default_rng(4)
    w_rgb = rng.normal(size=(1, 3, cam.height, cam.width))
    w_d = rng.normal(size=(1, cam.height, cam.width))
    # a large step moves the support across pixel centres
    _, stable = R.fd_gradient(p, [pose], cam, w_rgb, w_d, 0, 0, 0, 0.05)
    assert not stable
