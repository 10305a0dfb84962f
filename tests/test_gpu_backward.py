"""GPU render backward (gsr_render_backward) against float64 central differences
of the oracle renderer (oracle/render64.py).

The loss is a linear functional of the images, L = sum(w_rgb rgb) + sum(w_depth
depth) with seeded random weights, so its gradient with respect to the images is
(w_rgb, w_depth). Parameters are those of a map-training step: means, log-scales,
raw quaternions, opacity logits, colours; the GPU's linear-scale and opacity
gradients are chained through exp and the sigmoid here.

Bar, per parameter: |g - fd| <= 1e-3 |fd| + 512 u (1 + cond) S, with u = 2^-24,
S the sum over pixels of the magnitudes of the parameter's per-pixel central
differences and cond = a c / det of the Gaussian's screen covariance (largest
over the poses). The second term is what a float32 evaluation can lose where the
per-pixel terms cancel (|fd| much smaller than S): each term carries a relative
error of some hundred u (recomputed transmittance, the colour behind a layer
taken as a difference of sums, hardware exp2), growing with cond through the
float32 conic, and the terms are summed in float32. Measured on MI355X the
largest error is 260 u S (config 0 and oblique disks); where there is no
cancellation the first term governs. Only parameters whose central-difference
stencil is stable are checked (no change of any pixel's contributing list, no
decision within a float32 margin of its threshold).
"""
import numpy as np
import pytest

import workloads as W
from helpers import camera, say, to_dev
from oracle import render64 as R

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _bar(fd, scale, cond):
    return 1e-3 * np.abs(fd) + 512.0 * U32 * (1.0 + cond) * scale


def _check_rows(rows, label, min_stable=0.5):
    """rows[name] = [(fd, gpu, stable, scale, cond)]: every stable one within the
    bar; at least min_stable of each group stable. Returns the stable count."""
    n = 0
    for name in GROUPS:
        if not rows[name]:
            continue
        arr = np.array(rows[name], dtype=float)
        st = arr[:, 2] > 0
        assert st.mean() >= min_stable, f"{label} {name}: too few stable parameters ({st.sum()}/{len(arr)})"
        a = arr[st]
        err = np.abs(a[:, 1] - a[:, 0])
        tol = _bar(a[:, 0], a[:, 3], a[:, 4])
        rel = err / np.maximum(np.abs(a[:, 0]), 1e-300)
        say(f"  {label} {name}: {len(a)} stable of {len(arr)}, max rel error {rel.max():.2e}, max err / (u S) "
            f"{np.max(err / (U32 * np.maximum(a[:, 3], 1e-300))):.0f}, worst err/bar {np.max(err / tol):.3f}")
        bad = np.nonzero(err > tol)[0]
        assert bad.size == 0, f"{label} {name}: {a[bad[:3]]}"
        n += len(a)
    return n


def _fd_rows(p, poses, cam, w_rgb, w_depth, gpu, gaussians, rows=None):
    from oracle import render64 as R_
    rows = rows if rows is not None else {k: [] for k in GROUPS}
    conds = {}
    for gi in gaussians:
        gi = int(gi)
        conds[gi] = max(float(R_.project(p, ps, cam).cond[gi]) for ps in poses)
        for k, name in enumerate(GROUPS):
            for comp in range(WIDTH[name]):
                fd, stable, scale = R_.fd_gradient(p, poses, cam, w_rgb, w_depth, gi, k, comp, STEPS[name],
                                                   with_scale=True)
                got = gpu[name][gi] if gpu[name].ndim == 1 else gpu[name][gi, comp]
                rows[name].append((fd, got, stable, scale, conds[gi]))
    return rows

GROUPS = ["means", "log_scales", "quats", "logits", "rgb"]
STEPS = {"means": 1e-5, "log_scales": 1e-6, "quats": 1e-6, "logits": 1e-6, "rgb": 1e-6}
WIDTH = {"means": 3, "log_scales": 3, "quats": 4, "logits": 1, "rgb": 3}


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2403_11367_amd import Context
    assert torch.cuda.is_available()
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _gpu_grads(ctx, g, poses, cam, w_rgb, w_depth, cfg=None):
    import torch
    arrs = [to_dev(a.astype(np.float32)) for a in g.arrays()]
    sm = ctx.load_submap(*arrs)
    pt = to_dev(poses.astype(np.float32))
    rgb, depth = ctx.render(sm, camera(cam), pt, cfg)
    grads = ctx.render_backward(sm, arrs[1], arrs[2], pt, rgb, depth, to_dev(w_rgb.astype(np.float32)),
                                to_dev(w_depth.astype(np.float32)))
    torch.cuda.synchronize()
    out = [t.cpu().numpy().astype(np.float64) for t in grads]
    sm.free()
    return out


def test_backward_matches_central_differences_config0(ctx):
    sc = W.config0()
    cam = sc.camera
    poses = sc.poses[[0, 9]]
    rng = np.random.default_rng(77)
    w_rgb = rng.normal(size=(2, 3, cam.height, cam.width)).astype(np.float32).astype(np.float64)
    w_depth = (0.1 * rng.normal(size=(2, cam.height, cam.width))).astype(np.float32).astype(np.float64)
    say("render backward: config0, 2 poses, 30 sampled Gaussians x 14 parameters vs float64 central differences")
    gm, gs, gq, go, gc = _gpu_grads(ctx, sc.gaussians, poses, cam, w_rgb, w_depth)
    p = R.as_params(sc.gaussians)
    s = np.exp(p.log_scales)
    o = 1.0 / (1.0 + np.exp(-p.logits))
    gpu = {"means": gm, "log_scales": gs * s, "quats": gq, "logits": go * o * (1 - o), "rgb": gc}
    # Gaussians with some footprint in the first pose
    scr = R.project(p, poses[0], cam)
    area = (scr.rect[:, 1] - scr.rect[:, 0]) * (scr.rect[:, 3] - scr.rect[:, 2])
    inside = scr.visible & (scr.rect[:, 1] > 0) & (scr.rect[:, 0] < cam.width) & (scr.rect[:, 3] > 0) & \
        (scr.rect[:, 2] < cam.height) & (area > 4.0)
    pick = rng.choice(np.nonzero(inside)[0], 30, replace=False)
    rows = _fd_rows(p, poses, cam, w_rgb, w_depth, gpu, pick)
    assert _check_rows(rows, "config0") >= 200


@pytest.mark.parametrize("tw,th", [(32, 8), (8, 32)])
def test_backward_other_tile_shapes(ctx, tw, th):
    """The backward walks the forward's tiles: with 32x8 and 8x32 tiles, config 0
    (2 poses, 12 sampled Gaussians) against float64 central differences."""
    from paper_2403_11367_amd import default_cfg
    sc = W.config0()
    cam = sc.camera
    poses = sc.poses[[0, 9]]
    rng = np.random.default_rng(177)
    w_rgb = rng.normal(size=(2, 3, cam.height, cam.width)).astype(np.float32).astype(np.float64)
    w_depth = (0.1 * rng.normal(size=(2, cam.height, cam.width))).astype(np.float32).astype(np.float64)
    say(f"render backward: config0 with {tw}x{th} tiles, 12 sampled Gaussians")
    gm, gs, gq, go, gc = _gpu_grads(ctx, sc.gaussians, poses, cam, w_rgb, w_depth, default_cfg(tile_w=tw, tile_h=th))
    p = R.as_params(sc.gaussians)
    s = np.exp(p.log_scales)
    o = 1.0 / (1.0 + np.exp(-p.logits))
    gpu = {"means": gm, "log_scales": gs * s, "quats": gq, "logits": go * o * (1 - o), "rgb": gc}
    scr = R.project(p, poses[0], cam)
    area = (scr.rect[:, 1] - scr.rect[:, 0]) * (scr.rect[:, 3] - scr.rect[:, 2])
    inside = scr.visible & (scr.rect[:, 1] > 0) & (scr.rect[:, 0] < cam.width) & (scr.rect[:, 3] > 0) & \
        (scr.rect[:, 2] < cam.height) & (area > 4.0)
    rows = _fd_rows(p, poses, cam, w_rgb, w_depth, gpu, rng.choice(np.nonzero(inside)[0], 12, replace=False))
    assert _check_rows(rows, f"{tw}x{th}") >= 80


def test_backward_oblique_thin_disks(ctx):
    """Map-training layout: flat disks (in-plane log-scale N(-2.5, 0.4), normal
    N(-4, 0.3)) on the ground and two facades of a 30 m corridor, seen from 1.5 m
    above the ground along it (ground disks at grazing angles: thin, elongated
    footprints), 2 poses at 160x64."""
    g = W.corridor_map(6000, seed=3, length=30.0)
    cam = W.Camera(160, 64, 70.0, 70.0, 80.0, 32.0)
    poses = np.stack([W.pose_from_center(np.array([1.0, 0.5, 1.5]), W.AXES_ALONG_X, 0.0),
                      W.pose_from_center(np.array([2.0, -0.5, 1.4]), W.AXES_ALONG_X, np.deg2rad(4.0))]
                     ).astype(np.float32)
    rng = np.random.default_rng(78)
    w_rgb = rng.normal(size=(2, 3, cam.height, cam.width)).astype(np.float32).astype(np.float64)
    w_depth = (0.1 * rng.normal(size=(2, cam.height, cam.width))).astype(np.float32).astype(np.float64)
    say("render backward: oblique thin disks (corridor layout), 2 poses, 30 sampled Gaussians")
    gm, gs, gq, go, gc = _gpu_grads(ctx, g, poses, cam, w_rgb, w_depth)
    p = R.as_params(g)
    s = np.exp(p.log_scales)
    o = 1.0 / (1.0 + np.exp(-p.logits))
    gpu = {"means": gm, "log_scales": gs * s, "quats": gq, "logits": go * o * (1 - o), "rgb": gc}
    scr = R.project(p, poses[0], cam)
    area = (scr.rect[:, 1] - scr.rect[:, 0]) * (scr.rect[:, 3] - scr.rect[:, 2])
    inside = scr.visible & (scr.rect[:, 1] > 0) & (scr.rect[:, 0] < cam.width) & (scr.rect[:, 3] > 0) & \
        (scr.rect[:, 2] < cam.height) & (area > 4.0)
    # footprints: elongated (eigenvalue ratio of the screen covariance)
    det_c = scr.conic[:, 0] * scr.conic[:, 2] - scr.conic[:, 1] ** 2
    cov = np.stack([scr.conic[:, 2], -scr.conic[:, 1], scr.conic[:, 0]], 1) / det_c[:, None]
    tr, dt = cov[:, 0] + cov[:, 2], cov[:, 0] * cov[:, 2] - cov[:, 1] ** 2
    disc = np.sqrt(np.maximum(tr * tr / 4 - dt, 0))
    ratio = (tr / 2 + disc) / np.maximum(tr / 2 - disc, 1e-30)
    cand = np.nonzero(inside)[0]
    say(f"  {cand.size} footprints in view; eigenvalue ratio median {np.median(ratio[cand]):.1f}, 90% "
        f"{np.percentile(ratio[cand], 90):.1f}; a c / det max {scr.cond[cand].max():.2f}")
    # half the sample among the most elongated footprints
    elong = cand[np.argsort(-ratio[cand])][:200]
    pick = np.concatenate([rng.choice(elong, 15, replace=False),
                           rng.choice(np.setdiff1d(cand, elong), 15, replace=False)])
    rows = _fd_rows(p, poses, cam, w_rgb, w_depth, gpu, pick)
    assert _check_rows(rows, "oblique disks") >= 200


def test_backward_is_independent_of_pose_groups(ctx):
    """The same gradients (to float-atomic rounding) when the render ran in 2 pose groups."""
    from paper_2403_11367_amd import default_cfg
    sc = W.config0()
    poses = sc.poses[:4]
    rng = np.random.default_rng(5)
    w_rgb = rng.normal(size=(4, 3, sc.camera.height, sc.camera.width))
    w_depth = rng.normal(size=(4, sc.camera.height, sc.camera.width))
    say("render backward: 1 vs 2 pose groups")
    a = _gpu_grads(ctx, sc.gaussians, poses, sc.camera, w_rgb, w_depth)
    b = _gpu_grads(ctx, sc.gaussians, poses, sc.camera, w_rgb, w_depth, default_cfg(pose_groups=2))
    for x, y in zip(a, b):
        assert np.allclose(x, y, rtol=1e-4, atol=1e-5 * np.abs(x).max())


def test_backward_argument_checks(ctx):
    import torch
    from paper_2403_11367_amd import GsrError
    sc = W.config0()
    arrs = [to_dev(a.astype(np.float32)) for a in sc.gaussians.arrays()]
    sm = ctx.load_submap(*arrs)
    other = ctx.load_submap(*arrs)
    pt = to_dev(sc.poses[:2].astype(np.float32))
    rgb, depth = ctx.render(sm, camera(sc.camera), pt)
    g = torch.zeros_like(rgb), torch.zeros_like(depth)
    with pytest.raises(GsrError, match="EINVAL"):  # not the submap of the last render
        ctx.render_backward(other, arrs[1], arrs[2], pt, rgb, depth, *g)
    idx = to_dev(np.arange(100, dtype=np.int64))
    sub = ctx.load_submap(*arrs, index=idx)
    with pytest.raises(GsrError, match="EINVAL"):  # loaded with an index
        ctx.render_backward(sub, arrs[1][:100].contiguous(), arrs[2][:100].contiguous(), pt, rgb, depth, *g)
    torch.cuda.synchronize()
    for s in (sm, other, sub):
        s.free()


def test_backward_with_alpha_and_jacobian_clamps(ctx):
    """Gaussians whose alpha is clamped at alpha_max near their centre (opacity
    0.999) and a large one whose mean lies outside the Jacobian's clamp (1.3 x the
    half field of view) but whose footprint reaches into the image: the clamped
    branches of the backward against central differences."""
    say("render backward: alpha clamp and Jacobian clamp, 64x48")
    rng = np.random.default_rng(21)
    cam = W.Camera(64, 48, 40.0, 40.0, 32.0, 24.0)
    pose = W.pose_from_center(np.zeros(3), W.AXES_ALONG_Y)  # camera at the origin looking along +y
    # Gaussian 0 projects onto the centre of pixel (32, 24), where its alpha is clamped
    means = [[0.0625, 5.0, -0.0625], [0.8, 6.0, 0.3], [-5.5, 5.0, 0.2], [5.6, 5.2, -0.4]]
    scales = [[0.25, 0.2, 0.3], [0.2, 0.3, 0.25], [1.5, 1.2, 1.4], [1.3, 1.6, 1.1]]
    opac = [0.999, 0.995, 0.7, 0.6]
    g = W.Gaussians(np.array(means, np.float32), np.array(scales, np.float32),
                    rng.normal(size=(4, 4)).astype(np.float32), np.array(opac, np.float32),
                    rng.uniform(0, 1, (4, 3)).astype(np.float32))
    p = R.as_params(g)
    scr = R.project(p, pose, cam)
    lim = R.JAC_CLAMP * 0.5 * cam.width / cam.fx
    xt = (scr.u - cam.cx) / cam.fx
    assert abs(xt[2]) > lim and abs(xt[3]) > lim and scr.visible[2] and scr.visible[3]
    assert abs(scr.u[0] - 32.5) < 1e-9 and abs(scr.v[0] - 24.5) < 1e-9 and scr.opacity[0] > R.ALPHA_MAX
    poses = pose[None].astype(np.float32)
    w_rgb = rng.normal(size=(1, 3, cam.height, cam.width))
    w_depth = 0.1 * rng.normal(size=(1, cam.height, cam.width))
    gm, gs, gq, go, gc = _gpu_grads(ctx, g, poses, cam, w_rgb, w_depth)
    s = np.exp(p.log_scales)
    o = 1.0 / (1.0 + np.exp(-p.logits))
    gpu = {"means": gm, "log_scales": gs * s, "quats": gq, "logits": go * o * (1 - o), "rgb": gc}
    rows = _fd_rows(p, poses, cam, w_rgb, w_depth, gpu, range(4))
    n_checked = _check_rows(rows, "clamps", min_stable=0.0)
    say(f"  {n_checked} stable parameters checked")
    assert n_checked >= 30


def _stacked_scene(n, seed):
    """n small, faint, anisotropic Gaussians stacked over the two tiles at the centre
    of a 64x48 image: tile lists of about 0.6 n records, whose pixels never reach
    t_min."""
    rng = np.random.default_rng(seed)
    y = rng.uniform(3.0, 30.0, n)
    x = rng.uniform(-0.02, 0.02, n) * y
    z = rng.uniform(-0.02, 0.02, n) * y
    scales = 0.002 * y[:, None] * rng.uniform(0.6, 1.2, (n, 3))
    g = W.Gaussians(np.stack([x, y, z], 1).astype(np.float32), scales.astype(np.float32),
                    rng.normal(size=(n, 4)).astype(np.float32), np.full(n, 0.015, np.float32),
                    rng.uniform(0, 1, (n, 3)).astype(np.float32))
    cam = W.Camera(64, 48, 400.0, 400.0, 32.0, 24.0)
    poses = W.yaw_grid_poses(np.zeros(3), W.AXES_ALONG_Y, [0.0], [0.0], [0.0]).astype(np.float32)
    return g, cam, poses


def test_backward_splits_long_lists_at_kept_states(ctx):
    """Tile lists of about 5000 records: with GSR_RENDER_KEEP_STATE the forward keeps
    each pixel's state at records 2016 and 4032 (images unchanged, bit for bit) and
    the backward walks the list as three segments. Its gradients equal those of the
    one serial walk (to float-atomic rounding) and, for Gaussians in the later
    segments, float64 central differences."""
    import torch
    from paper_2403_11367_amd import default_cfg
    from paper_2403_11367_amd.gsr import RENDER_KEEP_STATE
    g, cam, poses = _stacked_scene(8000, 9)
    p = R.as_params(g)
    scr = R.project(p, poses[0], cam)
    rng = np.random.default_rng(3)
    w_rgb = rng.normal(size=(1, 3, cam.height, cam.width))
    w_depth = 0.1 * rng.normal(size=(1, cam.height, cam.width))
    say("render backward: tile lists of about 5000 records, kept states vs one serial walk")
    arrs = [to_dev(a.astype(np.float32)) for a in g.arrays()]
    sm = ctx.load_submap(*arrs)
    pt = to_dev(poses)
    res = []
    for cfg in (None, default_cfg(flags=RENDER_KEEP_STATE)):
        rgb, depth = ctx.render(sm, camera(cam), pt, cfg)
        grads = ctx.render_backward(sm, arrs[1], arrs[2], pt, rgb, depth, to_dev(w_rgb.astype(np.float32)),
                                    to_dev(w_depth.astype(np.float32)))
        torch.cuda.synchronize()
        res.append(([rgb.cpu().numpy(), depth.cpu().numpy()], [t.cpu().numpy().astype(np.float64) for t in grads]))
    from paper_2403_11367_amd import BUF_OFFSETS
    offs = ctx.debug_buffer(BUF_OFFSETS)
    longest = int(np.max(np.diff(offs.astype(np.int64))))
    say(f"  longest list {longest}")
    assert longest > 2 * 2016
    for a, b in zip(res[0][0], res[1][0]):
        assert np.array_equal(a, b)
    for a, b in zip(res[0][1], res[1][1]):
        assert np.allclose(a, b, rtol=1e-4, atol=1e-5 * np.abs(a).max())
    gm, gs, gq, go, gc = res[1][1]
    s = np.exp(p.log_scales)
    o = 1.0 / (1.0 + np.exp(-p.logits))
    gpu = {"means": gm, "log_scales": gs * s, "quats": gq, "logits": go * o * (1 - o), "rgb": gc}
    # the farther half by depth: about 2400 or more records into their tiles' lists
    vis = np.nonzero(scr.visible)[0]
    deep = vis[np.argsort(scr.z[vis], kind="stable")][4000:]
    rows = _fd_rows(p, poses, cam, w_rgb, w_depth, gpu, rng.choice(deep, 24, replace=False))
    n_checked = _check_rows(rows, "long lists", min_stable=0.0)
    assert n_checked >= 100
    sm.free()


def test_keep_state_rejects_count_evals_and_other_chunks(ctx):
    """Kept states are taken at 2016-record boundaries of the 252-record chunk walk
    without evaluation counting: other combinations are refused."""
    from paper_2403_11367_amd import GsrError, default_cfg
    from paper_2403_11367_amd.gsr import RENDER_COUNT_EVALS, RENDER_KEEP_STATE
    sc = W.config0()
    arrs = [to_dev(a.astype(np.float32)) for a in sc.gaussians.arrays()]
    sm = ctx.load_submap(*arrs)
    pt = to_dev(sc.poses[:2].astype(np.float32))
    for cfg in (default_cfg(flags=RENDER_KEEP_STATE | RENDER_COUNT_EVALS),
                default_cfg(flags=RENDER_KEEP_STATE, blend_chunk=124)):
        with pytest.raises(GsrError, match="EUNSUPPORTED"):
            ctx.render(sm, camera(sc.camera), pt, cfg)
    sm.free()
