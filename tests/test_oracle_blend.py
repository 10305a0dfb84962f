"""Pins for the oracle's compositing (Eq. 1, Eq. 2 read as o*exp(-d^2/2), Eq. 5).

Closed forms (one layer, two layers, a geometric stack with its termination
index), a hand-derived worked example, tiled == brute force on tiny scenes,
tile-shape invariance and the telescoping identities C = 1 - T (all colours 1)
and D = z0 (1 - T) (all depths z0).
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import blend, gaussians, keys, project, search

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _records(u, v, conic, z, op, rgb, rect):
    n = len(u)
    f = np.float32
    return project.ScreenRecords(
        visible=np.ones(n, bool), u=np.array(u, f), v=np.array(v, f), z=np.array(z, f),
        conic=np.array(conic, f), cov2d=np.zeros((n, 3), f), rx=np.zeros(n, f), ry=np.zeros(n, f),
        rect=np.array(rect, np.int64), tile_rect=np.array(rect, np.int64) // 16,
        opacity=np.array(op, f), rgb=np.array(rgb, f))


def _render(rec, width, height, tw=16, th=16):
    k, v = keys.make_pairs_fast(rec, width, height, tw, th)
    ks, vs = keys.sort_pairs(k, v)
    tx, ty = keys.tile_grid(width, height, tw, th)
    return blend.render_tiled(rec, vs, keys.tile_ranges(ks, tx * ty), width, height, tw, th)


def test_golden_single_gaussian_pixels():
    gd = json.load(open(os.path.join(GOLDEN, "single_gaussian_onaxis.json")))
    c = gd["camera"]
    g = gd["gaussian"]
    s = W.Scene("g", W.Gaussians(np.array([g["mean"]], np.float32), np.array([g["scale"]], np.float32),
                                 np.array([g["quat_wxyz"]], np.float32), np.array([g["opacity"]], np.float32),
                                 np.array([g["rgb"]], np.float32)),
                W.Camera(c["width"], c["height"], c["fx"], c["fy"], c["cx"], c["cy"]), (16, 16),
                np.array([gd["pose"]], np.float32), None, None, None)
    out = search.render_pose(search.prepare(s.gaussians), s.poses[0], s.camera)
    for px in gd["expect"]["pixels"]:
        i, j = px["ij"]
        np.testing.assert_allclose(out.rgb[:, j, i], px["rgb"], rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose(out.depth[j, i], px["depth"], rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose(out.t_final[j, i], 1.0 - px["alpha"], rtol=1e-6, atol=1e-9)
    # nothing outside the 3-sigma rectangle
    e = gd["expect"]["rect"]
    mask = np.zeros((c["height"], c["width"]), bool)
    mask[e[2]:e[3] + 1, e[0]:e[1] + 1] = True
    assert np.all(out.rgb[:, ~mask] == 0) and np.all(out.depth[~mask] == 0)


def test_two_layers_closed_form_depth_not_index_order():
    # index 0 is farther than index 1: compositing must follow depth, not index
    conic = [[0.05, 0.01, 0.08], [0.2, -0.03, 0.1]]
    rec = _records(u=[20.3, 22.1], v=[14.2, 15.7], conic=conic, z=[9.0, 4.0], op=[0.8, 0.6],
                   rgb=[[0.9, 0.1, 0.3], [0.2, 0.7, 0.5]], rect=[[0, 47, 0, 31], [0, 47, 0, 31]])
    out = _render(rec, 48, 32)
    for (i, j) in [(20, 14), (22, 16), (25, 12), (10, 20), (30, 30)]:
        x, y = i + 0.5, j + 0.5
        al = []
        for k in range(2):
            A, B, C = (float(t) for t in rec.conic[k])
            dx, dy = x - float(rec.u[k]), y - float(rec.v[k])
            d2 = A * dx * dx + 2 * B * dx * dy + C * dy * dy
            a = min(0.99, float(rec.opacity[k]) * np.exp(-0.5 * d2))
            al.append(a if (d2 <= 9 and a >= float(np.float32(1 / 255))) else 0.0)
        near, far = 1, 0
        ref_c = rec.rgb[near] * al[near] + rec.rgb[far] * al[far] * (1 - al[near])
        ref_d = 4.0 * al[near] + 9.0 * al[far] * (1 - al[near])
        np.testing.assert_allclose(out.rgb[:, j, i], ref_c, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(out.depth[j, i], ref_d, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(out.t_final[j, i], (1 - al[0]) * (1 - al[1]), rtol=1e-12)


@pytest.mark.parametrize("op", [0.3, 0.6, 0.9, 0.995])
def test_geometric_stack_and_termination_index(op):
    """n identical layers: C = c (1 - (1-a)^m), m = min(n, first m with (1-a)^m < 1e-4)."""
    n = 40
    rec = _records(u=[8.5] * n, v=[8.5] * n, conic=[[0.1, 0.0, 0.1]] * n,
                   z=list(np.linspace(2.0, 30.0, n)), op=[op] * n, rgb=[[0.25, 0.5, 1.0]] * n,
                   rect=[[0, 15, 0, 15]] * n)
    out = _render(rec, 16, 16)
    a = min(0.99, float(np.float32(op)))  # pixel (8, 8) sits on the mean: d^2 = 0
    m = n
    for k in range(1, n + 1):
        if (1 - a) ** k < 1e-4:
            m = k
            break
    ref = np.array([0.25, 0.5, 1.0], np.float32).astype(np.float64) * (1 - (1 - a) ** m)
    np.testing.assert_allclose(out.rgb[:, 8, 8], ref, rtol=1e-12)
    assert out.n_contrib[8, 8] == m
    z = np.linspace(2.0, 30.0, n).astype(np.float32).astype(np.float64)
    ref_d = sum(z[k] * a * (1 - a) ** k for k in range(m))
    np.testing.assert_allclose(out.depth[8, 8], ref_d, rtol=1e-12)


def test_alpha_floor_and_clamp():
    # opacity below 1/255 never contributes; opacity 1 at the mean clamps to 0.99
    rec = _records(u=[4.5, 12.5], v=[8.5, 8.5], conic=[[0.5, 0, 0.5]] * 2, z=[3.0, 3.0],
                   op=[0.003, 1.0], rgb=[[1, 1, 1]] * 2, rect=[[0, 15, 0, 15]] * 2)
    out = _render(rec, 16, 16)
    assert np.all(out.rgb[:, 8, 4] == 0)
    np.testing.assert_allclose(out.rgb[:, 8, 12], 0.99, rtol=1e-12)


def _scene_render_pair(seed, n, tile):
    sc = W.tiny_scene(seed, n=n, width=64, height=48)
    cam = sc.camera
    cov6 = gaussians.covariance(sc.gaussians.scales, sc.gaussians.quats)
    rec = project.preprocess(sc.gaussians.means, cov6, sc.gaussians.opacity, sc.gaussians.rgb,
                             sc.poses[0], cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                             tile[0], tile[1])
    return rec, _render(rec, cam.width, cam.height, *tile), blend.render_bruteforce(rec, cam.width, cam.height)


@pytest.mark.parametrize("seed,n", [(10, 40), (11, 128), (12, 256)])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_tiled_equals_bruteforce(seed, n, tile):
    rec, tiled, brute = _scene_render_pair(seed, n, tile)
    ok = ~(tiled.flag | brute.flag)
    assert ok.mean() > 0.99
    assert np.abs(tiled.rgb - brute.rgb)[:, ok].max() < 1e-12
    assert np.abs(tiled.depth - brute.depth)[ok].max() < 1e-10
    assert np.abs(tiled.t_final - brute.t_final)[ok].max() < 1e-12
    assert tiled.rgb.max() > 0.1


def test_tile_shape_invariance():
    outs = [_scene_render_pair(13, 200, t)[1] for t in [(16, 16), (8, 8), (32, 8), (16, 4)]]
    ok = ~np.any([o.flag for o in outs], axis=0)
    for o in outs[1:]:
        assert np.abs(o.rgb - outs[0].rgb)[:, ok].max() < 1e-12
        assert np.abs(o.depth - outs[0].depth)[ok].max() < 1e-10


def test_telescoping_identities():
    sc = W.tiny_scene(14, n=300, width=64, height=48, opacity_logit_mean=2.0)
    cam = sc.camera
    g = sc.gaussians
    cov6 = gaussians.covariance(g.scales, g.quats)
    ones = np.ones_like(g.rgb)
    rec = project.preprocess(g.means, cov6, g.opacity, ones, sc.poses[0], cam.width, cam.height,
                             cam.fx, cam.fy, cam.cx, cam.cy)
    out = _render(rec, cam.width, cam.height)
    for c in range(3):
        np.testing.assert_allclose(out.rgb[c], 1.0 - out.t_final, atol=1e-12)
    # constant depth: D = z0 (1 - T)
    rec.z[:] = np.float32(7.25)
    out2 = _render(rec, cam.width, cam.height)
    np.testing.assert_allclose(out2.depth, 7.25 * (1.0 - out2.t_final), atol=1e-11)
    assert (out.t_final < 1e-4).mean() > 0.05  # some pixels terminated early
    assert np.all(out.t_final <= 1.0) and np.all(out.t_final >= 0.0)


def test_transparent_scene_is_empty():
    sc = W.tiny_scene(15, n=100)
    g = sc.gaussians
    cam = sc.camera
    cov6 = gaussians.covariance(g.scales, g.quats)
    rec = project.preprocess(g.means, cov6, np.full(g.n, 0.0035, np.float32), g.rgb, sc.poses[0],
                             cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)
    out = _render(rec, cam.width, cam.height)
    assert np.all(out.rgb == 0) and np.all(out.depth == 0) and np.all(out.t_final == 1)


def test_empty_list_and_ragged_image():
    # 37 x 21 image: ragged tiles on both axes, no Gaussians at all
    rec = _records(u=[], v=[], conic=np.zeros((0, 3)), z=[], op=[], rgb=np.zeros((0, 3)),
                   rect=np.zeros((0, 4)))
    out = _render(rec, 37, 21)
    assert out.rgb.shape == (3, 21, 37) and np.all(out.rgb == 0) and np.all(out.t_final == 1)


def test_render_pixels_matches_full_render():
    sc = W.config0()
    prep = search.prepare(sc.gaussians)
    out, rec, ks, vs, rng = search.render_pose(prep, sc.poses[2], sc.camera, with_pairs=True)
    r = np.random.default_rng(0)
    pi = r.integers(0, sc.camera.width, 200)
    pj = r.integers(0, sc.camera.height, 200)
    rgb, dep, tf, fl = blend.render_pixels(rec, vs, rng, sc.camera.width, pi, pj)
    np.testing.assert_allclose(rgb, out.rgb[:, pj, pi], atol=1e-12)
    np.testing.assert_allclose(dep, out.depth[pj, pi], atol=1e-10)
    assert np.array_equal(fl, out.flag[pj, pi])


# ---- margin flag and outcomes: decisions within float32 error of a threshold ----

def _one_pixel(rec, w=16, h=16, tile=(16, 16)):
    return _render(rec, w, h, *tile)


def test_flag_cutoff_both_sides():
    # one Gaussian, pixel (8, 8) at dx = 3 from the mean, isotropic conic a: d^2 = 9 a
    base = dict(u=[5.5], v=[8.5], z=[2.0], op=[0.9], rgb=[[1.0, 0.5, 0.25]], rect=[[0, 15, 0, 15]])
    d2, p, m_cut, _ = blend._exponent_margins(np.array(3.0), np.array(0.0), 1.0, 0.0, 1.0, 0.9, 16, 16)
    margin_d2 = float(m_cut) / blend.S2
    assert 1e-6 < margin_d2 < 1e-4          # float32 error of d^2 near 9 at this geometry
    for a, flagged, inside in ((1.0 + 0.2 * margin_d2 / 9, True, False), (1.0 - 0.2 * margin_d2 / 9, True, True),
                               (1.0 + 3.0 * margin_d2 / 9, False, False), (1.0 - 3.0 * margin_d2 / 9, False, True)):
        rec = _records(conic=[[a, 0.0, a]], **base)
        out = _one_pixel(rec)
        assert bool(out.flag[8, 8]) == flagged, a
        expect_in = float(np.float32(0.9)) * np.exp(-0.5 * 9.0 * float(np.float32(a)))
        assert (out.t_final[8, 8] < 1.0) == inside
        outs = blend.outcomes(out, 8, 8)
        got = sorted(float(x) for x in outs[:, 4])
        if flagged:   # both decisions, with their closed-form results
            np.testing.assert_allclose(got, [1.0 - expect_in, 1.0], rtol=1e-12)
            np.testing.assert_allclose(sorted(outs[:, 0]), [0.0, expect_in], rtol=1e-12)
        else:
            assert len(got) == 1
        # pixels away from the threshold are never flagged
        assert not out.flag[8, 5] and not out.flag[3, 12]


def test_flag_alpha_floor_both_sides():
    amin = blend.ALPHA_MIN
    for rel, flagged in ((1e-6, True), (-1e-6, True), (3e-5, False), (-3e-5, False)):
        o = np.float32(amin * (1.0 + rel))
        rec = _records(u=[8.5], v=[8.5], conic=[[0.5, 0.0, 0.5]], z=[2.0], op=[o], rgb=[[1.0, 1.0, 1.0]],
                       rect=[[0, 15, 0, 15]])
        out = _one_pixel(rec)
        assert bool(out.flag[8, 8]) == flagged, rel
        takes = float(o) >= amin
        assert (out.rgb[0, 8, 8] > 0) == takes
        outs = blend.outcomes(out, 8, 8)
        if flagged:
            np.testing.assert_allclose(sorted(outs[:, 0]), [0.0, float(o)], rtol=1e-12)
        else:
            assert outs.shape[0] == 1


def test_flag_termination_both_sides():
    # three equal layers take T to 1e-4 (1 + rel); a fourth (blue) lies behind
    for rel, flagged in ((1e-6, True), (-1e-6, True), (3e-3, False), (-3e-3, False)):
        a = np.float32(1.0 - (1e-4 * (1.0 + rel)) ** (1.0 / 3.0))
        t3 = (1.0 - float(a)) ** 3
        rec = _records(u=[8.5] * 4, v=[8.5] * 4, conic=[[0.5, 0.0, 0.5]] * 4, z=[1.0, 2.0, 3.0, 4.0],
                       op=[a, a, a, 0.5], rgb=[[1.0, 0.0, 0.0]] * 3 + [[0.0, 0.0, 1.0]], rect=[[0, 15, 0, 15]] * 4)
        out = _one_pixel(rec)
        assert bool(out.flag[8, 8]) == flagged, rel
        stops = t3 < blend.T_MIN
        assert (out.rgb[2, 8, 8] == 0.0) == stops
        outs = blend.outcomes(out, 8, 8)
        blues = sorted(float(x) for x in outs[:, 2])
        if flagged:  # stop after the third layer, or take the fourth too
            np.testing.assert_allclose(blues, [0.0, 0.5 * t3], rtol=1e-12)
        else:
            assert len(blues) == 1


def _fma32(a, b, c):
    return np.float32(np.float64(a) * np.float64(b) + np.float64(c))


def test_margin_bounds_a_float32_evaluation():
    """The exponent margins bound the error of the float32 evaluation they
    describe: sum of squares of factors from a 1-ulp reciprocal square root and
    square root, expanded about the tile centre, with fused adds; on random
    geometry up to condition number 1e4, pixels of the tile, centres within the
    3-sigma reach."""
    r = np.random.default_rng(7)
    f = np.float32
    s = f(np.sqrt(f(0.5) * f(1.4426950408889634)))
    cut_p2 = f(f(-0.5) * f(1.4426950408889634) * f(9.0))
    worst = 0.0
    for _ in range(4000):
        sig = np.exp(r.uniform(np.log(0.3), np.log(60.0)))
        cond = np.exp(r.uniform(0.0, np.log(1e4)))
        th = r.uniform(0, np.pi)
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        cov = R @ np.diag([sig ** 2, sig ** 2 / cond]) @ R.T + 0.3 * np.eye(2)
        inv = np.linalg.inv(cov)
        A, B, C = f(inv[0, 0]), f(inv[0, 1]), f(inv[1, 1])
        o = f(r.uniform(0.01, 0.99))
        xc, yc = f(r.integers(0, 80) * 16 + 8), f(r.integers(0, 20) * 16 + 8)
        x, y = f(r.integers(0, 16) - 7.5), f(r.integers(0, 16) - 7.5)
        reach = 3.0 * np.sqrt(np.diag(cov)) + 1.0
        u = f(xc + x + r.uniform(-reach[0], reach[0]))
        v = f(yc + y + r.uniform(-reach[1], reach[1]))
        ulp = lambda t: np.spacing(np.float32(t))
        rr = f(f(1.0 / np.sqrt(np.float64(A))) + r.integers(-1, 2) * ulp(1.0 / np.sqrt(A)))
        m11, m12 = f(A * rr), f(B * rr)
        det = f(np.float64(A) * np.float64(C) - np.float64(B) * np.float64(B))
        sq = f(f(np.sqrt(np.float64(max(det, 0)))) + r.integers(-1, 2) * ulp(np.sqrt(max(det, 0))))
        m22 = f(sq * rr)
        a11, a12, a22 = f(m11 * s), f(m12 * s), f(m22 * s)
        lo = f(f(np.log2(np.float64(o))) + r.integers(-1, 2) * ulp(np.log2(o)))
        uc, vc = f(u - xc), f(v - yc)
        k1 = -_fma32(a11, uc, f(a12 * vc))
        k2 = -f(a22 * vc)
        t1 = _fma32(a11, x, _fma32(a12, y, k1))
        t2 = _fma32(a22, y, k2)
        p2 = _fma32(-t2, t2, _fma32(-t1, t1, lo))
        thr = f(cut_p2 + lo)
        dx, dy = np.float64(xc + x) - np.float64(u), np.float64(yc + y) - np.float64(v)
        d2, p, m_cut, m_amin = blend._exponent_margins(dx, dy, np.float64(A), np.float64(B), np.float64(C),
                                                       np.float64(o), 16, 16)
        err_cut = abs((np.float64(p2) - np.float64(thr)) - blend.S2 * (9.0 - d2))
        err_amin = abs((np.float64(p2) - np.float64(np.float32(np.log2(np.float32(1 / 255))))) -
                       (p - blend.LOG2_AMIN))
        assert err_cut <= m_cut and err_amin <= m_amin, (err_cut, m_cut, err_amin, m_amin)
        worst = max(worst, err_cut / m_cut, err_amin / m_amin)
    assert worst > 0.01  # the bound is not vacuous


def test_outcomes_hold_the_result_and_unflagged_are_unique():
    sc = W.config0()
    prep = search.prepare(sc.gaussians)
    n_flag = 0
    for p in (0, 5, 10, 15):
        out = search.render_pose(prep, sc.poses[p], sc.camera)
        res = np.concatenate([out.rgb, out.depth[None], out.t_final[None]])
        for j, i in np.argwhere(out.flag):
            o = blend.outcomes(out, int(i), int(j))
            assert np.abs(o - res[:, j, i]).max(axis=1).min() < 1e-12
            n_flag += 1
        r = np.random.default_rng(p)
        for j, i in zip(r.integers(0, 96, 300), r.integers(0, 128, 300)):
            if not out.flag[j, i]:
                o = blend.outcomes(out, int(i), int(j))
                assert o.shape[0] == 1
                np.testing.assert_allclose(o[0], res[:, j, i], rtol=1e-12, atol=1e-15)
    assert n_flag > 0


@pytest.mark.parametrize("seed,n", [(10, 40), (12, 256)])
def test_tiled_and_bruteforce_within_each_others_outcomes(seed, n):
    rec, tiled, brute = _scene_render_pair(seed, n, (16, 16))
    for a, b in ((tiled, brute), (brute, tiled)):
        for j, i in np.argwhere(b.flag & ~a.flag):
            o = blend.outcomes(b, int(i), int(j))
            res = np.array([*a.rgb[:, j, i], a.depth[j, i], a.t_final[j, i]])
            assert np.abs(o - res).max(axis=1).min() < 1e-10
