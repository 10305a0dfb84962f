"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bars: screen records, tile counts, keys and per-tile order bit-exact;
renders within 1e-4 abs on every pixel, of the oracle's result or, where the
oracle flags a decision within float32 error of its threshold, of one of the
pixel's outcomes with those decisions taken either way; NCC within 1e-4.
"""
import numpy as np
import pytest

import workloads as W
from helpers import (TOL_NCC, check_pairs, check_records, compare_render, gpu_buffers, gpu_render, load,
                     oracle_pose, prep, say, to_dev)
from oracle import crop as ocrop
from oracle import ncc as oncc
from oracle import search

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2403_11367_amd import Context
    assert torch.cuda.is_available()
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _tiles(cam):
    return ((cam.width + 15) // 16) * ((cam.height + 15) // 16)


def test_config0_records_pairs_render(ctx):
    say("config0: 4096 Gaussians, 16 poses, 128x96")
    sc = W.config0()
    sm = load(ctx, sc.gaussians)
    rgb, dep, tf = gpu_render(ctx, sm, sc.camera, sc.poses)
    recs, nts, offs, pairs = gpu_buffers(ctx)
    pr = prep(sc.gaussians)
    T = _tiles(sc.camera)
    for p in range(sc.poses.shape[0]):
        out, rec, ks, vs, rng = oracle_pose(pr, sc.poses[p], sc.camera)
        check_records(recs, nts, rec, sc.gaussians.n, p)
        check_pairs(offs, pairs, ks, vs, rng, p, T)
        compare_render(rgb[p], dep[p], tf[p], out, f"pose {p}")


@pytest.mark.parametrize("seed,n,w,h", [(21, 300, 64, 48), (22, 500, 37, 21), (23, 64, 16, 16),
                                        (24, 1000, 200, 9), (25, 1, 33, 17)])
def test_tiny_scenes_ragged_sizes(ctx, seed, n, w, h):
    say(f"tiny scene seed {seed}: n {n}, {w}x{h}")
    sc = W.tiny_scene(seed, n=n, width=w, height=h, n_poses=3)
    sm = load(ctx, sc.gaussians)
    rgb, dep, tf = gpu_render(ctx, sm, sc.camera, sc.poses)
    recs, nts, offs, pairs = gpu_buffers(ctx)
    pr = prep(sc.gaussians)
    T = _tiles(sc.camera)
    for p in range(3):
        out, rec, ks, vs, rng = oracle_pose(pr, sc.poses[p], sc.camera)
        check_records(recs, nts, rec, n, p)
        check_pairs(offs, pairs, ks, vs, rng, p, T)
        compare_render(rgb[p], dep[p], tf[p], out, f"pose {p}")


def test_alpha_clamp_in_some_chunks(ctx):
    """Every 500th Gaussian at opacity 0.9995, so that alpha is clamped at alpha_max
    near those centres: about half of the 252-record chunks hold such a record and
    composite with the clamp, the others without it, and both must match the
    oracle."""
    say("alpha clamp mixed into some chunks: 3000 Gaussians, 64x48, 3 poses")
    sc = W.tiny_scene(71, n=3000, width=64, height=48, n_poses=3)
    g = sc.gaussians
    op = g.opacity.copy()
    op[::500] = np.float32(0.9995)
    g = W.Gaussians(g.means, g.scales, g.quats, op, g.rgb)
    sm = load(ctx, g)
    rgb, dep, tf = gpu_render(ctx, sm, sc.camera, sc.poses)
    recs, nts, offs, pairs = gpu_buffers(ctx)
    pr = prep(g)
    T = _tiles(sc.camera)
    n_clamped = 0
    for p in range(3):
        out, rec, ks, vs, rng = oracle_pose(pr, sc.poses[p], sc.camera)
        check_records(recs, nts, rec, g.n, p)
        check_pairs(offs, pairs, ks, vs, rng, p, T)
        compare_render(rgb[p], dep[p], tf[p], out, f"pose {p}")
        n_clamped += int((rec.opacity[rec.visible] > 0.99).sum())
    assert n_clamped > 0
    sm.free()


@pytest.mark.parametrize("n", [1 << 19, 600_000])
def test_depth_sort_either_side_of_value_packing(ctx, n):
    """Submaps of up to 2^19 Gaussians carry each visible Gaussian's tile count
    with its index in the depth sort's value; larger ones gather the counts in
    the sort's last pass. Either way the records and the sorted pairs match the
    oracle bit for bit."""
    from oracle import keys, project
    say(f"depth sort with {n} Gaussians (value packing {'on' if n <= 1 << 19 else 'off'}), 64x48, 1 pose")
    sc = W.tiny_scene(81, n=n, width=64, height=48, n_poses=1, log_scale_mean=-3.0)
    cam = sc.camera
    sm = load(ctx, sc.gaussians)
    gpu_render(ctx, sm, cam, sc.poses)
    recs, nts, offs, pairs = gpu_buffers(ctx)
    mu, cov6, op, rgb = prep(sc.gaussians)
    rec = project.preprocess(mu, cov6, op, rgb, sc.poses[0], cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)
    T = _tiles(cam)
    k, v = keys.make_pairs_fast(rec, cam.width, cam.height, 16, 16)
    ks, vs = keys.sort_pairs(k, v)
    rng = keys.tile_ranges(ks, T)
    check_records(recs, nts, rec, n, 0)
    check_pairs(offs, pairs, ks, vs, rng, 0, T)
    sm.free()


@pytest.mark.parametrize("z_near", [0.2, 0.0])
def test_depth_sort_far_depths_and_the_fourth_pass(ctx, z_near):
    """Depth keys are float32 depth bits minus the near plane's. Keys below 2^27
    sort in three 9-bit radix passes; a key of 2^27 or more (beyond about 13 km
    for a 0.2 m near plane, and every depth above 0.5 m for a near plane at 0)
    makes the sort run a fourth pass and leave its output in the other buffers.
    Depths up to 60 km, keys on either side of 2^27 and equal depths (ties in
    index order) give records and sorted pairs equal to the oracle's bit for bit.
    No depth here lies in (0, 0.2], so the oracle's 0.2 m near plane culls the
    same Gaussians as a near plane at 0."""
    from paper_2403_11367_amd import default_cfg
    say(f"depth sort with depths to 60 km, near plane {z_near}, 64x48, 3 poses")
    # 12,000 Gaussians: each pose's visible run spans several radix blocks of 4,096
    sc = W.tiny_scene(83, n=12_000, width=64, height=48, n_poses=3, depth_range=(0.5, 30.0))
    g = sc.gaussians
    rng = np.random.default_rng(84)
    means = g.means.astype(np.float64)
    target = means[:, 1].copy()
    far = rng.random(g.n) < 0.4
    target[far] = rng.uniform(13_000.0, 60_000.0, int(far.sum()))
    # depths whose keys (for a 0.2 m near plane) lie just below, at and above 2^27
    z0 = int(np.float32(0.2).view(np.uint32))
    edge = np.array([z0 + (1 << 27) - 2, z0 + (1 << 27) - 1, z0 + (1 << 27), z0 + (1 << 27) + 1],
                    np.uint32).view(np.float32)
    target[:4] = edge
    target[4:8] = edge  # equal depths: the lower index first
    means = (means / means[:, 1:2] * target[:, None]).astype(np.float32)
    means[:8, 1] = np.concatenate([edge, edge])
    means[8:16] = means[0:8]  # duplicated Gaussians: equal depths everywhere
    gg = W.Gaussians(means, g.scales, g.quats, g.opacity, g.rgb)
    sm = load(ctx, gg)
    cfg = default_cfg(z_near=z_near)
    rgb, dep, tf = gpu_render(ctx, sm, sc.camera, sc.poses, cfg)
    recs, nts, offs, pairs = gpu_buffers(ctx)
    pr = prep(gg)
    T = _tiles(sc.camera)
    n_far = 0
    for p in range(3):
        out, rec, ks, vs, rng_ = oracle_pose(pr, sc.poses[p], sc.camera)
        check_records(recs, nts, rec, gg.n, p)
        check_pairs(offs, pairs, ks, vs, rng_, p, T)
        zk = rec.z[rec.visible].astype(np.float32).view(np.uint32).astype(np.int64) - z0
        n_far += int((zk >= 1 << 27).sum())
        if p == 1:
            assert (zk < 1 << 27).sum() > 4096 and (zk >= 1 << 27).sum() > 4096
    assert n_far > 4096
    sm.free()


@pytest.mark.parametrize("seed", [41, 42])
def test_thin_tilted_and_huge_gaussians(ctx, seed):
    """Needle-thin tilted footprints and a few that cover the whole image: the
    cases where a (band, quarter) overlap test of the support ellipse is most
    easily wrong, and where A C - B^2 of the conic cancels the most."""
    say(f"anisotropic scene seed {seed}")
    sc = W.tiny_scene(seed, n=400, width=96, height=64, n_poses=3)
    g = sc.gaussians
    rng = np.random.default_rng(seed + 1000)
    s = np.exp(np.stack([rng.normal(-0.3, 0.8, g.n), rng.normal(-5.0, 0.5, g.n),
                         rng.normal(-4.0, 1.0, g.n)], 1))
    s[:6] = np.exp(rng.normal(0.8, 0.2, (6, 3)))  # a few very large ones
    thin = W.Gaussians(g.means, s.astype(np.float32), g.quats, g.opacity, g.rgb)
    sm = load(ctx, thin)
    rgb, dep, tf = gpu_render(ctx, sm, sc.camera, sc.poses)
    recs, nts, offs, pairs = gpu_buffers(ctx)
    pr = prep(thin)
    T = _tiles(sc.camera)
    for p in range(3):
        out, rec, ks, vs, rng_ = oracle_pose(pr, sc.poses[p], sc.camera)
        check_records(recs, nts, rec, thin.n, p)
        check_pairs(offs, pairs, ks, vs, rng_, p, T)
        compare_render(rgb[p], dep[p], tf[p], out, f"pose {p}")


def test_empty_and_all_culled(ctx):
    say("empty submap and a scene entirely behind the camera")
    sc = W.tiny_scene(30, n=50)
    empty = W.Gaussians(*[a[:0] for a in sc.gaussians.arrays()])
    sm = load(ctx, empty)
    rgb, dep, tf = gpu_render(ctx, sm, sc.camera, sc.poses)
    assert np.all(rgb == 0) and np.all(dep == 0) and np.all(tf == 1)
    g = sc.gaussians
    behind = W.Gaussians(g.means * np.array([1, -1, 1], np.float32), g.scales, g.quats, g.opacity, g.rgb)
    sm2 = load(ctx, behind)
    rgb, dep, tf = gpu_render(ctx, sm2, sc.camera, sc.poses)
    assert np.all(rgb == 0) and np.all(dep == 0) and np.all(tf == 1)
    assert ctx.stats()["n_visible"] == 0


def test_nan_and_degenerate_inputs_are_culled(ctx):
    say("NaN / Inf means, scales, opacities and colours, zero scales, zero quaternion")
    sc = W.tiny_scene(31, n=200)
    g = sc.gaussians
    means = g.means.copy()
    means[5] = np.nan
    means[11, 1] = np.inf
    scales = g.scales.copy()
    scales[7] = 0.0
    scales[13, 2] = np.inf
    quats = g.quats.copy()
    quats[9] = 0.0
    op = g.opacity.copy()
    op[[20, 21]] = [np.nan, np.inf]
    rgb_in = g.rgb.copy()
    rgb_in[30, 0] = np.nan
    rgb_in[31, 2] = -np.inf
    bad = W.Gaussians(means, scales, quats, op, rgb_in)
    sm = load(ctx, bad)
    rgb, dep, tf = gpu_render(ctx, sm, sc.camera, sc.poses)
    st = ctx.stats()
    recs, nts, offs, pairs = gpu_buffers(ctx)
    pr = prep(bad)
    n_bad = int(search.project.nonfinite(*pr).sum())
    say(f"  non-finite: gpu {st['n_culled_nonfinite']} oracle {n_bad}")
    assert st["n_culled_nonfinite"] == n_bad >= 7
    for p in range(sc.poses.shape[0]):
        out, rec, ks, vs, rng = oracle_pose(pr, sc.poses[p], sc.camera)
        assert not rec.visible[[5, 9, 11, 13, 20, 21, 30, 31]].any()
        check_records(recs, nts, rec, g.n, p)
        check_pairs(offs, pairs, ks, vs, rng, p, _tiles(sc.camera))
        compare_render(rgb[p], dep[p], tf[p], out, f"pose {p}")
        assert np.isfinite(rgb[p]).all() and np.isfinite(dep[p]).all()


def test_topk_ranks_nan_scores_last(ctx):
    """Scores with NaN and infinities: the order equals the oracle's (NaN after -inf)."""
    import torch
    say("top-k over scores with NaN, +-inf and ties")
    s = np.array([0.5, np.nan, -np.inf, 0.5, np.inf, np.nan, -0.25, 0.9, -np.inf, 0.0], np.float32)
    got = ctx.topk(to_dev(s), s.size).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(got, search.topk(s, s.size)), (got, search.topk(s, s.size))


def _stack_scene(n, spread, seed):
    """n small Gaussians crowded over one 16x16 tile: a very long tile list."""
    rng = np.random.default_rng(seed)
    y = rng.uniform(3.0, 30.0, n)
    x = rng.uniform(-spread, spread, n) * y
    z = rng.uniform(-spread, spread, n) * y
    means = np.stack([x, y, z], 1).astype(np.float32)
    scales = np.full((n, 3), 0.002, np.float32) * y[:, None].astype(np.float32)
    quats = rng.normal(size=(n, 4)).astype(np.float32)
    op = np.full(n, 0.05, np.float32)  # low opacity: the pixel walks deep into the list
    rgb = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    g = W.Gaussians(means, scales, quats, op, rgb)
    cam = W.Camera(64, 48, 400.0, 400.0, 32.0, 24.0)
    poses = W.yaw_grid_poses(np.zeros(3), W.AXES_ALONG_Y, [0.0], [0.0], [0.0])
    return g, cam, poses


@pytest.mark.parametrize("n,label", [(3500, "> 2048 per list"), (12000, "> 8192 per list")])
def test_long_tile_lists(ctx, n, label):
    say(f"long tile lists: {n} Gaussians crowded over one tile ({label})")
    g, cam, poses = _stack_scene(n, 0.01, 40 + n)
    sm = load(ctx, g)
    rgb, dep, tf = gpu_render(ctx, sm, cam, poses)
    recs, nts, offs, pairs = gpu_buffers(ctx)
    out, rec, ks, vs, rng = oracle_pose(prep(g), poses[0], cam)
    lens = rng[:, 1] - rng[:, 0]
    say(f"  longest list {lens.max()}")
    assert lens.max() > (8192 if n > 8192 else 2048)
    check_records(recs, nts, rec, n, 0)
    check_pairs(offs, pairs, ks, vs, rng, 0, _tiles(cam))
    compare_render(rgb[0], dep[0], tf[0], out, "pose 0")


@pytest.mark.parametrize("w,h,n_poses", [(1000, 600, 2), (2048, 2048, 1)])
def test_many_tiles_bucketing(ctx, w, h, n_poses):
    """Tile bucketing with several 64-tile buckets: 2394 tiles (38 buckets, the last
    holding 26 tiles) and the largest supported image, 16384 tiles (256 buckets).
    Records, list offsets and lists bit for bit, images within tolerance."""
    T = ((w + 15) // 16) * ((h + 15) // 16)
    say(f"many tiles: {w}x{h} ({T} tiles), 3000 Gaussians, {n_poses} poses")
    sc = W.tiny_scene(61, n=3000, width=w, height=h, n_poses=max(n_poses, 2), log_scale_mean=-3.0)
    poses = sc.poses[:n_poses]
    sm = load(ctx, sc.gaussians)
    rgb, dep, tf = gpu_render(ctx, sm, sc.camera, poses)
    recs, nts, offs, pairs = gpu_buffers(ctx)
    pr = prep(sc.gaussians)
    assert T == _tiles(sc.camera)
    for p in range(n_poses):
        out, rec, ks, vs, rng = oracle_pose(pr, poses[p], sc.camera)
        check_records(recs, nts, rec, sc.gaussians.n, p)
        check_pairs(offs, pairs, ks, vs, rng, p, T)
        compare_render(rgb[p], dep[p], tf[p], out, f"pose {p}")
    sm.free()


def test_determinism_and_fixed_capacity(ctx):
    say("config0 twice (exact sizing) and once with a fixed pair capacity")
    from paper_2403_11367_amd import default_cfg
    sc = W.config0()
    sm = load(ctx, sc.gaussians)
    a = gpu_render(ctx, sm, sc.camera, sc.poses)
    b = gpu_render(ctx, sm, sc.camera, sc.poses)
    n_pairs = ctx.stats()["n_pairs"]
    c = gpu_render(ctx, sm, sc.camera, sc.poses, default_cfg(pair_capacity=n_pairs + 7))
    ctx.sync()
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y) and np.array_equal(x, z)


def test_pose_groups_do_not_change_results(ctx):
    """The poses may be rendered in groups on concurrent streams: images, pair
    lists and list offsets are the same for every grouping and capacity mode."""
    say("config0 with 1, 2, 3, 5 and 8 pose groups, exact and fixed capacity")
    from paper_2403_11367_amd import BUF_OFFSETS, BUF_PAIRS, default_cfg
    sc = W.config0()
    sm = load(ctx, sc.gaussians)
    ref = gpu_render(ctx, sm, sc.camera, sc.poses, default_cfg(pose_groups=1))
    ref_off, ref_pairs = ctx.debug_buffer(BUF_OFFSETS), ctx.debug_buffer(BUF_PAIRS)
    n_pairs = ctx.stats()["n_pairs"]
    for groups in (2, 3, 5, 8):
        for cap in (0, n_pairs):
            out = gpu_render(ctx, sm, sc.camera, sc.poses, default_cfg(pose_groups=groups, pair_capacity=cap))
            st = ctx.stats()
            assert st["n_groups"] == groups and st["n_pairs"] == n_pairs
            ctx.sync()
            for x, y in zip(ref, out):
                assert np.array_equal(x, y), f"{groups} groups, capacity {cap}"
            assert np.array_equal(ctx.debug_buffer(BUF_OFFSETS), ref_off)
            assert np.array_equal(ctx.debug_buffer(BUF_PAIRS), ref_pairs)


def test_overflow_and_bad_index_are_reported(ctx):
    say("forced pair overflow (capacity 1) and an out-of-range submap index")
    from paper_2403_11367_amd import GsrError, default_cfg
    sc = W.config0()
    sm = load(ctx, sc.gaussians)
    gpu_render(ctx, sm, sc.camera, sc.poses[:2], default_cfg(pair_capacity=1))
    with pytest.raises(GsrError) as e:
        ctx.sync()
    assert e.value.status == -5
    ctx.sync()  # flag cleared
    good = gpu_render(ctx, sm, sc.camera, sc.poses[:2])
    assert good[0].max() > 0
    idx = np.arange(10, dtype=np.int64)
    idx[3] = sc.gaussians.n + 5
    load(ctx, sc.gaussians, index=idx)
    with pytest.raises(GsrError) as e:
        ctx.sync()
    assert e.value.status == -7


def test_argument_errors(ctx):
    say("argument validation")
    import torch
    from paper_2403_11367_amd import GsrError, default_cfg
    sc = W.tiny_scene(32, n=10)
    sm = load(ctx, sc.gaussians)
    with pytest.raises(GsrError) as e:
        gpu_render(ctx, sm, sc.camera, sc.poses, default_cfg(tile_w=8, tile_h=8))
    assert e.value.status == -6
    with pytest.raises(GsrError):
        gpu_render(ctx, sm, sc.camera, sc.poses, default_cfg(tile_w=12))
    with pytest.raises(GsrError) as e:  # depth keys need a near plane >= 0
        gpu_render(ctx, sm, sc.camera, sc.poses, default_cfg(z_near=-0.1))
    assert e.value.status == -1
    s = torch.zeros(4, device="cuda")
    with pytest.raises(GsrError):
        ctx.topk(s, 5)


def test_ncc_matches_oracle_full_size(ctx):
    """Full headline size: 64 renders at 1408x376, seeded synthetic images."""
    say("NCC: 64 x 1408x376 seeded images")
    import torch
    imgs = W.random_images(7, 65, 376, 1408)
    q = imgs[0]
    r = imgs[1:].copy()
    r[3] = 0.25  # constant render -> 0
    r[5] = 2.0 * r[4] + 0.5  # affine copy -> same score as r[4]
    got = ctx.ncc(to_dev(q), to_dev(r)).cpu().numpy()
    ref = oncc.ncc(q, r)
    err = np.abs(got - ref).max()
    say(f"  max |dncc| {err:.2e}")
    assert err <= TOL_NCC
    assert got[3] == 0.0
    assert abs(got[5] - got[4]) <= 2 * TOL_NCC
    # ragged block and self-correlation
    small = W.random_images(8, 3, 37, 53)
    s = ctx.ncc(to_dev(small[0]), to_dev(small)).cpu().numpy()
    assert abs(s[0] - 1.0) <= TOL_NCC
    assert np.abs(s - oncc.ncc(small[0], small)).max() <= TOL_NCC
    # 4 | H x W but renders not 16-byte aligned (a view one float into a buffer):
    # the per-pixel loads instead of the 4-pixel ones
    even = W.random_images(9, 4, 32, 48)
    flat = torch.zeros(1 + even[1:].size, dtype=torch.float32, device="cuda")
    view = flat[1:].view(3, 3, 32, 48)
    view.copy_(to_dev(even[1:]))
    e = ctx.ncc(to_dev(even[0]), view).cpu().numpy()
    assert np.abs(e - oncc.ncc(even[0], even[1:])).max() <= TOL_NCC
    torch.cuda.synchronize()


def test_topk_ties_and_order(ctx):
    say("top-k with ties")
    rng = np.random.default_rng(3)
    for n in (1, 5, 64, 1000, 8192):
        s = rng.integers(0, 20, n).astype(np.float32) / 7.0
        k = min(n, 16)
        got = ctx.topk(to_dev(s), k).cpu().numpy()
        assert np.array_equal(got, search.topk(s, k))
        assert int(ctx.topk(to_dev(s), 1).cpu().numpy()[0]) == search.argmax(s)


def test_config0_end_to_end_search(ctx):
    say("config0 end to end: render 16 candidates, NCC against the query, argmax")
    sc = W.config0()
    pr = prep(sc.gaussians)
    q_ref = search.render_pose(pr, sc.hidden_pose, sc.camera)
    query = (q_ref.rgb + sc.query_noise).astype(np.float32)
    refs = [search.render_pose(pr, sc.poses[p], sc.camera) for p in range(16)]
    ref_scores = oncc.ncc(query, np.stack([r.rgb for r in refs]))
    sm = load(ctx, sc.gaussians)
    import torch
    rgb, dep = ctx.render(sm, __import__("helpers").camera(sc.camera), to_dev(sc.poses))
    scores = ctx.ncc(to_dev(query), rgb)
    best = ctx.topk(scores, 1)
    torch.cuda.synchronize()
    got = scores.cpu().numpy()
    say(f"  scores max err {np.abs(got - ref_scores).max():.2e}; best {int(best.cpu()[0])} "
        f"oracle {search.argmax(ref_scores)}")
    assert np.abs(got - ref_scores).max() <= TOL_NCC
    srt = np.sort(ref_scores)
    if srt[-1] - srt[-2] > 2 * TOL_NCC:
        assert int(best.cpu()[0]) == search.argmax(ref_scores)


def test_random_order_search_with_early_stop(ctx):
    """gsr_search against the oracle's early_stop_search on the oracle's scores
    (config0, 16 candidates in a seeded random order)."""
    say("config0 random-order search: batches, scored share, NCC threshold")
    sc = W.config0()
    pr = prep(sc.gaussians)
    q_ref = search.render_pose(pr, sc.hidden_pose, sc.camera)
    query = (q_ref.rgb + sc.query_noise).astype(np.float32)
    ref = oncc.ncc(query, np.stack([search.render_pose(pr, sc.poses[p], sc.camera).rgb for p in range(16)]))
    order = W.search_order(7, 16)
    sm = load(ctx, sc.gaussians)
    cam = __import__("helpers").camera(sc.camera)
    poses, q = to_dev(sc.poses), to_dev(query)
    # thresholds half-way between well separated oracle scores, so that float32 rounding
    # cannot move a score across one
    srt = np.sort(ref)
    mids = [(a + b) / 2 for a, b in zip(srt[:-1], srt[1:]) if b - a > 4 * TOL_NCC]
    cases = [(4, 16, np.inf), (3, 12, np.inf), (1, 16, mids[-1]), (4, 16, mids[len(mids) // 2]),
             (5, 13, mids[0]), (16, 16, mids[-1])]
    for batch, max_eval, thr in cases:
        best, score, n, scores = ctx.search(sm, cam, poses, order, batch, max_eval, float(thr), q)
        rb, rs, rn = search.early_stop_search(ref, order, batch, max_eval, thr)
        got = scores.cpu().numpy()
        scored = order[:n]
        say(f"  batch {batch} max {max_eval} thr {thr:.4f}: gpu ({best}, {score:.5f}, {n}) oracle ({rb}, {rs:.5f}, {rn})")
        assert n == rn
        assert abs(score - rs) <= TOL_NCC
        assert np.abs(got[scored] - ref[scored]).max() <= TOL_NCC
        assert np.all(np.isnan(np.delete(got, scored)))
        top = np.sort(ref[scored])
        if top.size < 2 or top[-1] - top[-2] > 2 * TOL_NCC:
            assert best == rb
    with pytest.raises(__import__("paper_2403_11367_amd").GsrError):
        ctx.search(sm, cam, poses, np.zeros(16, np.int32), 4, 16, 0.5, q)  # not a permutation


@pytest.fixture(scope="module")
def cfg1():
    sc = W.config1()
    idx = ocrop.crop_indices(sc.gaussians.means, sc.crop_cell, sc.prior_center[:2], sc.crop_radius, sc.crop_voxel)
    return sc, idx


def test_config1_full_size_frames(ctx, cfg1):
    """Headline shape: 500,143-Gaussian crop, 64 poses, 1408x376 (the bench launch);
    records, keys and order of 4 poses bit-exact, and those 4 frames compared
    with the oracle on every pixel (depth bar 1e-4 x max(1, depth))."""
    sc, idx = cfg1
    say(f"config1: crop {idx.size} of {sc.gaussians.n}, 64 poses, 1408x376")
    sm = load(ctx, sc.gaussians, index=idx)
    rgb, dep, tf = gpu_render(ctx, sm, sc.camera, sc.poses)
    st = ctx.stats()
    say(f"  stats {st}")
    recs, nts, offs, pairs = gpu_buffers(ctx)
    sub = sc.gaussians.take(idx)
    pr = prep(sub)
    T = _tiles(sc.camera)
    for p in (0, 21, 42, 63):
        out, rec, ks, vs, rng = oracle_pose(pr, sc.poses[p], sc.camera)
        check_records(recs, nts, rec, idx.size, p)
        check_pairs(offs, pairs, ks, vs, rng, p, T)
        compare_render(rgb[p], dep[p], tf[p], out, f"pose {p}", depth_rel=True)
    # properties at full size: T in [0, 1], colours in [0, 1] (all inputs are)
    assert tf.min() >= 0 and tf.max() <= 1
    assert rgb.min() >= 0 and rgb.max() <= 1 + 1e-5


def test_eval_counters_match_oracle(ctx):
    """GSR_RENDER_COUNT_EVALS: same images; contribution count equals the oracle's."""
    say("config0 with evaluation counting")
    from paper_2403_11367_amd import default_cfg
    from paper_2403_11367_amd.gsr import RENDER_COUNT_EVALS
    sc = W.config0()
    sm = load(ctx, sc.gaussians)
    a = gpu_render(ctx, sm, sc.camera, sc.poses)
    b = gpu_render(ctx, sm, sc.camera, sc.poses, default_cfg(flags=RENDER_COUNT_EVALS))
    st = ctx.stats()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    pr = prep(sc.gaussians)
    ref = 0
    flagged = 0
    for p in range(sc.poses.shape[0]):
        out = search.render_pose(pr, sc.poses[p], sc.camera)
        ref += int(out.n_contrib.sum())
        flagged += int(out.flag.sum())
    say(f"  contributions gpu {st['evals_contrib']} oracle {ref} (flagged px {flagged}); "
        f"lane slots {st['evals_lanes']}")
    assert abs(st["evals_contrib"] - ref) <= 2 * flagged
    assert st["evals_lanes"] >= st["evals_contrib"]


def test_fig2_ncc_profile_config0_and_config1(ctx, cfg1):
    """Sec. IV, Fig. 2 on the library: NCC of renders swept through the hidden
    pose in x and in yaw peaks at the hidden pose and falls with the error
    (config 0: the scores equal the oracle's within 1e-4; config 1: full-map
    query, cropped-submap renders at 1408x376). On config 1 the best of the 64
    grid candidates lies within one grid step (1 m, 1 m, 5 degrees) of the
    hidden pose."""
    import torch
    from test_oracle_search import FIG2_DX, FIG2_DYAW, check_fig2_profile, fig2_sweeps
    sc = W.config0()
    sm = load(ctx, sc.gaussians)
    pr = prep(sc.gaussians)
    query = (search.render_pose(pr, sc.hidden_pose, sc.camera).rgb + sc.query_noise).astype(np.float32)
    xs, ys = fig2_sweeps(sc)
    for poses, offs in ((xs, FIG2_DX), (ys, FIG2_DYAW)):
        rgb, _, _ = gpu_render(ctx, sm, sc.camera, poses)
        got = ctx.ncc(to_dev(query), to_dev(rgb)).cpu().numpy()
        ref = oncc.ncc(query, np.stack([search.render_pose(pr, p, sc.camera).rgb for p in poses]))
        say(f"  config0 sweep: gpu {np.round(got, 4)}")
        assert np.abs(got - ref).max() <= TOL_NCC
        check_fig2_profile(got, offs)
    sm.free()
    sc1, idx = cfg1
    full = load(ctx, sc1.gaussians)
    q_rgb, _, _ = gpu_render(ctx, full, sc1.camera, sc1.hidden_pose[None])
    query1 = to_dev(q_rgb[0] + sc1.query_noise)
    full.free()
    sm1 = load(ctx, sc1.gaussians, index=idx)
    xs, ys = fig2_sweeps(sc1)
    for poses, offs in ((xs, FIG2_DX), (ys, FIG2_DYAW)):
        rgb, _, _ = gpu_render(ctx, sm1, sc1.camera, poses)
        got = ctx.ncc(query1, to_dev(rgb)).cpu().numpy()
        say(f"  config1 sweep: {np.round(got, 4)}")
        check_fig2_profile(got, offs)
    rgb, _, _ = gpu_render(ctx, sm1, sc1.camera, sc1.poses)
    s = ctx.ncc(query1, to_dev(rgb)).cpu().numpy()
    torch.cuda.synchronize()
    best = int(np.argmax(s))
    steps = [-1.5, -0.5, 0.5, 1.5]
    grid = [(dx, dy, dyaw) for dx in steps for dy in steps for dyaw in [-7.5, -2.5, 2.5, 7.5]]
    hx, hy, hyaw = sc1.hidden_offset
    bx, by, byaw = grid[best]
    say(f"  config1 grid: best {best} at {grid[best]}, hidden ({hx:.2f}, {hy:.2f}, {hyaw:.2f}), NCC {s[best]:.4f}")
    assert abs(bx - hx) <= 1.0 and abs(by - hy) <= 1.0 and abs(byaw - hyaw) <= 5.0
    sm1.free()


TILE_SHAPES = [(32, 8), (8, 32)]


def _tiles_of(cam, tw, th):
    return ((cam.width + tw - 1) // tw) * ((cam.height + th - 1) // th)


def _shape_case(ctx, g, cam, poses, tw, th, label, depth_rel=False):
    from paper_2403_11367_amd import default_cfg
    sm = load(ctx, g)
    rgb, dep, tf = gpu_render(ctx, sm, cam, poses, default_cfg(tile_w=tw, tile_h=th))
    recs, nts, offs, pairs = gpu_buffers(ctx)
    pr = prep(g)
    T = _tiles_of(cam, tw, th)
    for p in range(poses.shape[0]):
        out, rec, ks, vs, rng = oracle_pose(pr, poses[p], cam, tile=(tw, th))
        check_records(recs, nts, rec, g.n, p)
        check_pairs(offs, pairs, ks, vs, rng, p, T)
        compare_render(rgb[p], dep[p], tf[p], out, f"{label} {tw}x{th} pose {p}", depth_rel=depth_rel)
    sm.free()


@pytest.mark.parametrize("tw,th", TILE_SHAPES)
def test_tile_shapes_config0_and_ragged(ctx, tw, th):
    """32x8 and 8x32 tiles (the compositing's other wave bands and cells): records,
    tile counts, keys, per-tile order bit for bit and images against the oracle
    rendering the same tiles, on config 0 and on ragged tiny scenes."""
    say(f"tile shape {tw}x{th}: config0 and ragged scenes")
    sc = W.config0()
    _shape_case(ctx, sc.gaussians, sc.camera, sc.poses[::3], tw, th, "config0")
    for seed, n, w, h in [(22, 500, 37, 21), (24, 1000, 200, 9), (23, 64, 16, 16)]:
        t = W.tiny_scene(seed, n=n, width=w, height=h, n_poses=2)
        _shape_case(ctx, t.gaussians, t.camera, t.poses, tw, th, f"tiny {seed}")


@pytest.mark.parametrize("tw,th", TILE_SHAPES)
def test_tile_shapes_thin_huge_and_long_lists(ctx, tw, th):
    """The same for needle-thin tilted and image-covering footprints, and for tile
    lists of a few thousand records."""
    say(f"tile shape {tw}x{th}: anisotropic scene and long lists")
    sc = W.tiny_scene(41, n=400, width=96, height=64, n_poses=2)
    g = sc.gaussians
    rng = np.random.default_rng(1041)
    s = np.exp(np.stack([rng.normal(-0.3, 0.8, g.n), rng.normal(-5.0, 0.5, g.n), rng.normal(-4.0, 1.0, g.n)], 1))
    s[:6] = np.exp(rng.normal(0.8, 0.2, (6, 3)))
    thin = W.Gaussians(g.means, s.astype(np.float32), g.quats, g.opacity, g.rgb)
    _shape_case(ctx, thin, sc.camera, sc.poses, tw, th, "anisotropic")
    g2, cam2, poses2 = _stack_scene(3500, 0.01, 3540)
    _shape_case(ctx, g2, cam2, poses2, tw, th, "long lists")


def test_tile_shapes_config1_frame(ctx, cfg1):
    """The headline submap at full size with 32x8 and 8x32 tiles: two whole
    frames each against the oracle (depth bar relative to max(1, depth))."""
    from paper_2403_11367_amd import default_cfg
    sc, idx = cfg1
    sub = sc.gaussians.take(idx)
    pr = prep(sub)
    for tw, th in TILE_SHAPES:
        say(f"config1 with {tw}x{th} tiles")
        sm = load(ctx, sc.gaussians, index=idx)
        poses = sc.poses[[5, 50]]
        rgb, dep, tf = gpu_render(ctx, sm, sc.camera, poses, default_cfg(tile_w=tw, tile_h=th))
        recs, nts, offs, pairs = gpu_buffers(ctx)
        T = _tiles_of(sc.camera, tw, th)
        for p in range(2):
            out, rec, ks, vs, rng = oracle_pose(pr, poses[p], sc.camera, tile=(tw, th))
            check_records(recs, nts, rec, idx.size, p)
            check_pairs(offs, pairs, ks, vs, rng, p, T)
            compare_render(rgb[p], dep[p], tf[p], out, f"config1 {tw}x{th} pose {p}", depth_rel=True)
        sm.free()


def test_host_input_load_equals_device_load(ctx):
    """gsr_submap_load_host (host arrays, with and without an index) gives the
    records and images of gsr_submap_load on the same data, bit for bit."""
    import torch
    say("host-input submap load")
    sc = W.tiny_scene(21, n=300, width=64, height=48, n_poses=3)
    g = sc.gaussians
    idx = np.random.default_rng(2).permutation(g.n)[:200].astype(np.int64)
    for index in (None, idx):
        a = load(ctx, g, index)
        ra = gpu_render(ctx, a, sc.camera, sc.poses)
        recs_a = ctx.debug_buffer(__import__("paper_2403_11367_amd").BUF_RECORDS)
        b = ctx.load_submap_host(*g.arrays(), index=index)
        assert b.n == (g.n if index is None else idx.size)
        rb = gpu_render(ctx, b, sc.camera, sc.poses)
        recs_b = ctx.debug_buffer(__import__("paper_2403_11367_amd").BUF_RECORDS)
        torch.cuda.synchronize()
        assert np.array_equal(recs_a.view(np.uint32), recs_b.view(np.uint32))
        for x, y in zip(ra, rb):
            assert np.array_equal(x, y)
        a.free()
        b.free()


def test_workspace_limit_and_overflow_retry(ctx):
    """A workspace limit below what a render needs fails with GSR_ENOMEM and the
    context keeps working once the limit is lifted; a fixed pair capacity that is
    too small, with GSR_RENDER_RETRY_OVERFLOW, renders again exactly and gives the
    exact render's images, while without it gsr_sync reports the overflow."""
    from paper_2403_11367_amd import Context, GsrError, default_cfg
    from paper_2403_11367_amd.gsr import RENDER_RETRY_OVERFLOW
    say("workspace limit and overflow retry")
    sc = W.config0()
    c2 = Context(0)
    sm = load(c2, sc.gaussians)
    c2.set_workspace_limit(1 << 20)
    with pytest.raises(GsrError) as e:
        gpu_render(c2, sm, sc.camera, sc.poses)
    assert e.value.status == -2 and "workspace limit" in str(e.value)
    c2.set_workspace_limit(0)
    exact = gpu_render(c2, sm, sc.camera, sc.poses)
    st = c2.stats()
    assert st["workspace_bytes"] > (1 << 20) and st["overflow_retried"] == 0
    small = default_cfg(pair_capacity=1000, flags=RENDER_RETRY_OVERFLOW)
    got = gpu_render(c2, sm, sc.camera, sc.poses, small)
    assert c2.stats()["overflow_retried"] == 1
    for x, y in zip(exact, got):
        assert np.array_equal(x, y)
    c2.sync()  # nothing left to report
    gpu_render(c2, sm, sc.camera, sc.poses, default_cfg(pair_capacity=1000))
    with pytest.raises(GsrError) as e:
        c2.sync()
    assert e.value.status == -5
    sm.free()
    c2.close()
