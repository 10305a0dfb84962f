"""Batched queries (gsr_render_multi), the launch variants the autotuner picks
from, and HIP graph capture: every path must give the images of separate
gsr_render calls bit for bit (and those match the oracle: test_gpu_parity)."""
import numpy as np
import pytest

import workloads as W
from helpers import camera, compare_render, load, prep, say, to_dev
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


def _separate(ctx, sms, poses_list, cam, cfg=None):
    import torch
    outs = [ctx.render(sm, cam, to_dev(p), cfg, with_tfinal=True) for sm, p in zip(sms, poses_list)]
    torch.cuda.synchronize()
    return [torch.cat([o[i] for o in outs]) for i in range(3)]


def test_multi_equals_separate_tiny_uneven(ctx):
    """Three tiny scenes of 300, 40 and 1000 Gaussians with 2, 3 and 1 poses in one
    render: bit-identical to three renders, and the first scene matches the oracle."""
    import torch
    say("render_multi: 3 tiny scenes (300, 40, 1000 Gaussians; 2, 3, 1 poses), 64x48")
    scenes = [W.tiny_scene(31, n=300, n_poses=2), W.tiny_scene(32, n=40, n_poses=3),
              W.tiny_scene(33, n=1000, n_poses=1)]
    cam = camera(scenes[0].camera)
    sms = [load(ctx, sc.gaussians) for sc in scenes]
    poses = [sc.poses for sc in scenes]
    ref = _separate(ctx, sms, poses, cam)
    got = ctx.render_multi(sms, [p.shape[0] for p in poses], cam, to_dev(np.concatenate(poses)), with_tfinal=True)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    pr = prep(scenes[0].gaussians)
    for p in range(2):
        out = search.render_pose(pr, scenes[0].poses[p], scenes[0].camera)
        compare_render(got[0][p].cpu().numpy(), got[1][p].cpu().numpy(), got[2][p].cpu().numpy(), out,
                       f"scene 0 pose {p}")
    for sm in sms:
        sm.free()


@pytest.fixture(scope="module")
def batch4(ctx):
    """Four queries of the batched workload (maps of 751,911 / 350,365 / 587,946 /
    498,125 Gaussians before the 50 m crop), 32 candidates each, 1408x376."""
    import torch
    from paper_2403_11367_amd import crop
    cam = camera(W.config1_camera())
    qs = [W.batch_query(s, W.config1_camera()) for s in W.BATCH_MAP_SEEDS[:4]]
    sms = []
    for q in qs:
        idx = crop(q.gaussians.means, 10.0, (100.0, 0.0), 50.0, 1.0)
        sms.append(load(ctx, q.gaussians, idx))
    poses = to_dev(np.concatenate([q.poses for q in qs]))
    yield cam, qs, sms, poses
    torch.cuda.synchronize()
    for sm in sms:
        sm.free()


def test_multi_and_launch_variants_equal_separate(ctx, batch4):
    """The batched render of 4 queries equals 4 separate renders bit for bit, for
    every chunk size, persistent and grid launches, and pose groups."""
    import torch
    from paper_2403_11367_amd import default_cfg
    cam, qs, sms, poses = batch4
    say(f"render_multi: 4 queries ({[sm.n for sm in sms]} Gaussians after the crop), 4 x 32 poses, 1408x376")
    ref = _separate(ctx, sms, [q.poses for q in qs], cam)
    counts = [32] * 4
    for chunk, blocks, groups in [(0, 0, 1), (124, 0, 1), (60, 0, 1), (252, 4, 1), (124, 8, 2), (60, 2, 4)]:
        cfg = default_cfg(blend_chunk=chunk, blend_blocks_per_cu=blocks, pose_groups=groups)
        got = ctx.render_multi(sms, counts, cam, poses, cfg, with_tfinal=True)
        torch.cuda.synchronize()
        same = all(torch.equal(a, b) for a, b in zip(got, ref))
        say(f"  chunk {chunk} blocks/CU {blocks} groups {groups}: identical {same}")
        assert same


def test_graph_replays_match_eager(ctx, batch4):
    """A captured batched render + NCC, replayed three times with other work of the
    context in between, gives the eager result every time."""
    import torch
    from paper_2403_11367_amd import default_cfg
    cam, qs, sms, poses = batch4
    say("graph capture: render_multi (4 x 32 poses) + NCC, 3 replays")
    counts = [32] * 4
    P = poses.shape[0]
    dev = poses.device
    query = torch.rand((3, cam.height, cam.width), device=dev)
    rgb = torch.empty((P, 3, cam.height, cam.width), device=dev)
    depth = torch.empty((P, cam.height, cam.width), device=dev)
    scores = torch.empty((P,), device=dev)
    ctx.render_multi(sms, counts, cam, poses)  # exact sizing: learns the pair count
    n_pairs = ctx.stats()["n_pairs"]
    cfg = default_cfg(pair_capacity=int(n_pairs * 1.1) + 4096, blend_blocks_per_cu=4)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx.render_multi(sms, counts, cam, poses, cfg, rgb=rgb, depth=depth)  # sizes every workspace
        ctx.ncc(query, rgb, scores)
        stream.synchronize()
        e_rgb, e_depth, e_scores = rgb.clone(), depth.clone(), scores.clone()
        ctx.capture_begin()
        ctx.render_multi(sms, counts, cam, poses, cfg, rgb=rgb, depth=depth)
        ctx.ncc(query, rgb, scores)
        graph = ctx.capture_end()
        for r in range(3):
            rgb.zero_()
            depth.zero_()
            scores.zero_()
            ctx.render(sms[0], cam, poses[:8].contiguous(), cfg)  # other work between replays
            graph.launch()
            stream.synchronize()
            ok = torch.equal(rgb, e_rgb) and torch.equal(depth, e_depth) and torch.equal(scores, e_scores)
            say(f"  replay {r}: identical {ok}")
            assert ok
        ctx.sync()
        graph.close()


def test_capture_rules(ctx, batch4):
    """Under capture a render without a fixed pair capacity, or one whose workspace
    would have to grow, is refused with GSR_EINVAL; the capture still ends cleanly."""
    import torch
    from paper_2403_11367_amd import GsrError, default_cfg
    cam, qs, sms, poses = batch4
    say("graph capture: refused calls")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        small = poses[:2].contiguous()
        rgb = torch.empty((2, 3, cam.height, cam.width), device=poses.device)
        depth = torch.empty((2, cam.height, cam.width), device=poses.device)
        cfg = default_cfg(pair_capacity=1 << 20)
        ctx.render(sms[0], cam, small, cfg, rgb=rgb, depth=depth)
        stream.synchronize()
        ctx.capture_begin()
        ctx.render(sms[0], cam, small, cfg, rgb=rgb, depth=depth)
        with pytest.raises(GsrError, match="EINVAL"):
            ctx.render(sms[0], cam, small, default_cfg(), rgb=rgb, depth=depth)  # exact sizing
        with pytest.raises(GsrError, match="EINVAL"):
            ctx.render(sms[0], cam, small, default_cfg(pair_capacity=1 << 30), rgb=rgb, depth=depth)  # growth
        graph = ctx.capture_end()
        graph.launch()
        stream.synchronize()
        graph.close()


def test_empty_submap(ctx):
    """A submap with no Gaussians renders background (colour and depth 0, T = 1),
    alone and inside a batch; its NCC against any query is 0."""
    import torch
    say("empty submap: render, batched render, NCC")
    sc = W.tiny_scene(41, n=200, n_poses=2)
    cam = camera(sc.camera)
    empty = W.Gaussians(*(np.zeros((0,) + a.shape[1:], np.float32) for a in sc.gaussians.arrays()))
    sm0 = load(ctx, empty)
    sm1 = load(ctx, sc.gaussians)
    assert sm0.n == 0
    rgb, depth, tf = ctx.render(sm0, cam, to_dev(sc.poses), with_tfinal=True)
    torch.cuda.synchronize()
    assert float(rgb.abs().max()) == 0 and float(depth.abs().max()) == 0 and float(tf.min()) == 1
    ref = ctx.render(sm1, cam, to_dev(sc.poses), with_tfinal=True)
    got = ctx.render_multi([sm0, sm1], [2, 2], cam, to_dev(np.concatenate([sc.poses, sc.poses])), with_tfinal=True)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a[2:], b)
    assert float(got[0][:2].abs().max()) == 0
    scores = ctx.ncc(torch.rand((3, cam.height, cam.width), device="cuda"), rgb)
    assert float(scores.abs().max()) == 0
    for sm in (sm0, sm1):
        sm.free()


@pytest.mark.parametrize("tw,th", [(32, 8), (8, 32)])
def test_multi_tile_shapes_equal_separate(ctx, batch4, tw, th):
    """With 32x8 and 8x32 tiles the batched render equals separate renders of the
    same tile shape bit for bit, for grid and persistent launches."""
    import torch
    from paper_2403_11367_amd import default_cfg
    cam, qs, sms, poses = batch4
    say(f"render_multi with {tw}x{th} tiles: 4 queries x 32 poses")
    outs = [ctx.render(sm, cam, to_dev(q.poses), default_cfg(tile_w=tw, tile_h=th), with_tfinal=True)
            for sm, q in zip(sms, qs)]
    ref = [torch.cat([o[i] for o in outs]) for i in range(3)]
    for chunk, blocks in [(0, 0), (124, 8)]:
        cfg = default_cfg(tile_w=tw, tile_h=th, blend_chunk=chunk, blend_blocks_per_cu=blocks)
        got = ctx.render_multi(sms, [32] * 4, cam, poses, cfg, with_tfinal=True)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(got, ref)), (chunk, blocks)


def test_autotune_per_bucket_and_cache(ctx, tmp_path):
    """The autotuner tries every tile shape, chunk, launch and grouping on a
    workload, keeps the fastest under its submap-size bucket key and answers the
    same key from its cache."""
    from paper_2403_11367_amd import autotune, default_cfg
    scenes = [W.tiny_scene(31, n=300, n_poses=2), W.tiny_scene(33, n=1000, n_poses=2)]
    cam = camera(scenes[0].camera)
    path = str(tmp_path / "tune.json")
    keys = set()
    for sc in scenes:
        sm = load(ctx, sc.gaussians)
        key = autotune.workload_key("test", cam.width, cam.height, 2, autotune.size_bucket(sm.n))
        keys.add(key)
        cfg, record = autotune.tune(key, default_cfg(), lambda c: ctx.render(sm, cam, to_dev(sc.poses), c),
                                    reps=1, path=path)
        assert len(record["variants"]) == len(autotune.variants())
        assert {(v["tile_w"], v["tile_h"]) for v in record["variants"]} == set(autotune.TILES)
        assert (cfg.tile_w, cfg.tile_h) in autotune.TILES
        cfg2, record2 = autotune.tune(key, default_cfg(), lambda c: ctx.render(sm, cam, to_dev(sc.poses), c),
                                      path=path)
        assert record2 == {} and (cfg2.tile_w, cfg2.blend_chunk) == (cfg.tile_w, cfg.blend_chunk)
        sm.free()
    assert len(keys) == 2  # 300 and 1000 Gaussians fall in different buckets
