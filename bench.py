#!/usr/bin/env python3
"""Headline benchmark: candidate poses rendered + NCC-scored per second.

Workload (the driving-scale relocalisation case): a 1,000,000-Gaussian
street-corridor map, cropped on the host to the 10 m voxel cells within 50 m
of the prior (500,143 Gaussians), 64 candidate poses at 1408x376, full-
resolution NCC against the query, top-1 selection. One step = one pass of the
whole hot path on device-resident inputs: pack the submap from the map
(gather by the crop index), preprocess + tile keys + per-tile sort + blend for
all 64 poses, NCC of the 64 renders, top-1. The crop itself is host code run
once per query and is not timed.

Beside the headline, on the same submap and query: the random-order search with
an early stop (Sec. IV), and learned vs plain over 1024 candidates (the trained
scorer prunes to 16 from quarter-resolution renders; the same pruning with
low-resolution NCC in place of the network; plain renders all at full
resolution), and batched queries: 8 maps of uneven size x 32 candidates in one
batched render per stage (autotuned launch) and as a HIP-graph replay, against
8 separate renders; and one map-training step (forward + backward of 4 views of a
500,000-Gaussian map, Adam).

Prints one JSON line (rank 0). See --help for flags.
"""
import argparse
import contextlib
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
FP32_VECTOR_PEAK = 157.3     # TFLOP/s, MI355X published fp32 vector (packed FMA)
FLOPS_PER_CONTRIB = 25       # flops of one (pixel, Gaussian) contribution, Eq. 1, 2, 5
# the compositing kernel's sources: the counters in TRAFFIC_FILE hold for this text
BLEND_SRCS = [os.path.join(ROOT, "paper_2403_11367_amd", "csrc", f) for f in ("blend.hip", "blend_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "blend_config1_traffic.md")


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def blend_source_sha256() -> str:
    h = hashlib.sha256()
    for f in BLEND_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def _blend_traffic(n_groups):
    """HBM bytes per blend launch from the committed rocprofv3 counter summary, if
    it was taken on the current blend source with the same number of launches per
    render; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    m_h = re.search(r"blend_source_sha256:\s*([0-9a-f]{64})", txt)
    m_g = re.search(r"launches_per_render:\s*([0-9]+)", txt)
    if not (m_b and m_h and m_g) or int(m_g.group(1)) != n_groups:
        return None
    cur = blend_source_sha256()
    return float(m_b.group(1)) if m_h.group(1) == cur else None


def _oracle_candidates(args):
    """Worker: the oracle on candidate poses `poses` of a submap (pack + project +
    keys + sort + float64 blend), one thread; returns their renders."""
    arrays, poses, cam = args
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import search

    with threadpool_limits(limits=1):
        prep = search.prepare(W.Gaussians(*arrays))
        return [search.render_pose(prep, pose, cam).rgb.astype(np.float32) for pose in poses]


def _noop(x):
    return x


def _cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, sub_idx, n_cand):
    """The oracle, untouched, on a bounded sample of the same workload: n_cand
    full-frame candidates on one thread (BLAS pools limited to 1), then one
    candidate per core on every core of this process's affinity set (a process
    pool, one thread each), each followed by the oracle's NCC."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import ncc as oncc
    from oracle import search

    sub = scene.gaussians.take(sub_idx)
    query = (0.5 + scene.query_noise).astype(np.float32)  # synthetic stand-in query
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        prep = search.prepare(sub)
        renders = []
        for p in range(n_cand):
            renders.append(search.render_pose(prep, scene.poses[p], scene.camera).rgb)
        oncc.ncc(query, np.stack(renders))
        dt1 = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    n_all = min(cores, scene.poses.shape[0])
    ctxm = mp.get_context("spawn")
    arrays = tuple(sub.arrays())
    with ctxm.Pool(n_all) as pool:
        pool.map(_noop, range(n_all))  # workers started and importing before the clock starts
        t0 = time.perf_counter()
        parts = pool.map(_oracle_candidates, [(arrays, [scene.poses[p]], scene.camera) for p in range(n_all)],
                         chunksize=1)
        with threadpool_limits(limits=1):
            oncc.ncc(query, np.stack([r for part in parts for r in part]))
        dt_all = time.perf_counter() - t0
    model = _cpu_model()
    return {"value": n_all / dt_all, "unit": "candidates/s", "cores": n_all, "kind": "oracle",
            "sample": f"{n_all} of the 64 full-frame candidates of the same workload, one per core in a process "
                      f"pool of started workers (each: pack + project + keys + sort + float64 blend; then NCC), "
                      f"{dt_all:.1f} s wall, on {n_all} cores of '{model}'",
            "cpu_model": model,
            "single_core": {"value": n_cand / dt1, "cores": 1,
                            "sample": f"{n_cand} candidates on one thread, {dt1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-candidates", type=int, default=2, help="oracle sample size (0 = skip)")
    ap.add_argument("--pose-groups", type=int, default=0,
                    help="pose groups per render (0 = the library's automatic choice)")
    ap.add_argument("--tile", type=int, nargs=2, default=(16, 16), metavar=("W", "H"),
                    help="screen tile of the headline renders: 16 16, 32 8 or 8 32")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-queries leg")
    ap.add_argument("--no-training", action="store_true", help="skip the map-training leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy before the timed loop (for rocprofv3 counter scaling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: measures one GPU only (the path would shard by candidate pose, each GPU "
              "rendering and scoring its own slice); run with --gpus 1", file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2403_11367_amd import Camera, Context, crop, default_cfg
    from paper_2403_11367_amd.gsr import RENDER_COUNT_EVALS

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    t_setup = time.perf_counter()
    sc = W.config1()
    idx = crop(sc.gaussians.means, sc.crop_cell, sc.prior_center[:2], sc.crop_radius, sc.crop_voxel)
    P = sc.poses.shape[0]
    cam = Camera(sc.camera.width, sc.camera.height, sc.camera.fx, sc.camera.fy, sc.camera.cx, sc.camera.cy)
    H, Wd = cam.height, cam.width
    ctx = Context(0)
    gmap = [torch.as_tensor(a, device=dev) for a in sc.gaussians.arrays()]
    idx_t = torch.as_tensor(idx, device=dev)
    poses_t = torch.as_tensor(sc.poses, device=dev)
    # query: render of the full (uncropped) map at the hidden pose + N(0, 0.02) noise
    full = ctx.load_submap(*gmap)
    q_rgb, _ = ctx.render(full, cam, torch.as_tensor(sc.hidden_pose[None], device=dev))
    query = (q_rgb[0] + torch.as_tensor(sc.query_noise, device=dev)).contiguous()
    full.free()
    _log(f"setup: crop {idx.size} of {sc.gaussians.n} Gaussians, {P} poses, {Wd}x{H}")

    # one counting render (untimed): exact pair total and evaluation counts of this workload
    sm = ctx.load_submap(*gmap, index=idx_t)
    tw, th = args.tile
    ctx.render(sm, cam, poses_t, default_cfg(flags=RENDER_COUNT_EVALS, pose_groups=args.pose_groups, tile_w=tw,
                                             tile_h=th))
    st0 = ctx.stats()
    n_pairs, n_vis, n_groups = st0["n_pairs"], st0["n_visible"], st0["n_groups"]
    # fixed capacity (it bounds each pose group): no host wait per step
    cfg = default_cfg(pair_capacity=int(n_pairs * 1.05) + 4096, pose_groups=args.pose_groups, tile_w=tw, tile_h=th)
    rgb = torch.empty((P, 3, H, Wd), dtype=torch.float32, device=dev)
    depth = torch.empty((P, H, Wd), dtype=torch.float32, device=dev)
    scores = torch.empty((P,), dtype=torch.float32, device=dev)
    best = torch.empty((1,), dtype=torch.int32, device=dev)

    def step():
        nonlocal sm
        sm = ctx.load_submap(*gmap, index=idx_t, into=sm)           # S0
        ctx.render(sm, cam, poses_t, cfg, rgb=rgb, depth=depth)     # S1-S5
        ctx.ncc(query, rgb, scores)                                  # S6
        ctx.topk(scores, 1, out=best)                                # S7

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.sync()
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    _log(f"setup done in {time.perf_counter() - t_setup:.1f} s; pairs {n_pairs}, visible {n_vis}")

    ctx.set_profiling(True)
    ctx.stats()  # reset the profiled-call window
    # per-step HIP events on the stream the library enqueues on (torch's current)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(args.steps):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
    med_ms = step_ms[len(step_ms) // 2] if len(step_ms) % 2 else 0.5 * (step_ms[len(step_ms) // 2 - 1] +
                                                                         step_ms[len(step_ms) // 2])
    st = ctx.stats()
    ctx.set_profiling(False)
    ctx.sync()  # raises on overflow: the timed images would be invalid
    elapsed = t1 - t0
    ms_step = elapsed / args.steps * 1e3
    cand_s = P * args.steps / elapsed
    best_i = int(best.cpu()[0])
    _log(f"timed: {args.steps} steps in {elapsed * 1e3:.1f} ms; stage means (ms): preprocess "
         f"{st['ms_preprocess']:.3f} sort/group {st['ms_sort']:.3f} blend/group {st['ms_blend']:.3f} render "
         f"{st['ms_render']:.3f} ({n_groups} groups) ncc {st['ms_ncc']:.3f}; "
         f"best candidate {best_i}")

    # roofline of the dominant kernel (blend): algorithmic flops of one launch (one
    # pose group: the render's contributions / groups) / mean launch duration
    e_contrib, e_lanes = st0["evals_contrib"], st0["evals_lanes"]
    blend_s = st["ms_blend"] * 1e-3
    flops_launch = e_contrib * FLOPS_PER_CONTRIB / n_groups
    achieved = flops_launch / blend_s / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VECTOR_PEAK, 4), "traffic": _blend_traffic(n_groups),
            "kernel": "k_blend", "ms_per_launch": round(st["ms_blend"], 4), "launches_per_render": n_groups,
            "flops_per_launch": int(flops_launch), "evals_contrib_per_render": e_contrib,
            "evals_lane_slots_per_render": e_lanes}
    # end to end against HBM with the algorithmic bytes of the whole path
    n_c, px = int(idx.size), H * Wd
    bytes_step = 52 * n_c + 60 * n_vis + 88 * n_pairs + 28 * px * P
    e2e_gbs = bytes_step / (ms_step * 1e-3) / 1e9

    out = {
        "metric": "candidate poses rendered+NCC-scored/sec @1408x376,1M Gaussians; learned vs plain",
        "value": round(cand_s, 2), "unit": "candidates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "config1: 1M-Gaussian street-corridor map, 10 m voxel / 50 m crop "
                               f"({n_c} Gaussians), {P} candidate poses, {Wd}x{H}, full-res NCC, top-1",
                   "global_batch": P, "parallelism": "single GPU", "tile": f"{tw}x{th}",
                   "path": "plain: every candidate rendered at full resolution and NCC-scored"},
        "pixels_per_s": round(cand_s * px, 1),
        "step_ms": {"mean": round(ms_step, 4), "median": round(med_ms, 4), "min": round(step_ms[0], 4),
                    "max": round(step_ms[-1], 4), "median_candidates_per_s": round(P / (med_ms * 1e-3), 1)},
        "roofline": roof,
        "e2e_hbm": {"bytes_per_step": bytes_step, "achieved_GBs": round(e2e_gbs, 1), "peak_GBs": HBM_PEAK_GBS,
                    "frac": round(e2e_gbs / HBM_PEAK_GBS, 4)},
        "stages_ms": {k: round(st[k], 4) for k in ("ms_preprocess", "ms_sort", "ms_blend", "ms_render", "ms_ncc")},
        "counts": {"n_submap": n_c, "n_visible": n_vis, "n_pairs": n_pairs, "best_candidate": best_i},
    }
    # random-order search with an early stop (Sec. IV) on the same workload: a seeded
    # order, at most 20% of the candidates in batches of 8, stopping once the best NCC
    # reaches 95% of the plain search's best
    order = W.search_order(12, P)
    s_np = scores.cpu().numpy()
    thr = float(0.95 * s_np.max())
    max_eval = max(1, int(np.ceil(0.2 * P)))
    ctx.search(sm, cam, poses_t, order, 8, max_eval, thr, query, cfg)  # warm-up (buffers)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        e_best, e_score, e_n, _ = ctx.search(sm, cam, poses_t, order, 8, max_eval, thr, query, cfg)
    torch.cuda.synchronize()
    t_s = (time.perf_counter() - t0) / reps
    out["early_stop"] = {"order_seed": 12, "share": 0.2, "batch": 8, "threshold": round(thr, 5),
                         "candidates_scored": e_n, "best": e_best, "best_ncc": round(e_score, 5),
                         "plain_best": best_i, "ms_per_search": round(t_s * 1e3, 3),
                         "scored_candidates_per_s": round(e_n / t_s, 1)}
    _log(f"early-stop search: {e_n} of {P} scored in {t_s * 1e3:.2f} ms, best {e_best} (plain {best_i})")
    if not args.no_learned:
        out["learned"] = learned_leg(ctx, sm, cam, sc, query, dev)
    if not args.no_batched:
        out["batched"] = batched_leg(ctx, cam, dev)
    if not args.no_training:
        out["training"] = training_leg(ctx, cam, dev)
    if args.cpu_candidates > 0:
        _log(f"cpu baseline: oracle on {args.cpu_candidates} candidates ...")
        out["cpu_baseline"] = cpu_baseline(sc, idx, args.cpu_candidates)
    print(json.dumps(out), flush=True)
    sm.free()
    ctx.close()


def _with(cfg, **over):
    """A copy of a render configuration with some fields replaced."""
    from paper_2403_11367_amd import default_cfg
    c = default_cfg(**{f: getattr(cfg, f) for f, _ in cfg._fields_})
    for k, v in over.items():
        setattr(c, k, v)
    return c


def batched_leg(ctx, cam, dev, reps=5):
    """Batched queries: 8 corridor maps of uneven size (batch_query seeds 200-207,
    cropped like config 1), 32 candidates each, full-resolution NCC and top-1 per
    query. The queries are grouped by submap-size bucket (powers of two); the
    autotuner picks tile shape, LDS chunk, grid or persistent launch and pose
    groups per bucket, and each bucket renders as one batched render. Times 8
    separate default renders, the per-bucket batched renders and their HIP-graph
    replay. The batched images equal separate renders with the same settings bit
    for bit; against the default 16x16 renders they differ within float32
    rounding where a bucket chose another tile shape (reported)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2403_11367_amd import autotune, crop, default_cfg

    t_setup = time.perf_counter()
    qs = [W.batch_query(s, W.config1_camera()) for s in W.BATCH_MAP_SEEDS]
    sms, queries = [], []
    for q in qs:
        arrs = [torch.as_tensor(a, device=dev) for a in q.gaussians.arrays()]
        full = ctx.load_submap(*arrs)
        img, _ = ctx.render(full, cam, torch.as_tensor(q.hidden[None], device=dev))
        queries.append((img[0] + torch.as_tensor(q.noise, device=dev)).contiguous())
        full.free()
        idx = crop(q.gaussians.means, 10.0, (100.0, 0.0), 50.0, 1.0)
        sms.append(ctx.load_submap(*arrs, index=torch.as_tensor(idx, device=dev)))
        del arrs
    # queries ordered by submap-size bucket (stable), so each bucket's poses are contiguous
    bucket_of = [autotune.size_bucket(sm.n) for sm in sms]
    order = sorted(range(len(qs)), key=lambda i: bucket_of[i])
    qs, sms, queries, bucket_of = ([x[i] for i in order] for x in (qs, sms, queries, bucket_of))
    counts = [q.poses.shape[0] for q in qs]
    P = sum(counts)
    poses = torch.as_tensor(np.concatenate([q.poses for q in qs]), device=dev)
    starts = np.concatenate([[0], np.cumsum(counts)])
    H, Wd = cam.height, cam.width
    rgb = torch.empty((P, 3, H, Wd), device=dev)
    depth = torch.empty((P, H, Wd), device=dev)
    scores = torch.empty((P,), device=dev)
    best = torch.empty((len(qs),), dtype=torch.int32, device=dev)
    # fixed pair capacities (no host wait when timed): the largest exact count over
    # the tile shapes the autotuner tries
    caps = []
    for i, sm in enumerate(sms):
        n_max = 0
        for tw, th in autotune.TILES:
            ctx.render(sm, cam, poses[starts[i]:starts[i + 1]].contiguous(), default_cfg(tile_w=tw, tile_h=th))
            n_max = max(n_max, ctx.stats()["n_pairs"])
        caps.append(int(n_max * 1.05) + 4096)
    buckets = sorted(set(bucket_of))
    groups = [[i for i in range(len(qs)) if bucket_of[i] == b] for b in buckets]
    _log(f"batched: {len(qs)} queries, maps {[q.n for q in qs]}, crops {[sm.n for sm in sms]}, buckets "
         f"{[(b, len(g)) for b, g in zip(buckets, groups)]}, setup {time.perf_counter() - t_setup:.1f} s")

    def scored(i):
        a, b = int(starts[i]), int(starts[i + 1])
        ctx.ncc(queries[i], rgb[a:b], scores[a:b])
        ctx.topk(scores[a:b], 1, out=best[i:i + 1])

    def separate(cfg_of=None):
        for i, sm in enumerate(sms):
            a, b = int(starts[i]), int(starts[i + 1])
            cfg = default_cfg(pair_capacity=caps[i]) if cfg_of is None else cfg_of(i)
            ctx.render(sm, cam, poses[a:b].contiguous(), cfg, rgb=rgb[a:b], depth=depth[a:b])
            scored(i)

    def span(g):
        return int(starts[g[0]]), int(starts[g[-1] + 1])

    tuned, records, keys = [], [], []
    for b, g in zip(buckets, groups):
        a0, a1 = span(g)
        key = autotune.workload_key(torch.cuda.get_device_name(dev), Wd, H, a1 - a0, b)
        base = default_cfg(pair_capacity=sum(caps[i] for i in g))
        cfg, record = autotune.tune(key, base, lambda cfg, g=g, a0=a0, a1=a1: ctx.render_multi(
            [sms[i] for i in g], [counts[i] for i in g], cam, poses[a0:a1], cfg, rgb=rgb[a0:a1], depth=depth[a0:a1]))
        tuned.append(cfg)
        records.append(record)
        keys.append(key)

    # for comparison: the whole batch as one render with one tuned setting (key: largest submap)
    key_one = autotune.workload_key(torch.cuda.get_device_name(dev), Wd, H, P, max(sm.n for sm in sms))
    tuned_one, record_one = autotune.tune(key_one, default_cfg(pair_capacity=sum(caps)), lambda cfg: ctx.render_multi(
        sms, counts, cam, poses, cfg, rgb=rgb, depth=depth))

    def batched_one():
        ctx.render_multi(sms, counts, cam, poses, tuned_one, rgb=rgb, depth=depth)
        for i in range(len(qs)):
            scored(i)

    def batched():
        for g, cfg in zip(groups, tuned):
            a0, a1 = span(g)
            ctx.render_multi([sms[i] for i in g], [counts[i] for i in g], cam, poses[a0:a1], cfg, rgb=rgb[a0:a1],
                             depth=depth[a0:a1])
        for i in range(len(qs)):
            scored(i)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_sep = timed(separate)
    ref_default = (rgb.clone(), depth.clone(), scores.clone(), best.clone())
    group_of = {i: k for k, g in enumerate(groups) for i in g}

    def cfg_same(i):  # query i rendered alone with its bucket's tuned settings
        return _with(tuned[group_of[i]], pair_capacity=caps[i], pose_groups=1)

    separate(cfg_same)
    torch.cuda.synchronize()
    ref = (rgb.clone(), depth.clone(), scores.clone(), best.clone())
    t_bat = timed(batched)
    same_batched = all(torch.equal(a, b) for a, b in zip((rgb, depth, scores, best), ref))
    diff_default = {"max_abs_rgb": float((rgb - ref_default[0]).abs().max()),
                    "max_abs_score": float((scores - ref_default[2]).abs().max()),
                    "same_best": bool(torch.equal(best, ref_default[3]))}
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batched()
        stream.synchronize()
        ctx.capture_begin()
        batched()
        graph = ctx.capture_end()
        rgb.zero_()
        graph.launch()
        stream.synchronize()
        same_graph = all(torch.equal(a, b) for a, b in zip((rgb, depth, scores, best), ref))
        t_graph = timed(graph.launch)
        graph.close()
        # the single-setting batch and its graph
        separate(lambda i: _with(tuned_one, pair_capacity=caps[i], pose_groups=1))
        stream.synchronize()
        ref_one = (rgb.clone(), depth.clone(), scores.clone(), best.clone())
        t_one = timed(batched_one)
        same_one = all(torch.equal(a, b) for a, b in zip((rgb, depth, scores, best), ref_one))
        ctx.capture_begin()
        batched_one()
        graph = ctx.capture_end()
        rgb.zero_()
        graph.launch()
        stream.synchronize()
        same_one_graph = all(torch.equal(a, b) for a, b in zip((rgb, depth, scores, best), ref_one))
        t_one_graph = timed(graph.launch)
        graph.close()
    ctx.sync()
    knobs = ("tile_w", "tile_h", "blend_chunk", "blend_blocks_per_cu", "pose_groups")
    res = {"queries": len(qs), "poses_per_query": counts[0], "renders": P,
           "map_gaussians": [q.n for q in qs], "submap_gaussians": [sm.n for sm in sms],
           "separate": {"ms": round(t_sep * 1e3, 3), "renders_per_s": round(P / t_sep, 1)},
           "batched": {"ms": round(t_bat * 1e3, 3), "renders_per_s": round(P / t_bat, 1),
                       "identical_to_separate_same_settings": bool(same_batched),
                       "against_default_separate": diff_default},
           "graph": {"ms": round(t_graph * 1e3, 3), "renders_per_s": round(P / t_graph, 1),
                     "identical_to_separate_same_settings": bool(same_graph)},
           "one_batch_one_setting": {
               "key": key_one, "chosen": {f: getattr(tuned_one, f) for f in knobs},
               "ms": round(t_one * 1e3, 3), "renders_per_s": round(P / t_one, 1),
               "graph_ms": round(t_one_graph * 1e3, 3), "graph_renders_per_s": round(P / t_one_graph, 1),
               "identical_to_separate_same_settings": bool(same_one and same_one_graph)},
           "autotune": [{"key": k, "bucket": b, "queries": len(g),
                         "chosen": {f: getattr(c, f) for f in knobs},
                         "launch": "persistent queue" if c.blend_blocks_per_cu > 0 else "grid",
                         "variants_ms": r.get("variants", "cached")[:6] if r else "cached"}
                        for k, b, g, c, r in zip(keys, buckets, groups, tuned, records)],
           "best_per_query": best.cpu().tolist()}
    for sm in sms:
        sm.free()
    _log(f"batched: separate {res['separate']['ms']:.2f} ms, per-bucket batched {res['batched']['ms']:.2f} ms, "
         f"graph {res['graph']['ms']:.2f} ms for {P} renders; chosen per bucket "
         f"{[(a['bucket'], a['chosen']) for a in res['autotune']]}; one batch, one setting "
         f"{res['one_batch_one_setting']['ms']:.2f} ms, graph {res['one_batch_one_setting']['graph_ms']:.2f} ms, "
         f"chosen {res['one_batch_one_setting']['chosen']}")
    return res


def training_leg(ctx, cam, dev, steps=8, warmup=2):
    """Map-training step (500,000-Gaussian corridor map, seed 3, perturbed; 4 views at
    1408x376 per step; L1 on colour + 0.1 x L1 on 5%-valid LiDAR depth; Adam): the
    library's forward and backward through torch.autograd, timed per step."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2403_11367_amd import train

    tm = W.training_map(500_000)
    data = train.make_training_data(ctx, tm.gt, cam, n_steps=steps + warmup, views=4, seed=33)
    res = {"gaussians": 500_000, "views_per_step": 4, "image": f"{cam.width}x{cam.height}"}
    # kept compositing states (the default) and the backward that recomputes every
    # list's transmittance from its front, each from the same initial map
    for mode, keep in (("kept_states", True), ("recompute", False)):
        tr = train.MapTrainer(ctx, cam, tm.means, tm.log_scales, tm.quats, tm.logits, tm.rgb, keep_state=keep)
        losses = []
        for s in range(warmup):
            losses.append(float(tr.step(data.poses[s], data.rgb[s], data.lidar[s], data.mask[s])))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = [tr.step(data.poses[s], data.rgb[s], data.lidar[s], data.mask[s]) for s in range(warmup, warmup + steps)]
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        losses += [float(x) for x in out]
        tr.close()
        res[mode] = {"ms_per_step": round(t * 1e3, 3), "views_per_s": round(4 / t, 1),
                     "loss_first": round(losses[0], 5), "loss_last": round(losses[-1], 5)}
        _log(f"training ({mode}): {t * 1e3:.2f} ms per step of 4 views, loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    res["ms_per_step"] = res["kept_states"]["ms_per_step"]
    return res


def learned_leg(ctx, sm, cam, sc, query, dev, k=16, reps=5, recall_queries=24):
    """Learned vs plain on the same submap and query: 1024 candidates (8 dx x 8 dy
    x 16 dyaw at 1 m / 1 m / 5 degrees around the prior). Plain renders and scores
    all of them at full resolution; the pruned searches render all at a quarter of
    the resolution, predict (trained scorer, or low-resolution NCC), and decide
    among the k best by full-resolution NCC. Renders use exact pair buffers."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2403_11367_amd import Camera, Scorer, learned

    poses = torch.as_tensor(W.yaw_grid_poses(sc.prior_center, W.AXES_ALONG_X, W.SCORER_DX, W.SCORER_DY,
                                             W.SCORER_DYAW), device=dev)
    P = poses.shape[0]
    lc = W.low_res_camera(W.config1_camera(), W.SCORER_FACTOR)
    cam_low = Camera(lc.width, lc.height, lc.fx, lc.fy, lc.cx, lc.cy)
    scorer = Scorer(ctx, lc.height, lc.width, 256)
    scorer.set_params(torch.as_tensor(learned.load_weights(), device=dev))
    best_t = torch.empty((1,), dtype=torch.int32, device=dev)

    def plain():
        s = learned.exhaustive_ncc(ctx, sm, cam, poses, query)
        ctx.topk(s, 1, out=best_t)
        return s

    def timed(fn):
        r = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) / reps

    s_plain, t_plain = timed(plain)
    s_np = s_plain.cpu().numpy()
    best = int(np.argmax(s_np))
    res = {"candidates": P, "k": k, "low_res": f"{lc.width}x{lc.height}",
           "plain": {"ms": round(t_plain * 1e3, 3), "candidates_per_s": round(P / t_plain, 1), "best": best,
                     "best_ncc": round(float(s_np[best]), 5)}}
    for name, net in (("learned", scorer), ("lowres_ncc", None)):
        (b, bs, pred, top, ncc), t = timed(lambda net=net: ctx.search_pruned(sm, cam, cam_low, poses, query, k,
                                                                           scorer=net))
        res[name] = {"ms": round(t * 1e3, 3), "candidates_per_s": round(P / t, 1), "best": b,
                     "best_ncc": round(bs, 5), "found_plain_best": b == best,
                     "speedup_vs_plain": round(t_plain / t, 3)}
    # top-5 recall of the exhaustive NCC best on held-out queries (a map the scorer
    # was not trained on), measured here
    with contextlib.redirect_stdout(sys.stderr):  # its progress lines; stdout carries only the JSON line
        ev = learned.evaluate(ctx, scorer, [W.SCORER_EVAL_MAPS[0]], recall_queries, k=k, reps=1)
    res["recall"] = {"queries": ev["queries"], "map_seed": W.SCORER_EVAL_MAPS[0],
                     "top5_recall_learned": ev["top5_recall_learned"],
                     "top5_recall_lowres_ncc": ev["top5_recall_lowres"],
                     "median_rank_of_best_learned": ev["median_rank_of_best_learned"],
                     "max_rank_of_best_learned": ev["max_rank_of_best_learned"],
                     "median_rank_of_best_lowres_ncc": ev["median_rank_of_best_lowres"],
                     "max_rank_of_best_lowres_ncc": ev["max_rank_of_best_lowres"],
                     "ms_per_query": {"plain": ev["ms_per_query_plain"], "learned": ev["ms_per_query_learned"],
                                      "lowres_ncc": ev["ms_per_query_lowres"]}}
    res["learned_vs_lowres_ncc"] = round(res["lowres_ncc"]["ms"] / res["learned"]["ms"], 3)
    scorer.close()
    _log(f"learned vs plain ({P} candidates): plain {res['plain']['ms']:.1f} ms, learned "
         f"{res['learned']['ms']:.1f} ms, low-res NCC {res['lowres_ncc']['ms']:.1f} ms; top-5 recall on "
         f"{ev['queries']} held-out queries: learned {ev['top5_recall_learned']}, low-res NCC "
         f"{ev['top5_recall_lowres']}")
    return res


if __name__ == "__main__":
    main()
