"""Learned candidate pruning: training data made by the renderer, training of
the scorer (include/gsr_scorer.h) on the GPU, and evaluation against the
exhaustive NCC search of Sec. III-C1.

Per query, every candidate of a 1024-pose grid is rendered at full resolution
and scored by NCC (Eq. 10): that NCC is the label, and its argmax the pose the
pruned search must keep. The scorer sees the candidate's render at a quarter of
the resolution and the equally pooled query, and predicts the NCC. The pruned
search (gsr_search_pruned) keeps the k best predictions and decides among them
by full-resolution NCC; top-5 recall is the share of queries whose exhaustive
best is among the pruned search's five best. The same search with low-resolution
NCC in place of the network is the comparison without the network.

    python -m paper_2403_11367_amd.learned train --out DIR [--epochs N]
    python -m paper_2403_11367_amd.learned eval --weights DIR/scorer.npy

All computation runs in libgsr; torch holds device memory and shuffles the
training pairs (index gathers).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(_HERE, "weights", "scorer.npy")


def _log(msg: str):
    print(msg, flush=True)


def _camera(c):
    from .gsr import Camera
    return Camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy)


class DeviceMap:
    """A corridor map on the device: the full map (for query renders) and the
    crop around each prior (gsr_crop, host)."""

    def __init__(self, ctx, gaussians):
        import torch
        self.ctx = ctx
        self.host_means = gaussians.means
        dev = torch.device("cuda", ctx.device)
        self.arrays = [torch.as_tensor(a, device=dev) for a in gaussians.arrays()]
        self.full = ctx.load_submap(*self.arrays)
        self.sub = None

    def crop(self, prior, cell=10.0, radius=50.0, voxel=1.0):
        import torch
        from .gsr import crop
        idx = crop(self.host_means, cell, prior[:2], radius, voxel)
        self.sub = self.ctx.load_submap(*self.arrays, index=torch.as_tensor(idx, device=self.arrays[0].device),
                                        into=self.sub)
        return self.sub

    def free(self):
        for s in (self.full, self.sub):
            if s is not None:
                s.free()


def render_query(ctx, dmap: DeviceMap, cam, q):
    """Query image: render of the full map at the hidden pose plus the query noise."""
    import torch
    dev = dmap.arrays[0].device
    rgb, _ = ctx.render(dmap.full, cam, torch.as_tensor(q.hidden[None], device=dev))
    return (rgb[0] + torch.as_tensor(q.noise, device=dev)).contiguous()


def exhaustive_ncc(ctx, sm, cam, poses_t, query, batch=128, out=None):
    """NCC of every candidate at full resolution (the labels and the final ranking)."""
    import torch
    P = poses_t.shape[0]
    if out is None:
        out = torch.empty((P,), dtype=torch.float32, device=poses_t.device)
    for b0 in range(0, P, batch):
        b1 = min(P, b0 + batch)
        rgb, _ = ctx.render(sm, cam, poses_t[b0:b1].contiguous())
        ctx.ncc(query, rgb, out[b0:b1])
    return out


def scorer_inputs(ctx, scorer, sm, cam_low, poses_t, query_grey, x_out, batch=256):
    """Network inputs of every candidate (low-resolution render + pooled query)."""
    P = poses_t.shape[0]
    for b0 in range(0, P, batch):
        b1 = min(P, b0 + batch)
        rgb, _ = ctx.render(sm, cam_low, poses_t[b0:b1].contiguous())
        scorer.inputs(rgb, query_grey, out=x_out[b0:b1])


@dataclasses.dataclass
class PairSet:
    x: object          # torch bfloat16 [N, h, w, 2]
    labels: object     # torch float32 [N]
    n_queries: int


def generate(ctx, scorer, map_seeds, per_map, n_gauss=1_000_000):
    """Training pairs of per_map queries on each map seed."""
    import torch
    import workloads as W
    wcam = W.config1_camera()
    cam, cam_low = _camera(wcam), _camera(W.low_res_camera(wcam, W.SCORER_FACTOR))
    n_cand = len(W.SCORER_DX) * len(W.SCORER_DY) * len(W.SCORER_DYAW)
    N = len(map_seeds) * per_map * n_cand
    dev = torch.device("cuda", ctx.device)
    x = torch.empty((N, cam_low.height, cam_low.width, 2), dtype=torch.bfloat16, device=dev)
    labels = torch.empty((N,), dtype=torch.float32, device=dev)
    row = 0
    for ms in map_seeds:
        t0 = time.perf_counter()
        dmap = DeviceMap(ctx, W.corridor_map(n_gauss, seed=ms))
        _log(f"map {ms}: {time.perf_counter() - t0:.1f} s")
        for i in range(per_map):
            t1 = time.perf_counter()
            q = W.scorer_query(W.scorer_query_seed(ms, i), wcam)
            poses_t = torch.as_tensor(q.poses, device=dev)
            sm = dmap.crop(q.prior)
            query = render_query(ctx, dmap, cam, q)
            exhaustive_ncc(ctx, sm, cam, poses_t, query, out=labels[row:row + n_cand])
            qg = ctx.pool_grey(query[None].contiguous(), W.SCORER_FACTOR)[0]
            scorer_inputs(ctx, scorer, sm, cam_low, poses_t, qg, x[row:row + n_cand])
            torch.cuda.synchronize()
            lab = labels[row:row + n_cand]
            _log(f"  query {ms}/{i}: best NCC {float(lab.max()):.3f}, mean {float(lab.mean()):.3f} "
                 f"({time.perf_counter() - t1:.2f} s)")
            row += n_cand
        dmap.free()
    return PairSet(x, labels, len(map_seeds) * per_map)


def train(scorer, data: PairSet, epochs=8, batch=256, lr=1e-3, weight_decay=1e-4, seed=0):
    """AdamW on the mean squared error between predicted and full-resolution NCC,
    shuffled pairs, cosine learning-rate decay. Returns the mean loss per epoch."""
    import torch
    N = data.labels.shape[0]
    steps_per_epoch = N // batch
    total = epochs * steps_per_epoch
    gen = torch.Generator(device=data.labels.device)
    gen.manual_seed(seed)
    loss = torch.zeros((1,), dtype=torch.float32, device=data.labels.device)
    acc = torch.zeros((1,), dtype=torch.float32, device=data.labels.device)
    history = []
    step = 0
    for e in range(epochs):
        t0 = time.perf_counter()
        perm = torch.randperm(N, device=data.labels.device, generator=gen)
        acc.zero_()
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            xb = data.x.index_select(0, idx)
            lb = data.labels.index_select(0, idx)
            cur = 0.5 * lr * (1 + math.cos(math.pi * step / total))
            scorer.train_step(xb, lb, scorer.adamw_cfg(lr=cur, weight_decay=weight_decay), loss=loss)
            acc += loss
            step += 1
        torch.cuda.synchronize()
        history.append(float(acc) / steps_per_epoch)
        _log(f"epoch {e}: loss {history[-1]:.5f} ({time.perf_counter() - t0:.1f} s)")
    return history


def evaluate(ctx, scorer, map_seeds, per_map, k=16, n_gauss=1_000_000, reps=3):
    """Top-5 recall of the exhaustive NCC best, for the learned and the low-resolution
    NCC pruning, and the time of each search per query (mean of `reps` runs)."""
    import torch
    import workloads as W
    wcam = W.config1_camera()
    cam, cam_low = _camera(wcam), _camera(W.low_res_camera(wcam, W.SCORER_FACTOR))
    dev = torch.device("cuda", ctx.device)
    rows = []
    for ms in map_seeds:
        dmap = DeviceMap(ctx, W.corridor_map(n_gauss, seed=ms))
        for i in range(per_map):
            q = W.scorer_query(W.scorer_query_seed(ms, i), wcam)
            poses_t = torch.as_tensor(q.poses, device=dev)
            sm = dmap.crop(q.prior)
            query = render_query(ctx, dmap, cam, q)
            res = {}

            def timed(fn):
                fn()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    r = fn()
                torch.cuda.synchronize()
                return r, (time.perf_counter() - t0) / reps

            scores, res["t_plain"] = timed(lambda: exhaustive_ncc(ctx, sm, cam, poses_t, query))
            s = scores.cpu().numpy()
            best = int(np.argmax(s))  # ties: first
            for name, sc in (("learned", scorer), ("lowres", None)):
                (b, bs, pred, top, ncc), t = timed(
                    lambda sc=sc: ctx.search_pruned(sm, cam, cam_low, poses_t, query, k, scorer=sc))
                order = np.lexsort((top.cpu().numpy(), -ncc.cpu().numpy()))
                final = top.cpu().numpy()[order]
                p = pred.cpu().numpy()
                res[f"t_{name}"] = t
                res[f"hit5_{name}"] = bool(best in final[:5])
                res[f"rank_{name}"] = int(np.sum(p > p[best]))  # candidates predicted above the best
            rows.append(res)
            _log(f"  eval {ms}/{i}: best {best} NCC {s[best]:.3f}; learned rank {res['rank_learned']} "
                 f"hit {res['hit5_learned']}; low-res rank {res['rank_lowres']} hit {res['hit5_lowres']}; "
                 f"ms plain {res['t_plain'] * 1e3:.1f} learned {res['t_learned'] * 1e3:.1f} "
                 f"low-res {res['t_lowres'] * 1e3:.1f}")
        dmap.free()
    n_cand = len(W.SCORER_DX) * len(W.SCORER_DY) * len(W.SCORER_DYAW)
    out = {"queries": len(rows), "candidates_per_query": n_cand, "k": k}
    for name in ("plain", "learned", "lowres"):
        t = float(np.mean([r[f"t_{name}"] for r in rows]))
        out[f"ms_per_query_{name}"] = round(t * 1e3, 3)
        out[f"candidates_per_s_{name}"] = round(n_cand / t, 1)
    for name in ("learned", "lowres"):
        out[f"top5_recall_{name}"] = float(np.mean([r[f"hit5_{name}"] for r in rows]))
        out[f"median_rank_of_best_{name}"] = float(np.median([r[f"rank_{name}"] for r in rows]))
        out[f"max_rank_of_best_{name}"] = int(np.max([r[f"rank_{name}"] for r in rows]))
    return out


def load_weights(path=WEIGHTS) -> np.ndarray:
    return np.load(path, allow_pickle=False).astype(np.float32)


def main(argv=None):
    import torch
    import workloads as W
    from .gsr import Context, Scorer
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--out", required=True)
    tr.add_argument("--epochs", type=int, default=8)
    tr.add_argument("--lr", type=float, default=1e-3)
    tr.add_argument("--init-seed", type=int, default=0)
    tr.add_argument("--queries-per-map", type=int, default=W.SCORER_QUERIES_PER_TRAIN_MAP)
    tr.add_argument("--eval-queries-per-map", type=int, default=W.SCORER_QUERIES_PER_EVAL_MAP)
    ev = sub.add_parser("eval")
    ev.add_argument("--weights", default=WEIGHTS)
    ev.add_argument("--queries-per-map", type=int, default=W.SCORER_QUERIES_PER_EVAL_MAP)
    ev.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    ctx = Context(0)
    h, w = 376 // W.SCORER_FACTOR, 1408 // W.SCORER_FACTOR
    scorer = Scorer(ctx, h, w, 256)
    summary = {}
    if a.cmd == "train":
        os.makedirs(a.out, exist_ok=True)
        scorer.set_params(torch.as_tensor(W.scorer_params(a.init_seed), device=f"cuda:{ctx.device}"))
        t0 = time.perf_counter()
        data = generate(ctx, scorer, W.SCORER_TRAIN_MAPS, a.queries_per_map)
        summary["pairs"] = int(data.labels.shape[0])
        summary["generate_s"] = round(time.perf_counter() - t0, 1)
        t0 = time.perf_counter()
        summary["loss_per_epoch"] = train(scorer, data, epochs=a.epochs, lr=a.lr, seed=a.init_seed)
        summary["train_s"] = round(time.perf_counter() - t0, 1)
        summary.update(epochs=a.epochs, lr=a.lr, batch=256, weight_decay=1e-4, init_seed=a.init_seed,
                       train_maps=list(W.SCORER_TRAIN_MAPS), queries_per_map=a.queries_per_map)
        del data
        params = scorer.get_params().cpu().numpy()
        np.save(os.path.join(a.out, "scorer.npy"), params)
        n_eval = a.eval_queries_per_map
        out_file = os.path.join(a.out, "summary.json")
    else:
        scorer.set_params(torch.as_tensor(load_weights(a.weights), device=f"cuda:{ctx.device}"))
        n_eval = a.queries_per_map
        out_file = a.out
    if n_eval > 0:
        summary["eval"] = evaluate(ctx, scorer, W.SCORER_EVAL_MAPS, n_eval)
        summary["eval_maps"] = list(W.SCORER_EVAL_MAPS)
    _log(json.dumps(summary))
    if out_file:
        with open(out_file, "w") as f:
            json.dump(summary, f, indent=1)
    scorer.close()
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
