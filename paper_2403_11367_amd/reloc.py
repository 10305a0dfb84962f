"""Initial relocalisation driver (Sec. III-C1): prior pose -> submap -> render
every candidate pose -> NCC against the query -> best candidates.

The submap crop is host code (gsr_crop); render, NCC and selection run in
the HIP library on the current torch stream.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .gsr import Camera, Context, RenderCfg, Submap, crop


@dataclasses.dataclass
class SearchResult:
    best: int              # index of the best candidate (ties -> lowest index)
    top: np.ndarray        # top-k candidate indices, best first
    scores: np.ndarray     # NCC of every candidate, float32


class Relocalizer:
    """Holds a map on the GPU and runs the brute-force NCC search around priors."""

    def __init__(self, ctx: Context, means, scales, quats, opacity, rgb):
        import torch
        self.ctx = ctx
        self.host_means = np.ascontiguousarray(means, dtype=np.float32)
        dev = torch.device("cuda", ctx.device)
        as_dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev)  # noqa: E731
        self.map = [as_dev(a) for a in (means, scales, quats, opacity, rgb)]
        self.submap: Optional[Submap] = None

    def select_submap(self, prior_xy, radius: float, cell: float, voxel: float = 1.0):
        """Crop (host) + pack (device): the submap nearest the prior."""
        import torch
        idx = crop(self.host_means, cell, prior_xy, radius, voxel)
        index = torch.as_tensor(idx, device=self.map[0].device)
        self.submap = self.ctx.load_submap(*self.map, index=index, into=self.submap)
        return idx.size

    def search(self, camera: Camera, poses, query, k: int = 1, cfg: Optional[RenderCfg] = None) -> SearchResult:
        rgb, _ = self.ctx.render(self.submap, camera, poses, cfg)
        scores = self.ctx.ncc(query, rgb)
        top = self.ctx.topk(scores, k)
        s = scores.cpu().numpy()
        t = top.cpu().numpy()
        return SearchResult(int(t[0]), t, s)

    def search_random(self, camera: Camera, poses, query, order, share: float = 0.2, batch: int = 8,
                      threshold: float = 0.9, cfg: Optional[RenderCfg] = None):
        """Random-order search with an early stop (Sec. IV): candidates in `order`,
        `batch` at a time, over at most `share` of them, stopping once the best NCC
        reaches `threshold`. Returns (best candidate, its NCC, candidates scored)."""
        P = poses.shape[0]
        max_eval = max(1, min(P, int(np.ceil(share * P))))
        best, score, n, _ = self.ctx.search(self.submap, camera, poses, order, batch, max_eval, threshold,
                                            query, cfg)
        return best, score, n
