"""Map training through the renderer: a torch.autograd.Function around
gsr_render / gsr_render_backward, and the map-training step of a LiDAR-initialised
Gaussian map (the paper builds its map by optimising the Gaussians against camera
images, Sec. III-B).

Parameters are means, log-scales, raw quaternions, opacity logits and colours;
torch maps log-scales and logits to the linear scales and opacities the library
takes (exp, sigmoid) and chains their gradients. The library renders and
differentiates; torch holds the tensors, computes the loss and runs Adam.
"""
from __future__ import annotations

import copy
import dataclasses

import numpy as np


def _torch():
    import torch
    return torch


class _SubmapSlot:
    """The submap a training render loads its parameters into (reused)."""

    def __init__(self):
        self.sm = None


def _render_function():
    torch = _torch()

    class RenderFunction(torch.autograd.Function):
        """(means, scales, quats, opacity, rgb) -> (rgb images [P,3,H,W], depth [P,H,W])."""

        @staticmethod
        def forward(fctx, means, scales, quats, opacity, colours, ctx, slot, camera, poses, cfg, keep_state):
            from .gsr import RENDER_KEEP_STATE, default_cfg
            args = [t.detach().contiguous() for t in (means, scales, quats, opacity, colours)]
            slot.sm = ctx.load_submap(*args, into=slot.sm)
            cfg = default_cfg() if cfg is None else copy.copy(cfg)
            if keep_state:
                # keep the long lists' compositing states, so that the backward walks
                # them in segments (without: each list is one serial walk that
                # recomputes its transmittance from the front)
                cfg.flags |= RENDER_KEEP_STATE
            img, depth = ctx.render(slot.sm, camera, poses, cfg)
            fctx.ctx, fctx.sm = ctx, slot.sm
            fctx.serial = ctx.stats()["render_serial"]
            fctx.save_for_backward(args[1], args[2], poses, img, depth)
            return img, depth

        @staticmethod
        def backward(fctx, g_img, g_depth):
            scales, quats, poses, img, depth = fctx.saved_tensors
            if fctx.ctx.stats()["render_serial"] != fctx.serial:
                raise RuntimeError("another render ran on this context between forward and backward")
            g_img = torch.zeros_like(img) if g_img is None else g_img.contiguous()
            g_depth = torch.zeros_like(depth) if g_depth is None else g_depth.contiguous()
            gm, gs, gq, go, gc = fctx.ctx.render_backward(fctx.sm, scales, quats, poses, img, depth, g_img, g_depth)
            return gm, gs, gq, go, gc, None, None, None, None, None, None

    return RenderFunction


_FN = None


def render(ctx, slot: _SubmapSlot, means, scales, quats, opacity, colours, camera, poses, cfg=None,
           keep_state: bool = True):
    """Differentiable render of all Gaussians at `poses`: (rgb, depth). keep_state:
    the forward keeps the compositing state every 2016 records of a long list
    (GSR_RENDER_KEEP_STATE) and the backward walks such lists in segments;
    without it the backward recomputes each list's transmittance in one walk
    from the front."""
    global _FN
    if _FN is None:
        _FN = _render_function()
    return _FN.apply(means, scales, quats, opacity, colours, ctx, slot, camera, poses, cfg, keep_state)


@dataclasses.dataclass
class TrainData:
    poses: object        # [S, V, 3, 4] views per step
    rgb: object          # [S, V, 3, H, W] targets
    lidar: object        # [S, V, H, W] depth at the valid pixels
    mask: object         # [S, V, H, W] 1 where the LiDAR depth is valid


class MapTrainer:
    """Optimises a Gaussian map against target images and sparse LiDAR depth:
    loss = mean |rgb - target| + depth_weight * mean over valid pixels |depth - lidar|."""

    def __init__(self, ctx, camera, means, log_scales, quats, logits, colours, lr=None, depth_weight=0.1,
                 keep_state: bool = True):
        torch = _torch()
        self.ctx, self.camera, self.depth_weight = ctx, camera, depth_weight
        self.keep_state = keep_state
        dev = torch.device("cuda", ctx.device)
        mk = lambda a: torch.nn.Parameter(torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev))  # noqa
        self.means, self.log_scales, self.quats = mk(means), mk(log_scales), mk(quats)
        self.logits, self.colours = mk(logits), mk(colours)
        lr = lr or dict(means=1e-3, log_scales=5e-3, quats=1e-3, logits=2e-2, colours=5e-3)
        self.opt = torch.optim.Adam([{"params": [getattr(self, k)], "lr": v} for k, v in lr.items()], eps=1e-15)
        self.slot = _SubmapSlot()

    def params(self):
        return self.means, self.log_scales, self.quats, self.logits, self.colours

    def loss(self, poses, target_rgb, lidar, mask, cfg=None):
        torch = _torch()
        img, depth = render(self.ctx, self.slot, self.means, torch.exp(self.log_scales), self.quats,
                            torch.sigmoid(self.logits), self.colours, self.camera, poses, cfg, self.keep_state)
        l_rgb = (img - target_rgb).abs().mean()
        l_depth = ((depth - lidar).abs() * mask).sum() / mask.sum().clamp(min=1)
        return l_rgb + self.depth_weight * l_depth

    def step(self, poses, target_rgb, lidar, mask, cfg=None):
        self.opt.zero_grad(set_to_none=True)
        loss = self.loss(poses, target_rgb, lidar, mask, cfg)
        loss.backward()
        self.opt.step()
        return loss.detach()

    def close(self):
        if self.slot.sm is not None:
            self.slot.sm.free()
            self.slot.sm = None


def make_training_data(ctx, gt, camera, n_steps: int, views: int, seed: int, valid: float = 0.05,
                       mask_seed: int = 31, length: float = 200.0):
    """Views, target images (renders of the ground-truth map) and sparse LiDAR depth
    (the ground-truth depth at a `valid` share of the pixels) for n_steps steps of
    `views` views (poses from workloads.training_views along a corridor of `length`)."""
    torch = _torch()
    import workloads as W
    dev = torch.device("cuda", ctx.device)
    poses = torch.as_tensor(W.training_views(seed, n_steps * views, length), device=dev).reshape(n_steps, views, 3, 4)
    arrs = [torch.as_tensor(a, device=dev) for a in gt.arrays()]
    sm = ctx.load_submap(*arrs)
    rgbs, depths = [], []
    for s in range(n_steps):
        img, dep = ctx.render(sm, camera, poses[s].contiguous())
        rgbs.append(img)
        depths.append(dep)
    sm.free()
    H, Wd = camera.height, camera.width
    mrng = np.random.default_rng(mask_seed)
    mask = torch.as_tensor((mrng.random((n_steps, views, H, Wd)) < valid).astype(np.float32), device=dev)
    depth = torch.stack(depths)
    return TrainData(poses, torch.stack(rgbs), depth * mask, mask)
