"""Float64 renderer for gradient checks (oracle; test infrastructure only).

The forward of Sec. III-A (Eq. 1-5) with the readings of the float32 pipeline
(dilation eps, near plane, Jacobian clamp, 3-sigma support, alpha floor and
clamp, include-then-stop at t_min), evaluated in float64 throughout and per
pixel by brute force: every visible Gaussian whose support contains the pixel
centre, in (camera depth, index) order. Parameters are those a map-training
step optimises: means, log-scales, raw quaternions (w, x, y, z; normalised
inside), opacity logits and colours.

Gradients are central differences of a linear functional of the images,
L = sum(w_rgb * rgb) + sum(w_depth * depth), with respect to one parameter at a
time. Only the pixels whose contributing list can change are re-rendered. A
parameter is excluded ("unstable") when its +-h stencil changes any pixel's
contributing list or order, or when one of the Gaussian's decisions lies within
a float32-sized margin of its threshold (there the float32 renderer may decide
the other way and no gradient is defined).
"""
from __future__ import annotations

import dataclasses

import numpy as np

EPS = 0.3
Z_NEAR = 0.2
JAC_CLAMP = 1.3
CUTOFF = 9.0
ALPHA_MIN = float(np.float32(1.0 / 255.0))
ALPHA_MAX = 0.99
T_MIN = 1e-4
# decision margins within which a float32 evaluation may flip (relative / absolute).
# The float32 conic is the inverse of the screen covariance with det = a c - b^2
# formed in float32: its relative error is up to about (2 cond + 3) u, u = 2^-24,
# cond = a c / det. A footprint is flagged where that exceeds 1e-4, a tenth of the
# gradient bar (cond > 800): there the float32 footprint itself, not only its
# decisions, departs from the float64 one by more than the bar can absorb. (Seen
# from a street, the flat map disks are elongated but mostly axis-aligned on
# screen, which keeps cond near 1: at most 12 over a 1408x376 view.)
M_COND = 1.0 / 800.0  # flag det < M_COND a c
M_D2 = 2e-5        # |d^2 - cutoff| / cutoff
M_ALPHA = 1e-5     # |alpha - alpha_min| / alpha_min, |o G - alpha_max| / alpha_max
M_T = 1e-6         # |T - t_min| / t_min
M_RECT = 1e-4      # pixel centre within this of the 3-sigma rectangle edge (pixels)


@dataclasses.dataclass
class Params:
    means: np.ndarray       # [N, 3]
    log_scales: np.ndarray  # [N, 3]
    quats: np.ndarray       # [N, 4] (w, x, y, z), not necessarily unit
    logits: np.ndarray      # [N]
    rgb: np.ndarray         # [N, 3]

    def copy(self) -> "Params":
        return Params(*(a.copy() for a in (self.means, self.log_scales, self.quats, self.logits, self.rgb)))

    def field(self, k: int):
        """(array, row-shape) of parameter group k in the order means, log_scales,
        quats, logits, rgb."""
        return (self.means, self.log_scales, self.quats, self.logits, self.rgb)[k]


def as_params(g) -> Params:
    """From a Gaussians set with linear scales and post-sigmoid opacities."""
    f = lambda a: np.asarray(a, dtype=np.float64)  # noqa: E731
    op = f(g.opacity)
    return Params(f(g.means).copy(), np.log(f(g.scales)), f(g.quats).copy(), np.log(op / (1.0 - op)), f(g.rgb).copy())


def rotation(q):
    """Rotation matrices [N, 3, 3] of quaternions q [N, 4] (w, x, y, z), normalised."""
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


@dataclasses.dataclass
class Screen:
    visible: np.ndarray  # [N] bool
    u: np.ndarray
    v: np.ndarray
    z: np.ndarray
    conic: np.ndarray    # [N, 3] (A, B, C)
    opacity: np.ndarray
    rgb: np.ndarray      # [N, 3]
    rect: np.ndarray     # [N, 4] (x_lo, x_hi, y_lo, y_hi) support box in pixel-centre coordinates
    margin: np.ndarray   # [N] bool: a culling decision is within its margin
    cond: np.ndarray     # [N] a c / det of the screen covariance (>= 1)


def project(p: Params, pose, cam) -> Screen:
    """Eq. 3-4 in float64 for every Gaussian at one pose."""
    R, t = np.asarray(pose, np.float64)[:, :3], np.asarray(pose, np.float64)[:, 3]
    Rq = rotation(p.quats)
    M = Rq * np.exp(p.log_scales)[:, None, :]
    S = M @ np.transpose(M, (0, 2, 1))
    tc = p.means @ R.T + t
    tz = tc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        xt, yt = tc[:, 0] / tz, tc[:, 1] / tz
        lx = JAC_CLAMP * (0.5 * cam.width) / cam.fx
        ly = JAC_CLAMP * (0.5 * cam.height) / cam.fy
        xc, yc = np.clip(xt, -lx, lx), np.clip(yt, -ly, ly)
        J = np.zeros((len(tz), 2, 3))
        J[:, 0, 0] = cam.fx / tz
        J[:, 0, 2] = -cam.fx * xc / tz
        J[:, 1, 1] = cam.fy / tz
        J[:, 1, 2] = -cam.fy * yc / tz
        T = J @ R
        S2 = T @ S @ np.transpose(T, (0, 2, 1))
        a, b, c = S2[:, 0, 0] + EPS, S2[:, 0, 1], S2[:, 1, 1] + EPS
        det = a * c - b * b
        conic = np.stack([c / det, -b / det, a / det], 1)
        u, v = cam.fx * xt + cam.cx, cam.fy * yt + cam.cy
        rx, ry = 3.0 * np.sqrt(a), 3.0 * np.sqrt(c)
    vis = (tz > Z_NEAR) & (det > 0) & np.isfinite(u) & np.isfinite(v) & np.isfinite(rx) & np.isfinite(ry)
    rect = np.stack([u - rx, u + rx, v - ry, v + ry], 1)
    margin = np.abs(tz - Z_NEAR) < 1e-6 * Z_NEAR
    with np.errstate(invalid="ignore"):
        margin |= det < M_COND * np.abs(a * c)
    op = 1.0 / (1.0 + np.exp(-p.logits))
    with np.errstate(divide="ignore", invalid="ignore"):
        cond = np.where(det > 0, a * c / det, np.inf)
    return Screen(vis, u, v, tz, conic, op, p.rgb, rect, margin, cond)


def _pixel(scr: Screen, cand: np.ndarray, px: float, py: float):
    """Composite one pixel centre over candidate Gaussians (indices); returns
    (rgb, depth, contributing indices in order, margin flag)."""
    if cand.size == 0:
        return np.zeros(3), 0.0, cand, False
    order = cand[np.lexsort((cand, scr.z[cand]))]
    dx, dy = px - scr.u[order], py - scr.v[order]
    A, B, C = scr.conic[order, 0], scr.conic[order, 1], scr.conic[order, 2]
    d2 = A * dx * dx + 2 * B * dx * dy + C * dy * dy
    g = scr.opacity[order] * np.exp(-0.5 * d2)
    alpha = np.minimum(ALPHA_MAX, g)
    take = (d2 <= CUTOFF) & (alpha >= ALPHA_MIN)
    # float32 d^2 is good to about 2e-7 a c / det (relative); never less than M_D2
    m_d2 = CUTOFF * np.maximum(M_D2, 2e-7 * scr.cond[order])
    margin = bool(np.any(np.abs(d2 - CUTOFF) < m_d2)
                  | np.any(take & (np.abs(alpha - ALPHA_MIN) < M_ALPHA * ALPHA_MIN))
                  | np.any(take & (np.abs(g - ALPHA_MAX) < M_ALPHA * ALPHA_MAX)))
    a = np.where(take, alpha, 0.0)
    T_after = np.cumprod(1.0 - a)
    T_before = np.concatenate([[1.0], T_after[:-1]])
    stop = np.nonzero(take & (T_after < T_MIN))[0]
    if stop.size:
        k = stop[0]
        take[k + 1:] = False
        a[k + 1:] = 0.0
    margin |= bool(np.any(take & (np.abs(T_after - T_MIN) < M_T * T_MIN)))
    w = a * T_before
    rgb = (w[:, None] * scr.rgb[order]).sum(0)
    depth = float((w * scr.z[order]).sum())
    return rgb, depth, order[take], margin


def _candidates(scr: Screen, px: float, py: float) -> np.ndarray:
    r = scr.rect
    inside = scr.visible & (r[:, 0] <= px) & (px <= r[:, 1]) & (r[:, 2] <= py) & (py <= r[:, 3])
    return np.nonzero(inside)[0]


def render(p: Params, pose, cam, pixels=None):
    """Images (rgb [3, H, W], depth [H, W]) at one pose; with `pixels` ([K, 2]
    integer (i, j)), only those: (rgb [K, 3], depth [K], lists, margins)."""
    scr = project(p, pose, cam)
    if pixels is None:
        ij = np.stack(np.meshgrid(np.arange(cam.width), np.arange(cam.height), indexing="xy"), -1).reshape(-1, 2)
    else:
        ij = np.asarray(pixels)
    rgb = np.zeros((len(ij), 3))
    depth = np.zeros(len(ij))
    lists, margins = [], np.zeros(len(ij), bool)
    for k, (i, j) in enumerate(ij):
        c, d, lst, m = _pixel(scr, _candidates(scr, i + 0.5, j + 0.5), i + 0.5, j + 0.5)
        rgb[k], depth[k], margins[k] = c, d, m
        lists.append(lst)
    if pixels is None:
        return rgb.T.reshape(3, cam.height, cam.width), depth.reshape(cam.height, cam.width)
    return rgb, depth, lists, margins


def _touched(scr: Screen, i: int, cam) -> set:
    """Pixels whose centre lies in Gaussian i's support box."""
    if not scr.visible[i]:
        return set()
    x0, x1, y0, y1 = scr.rect[i]
    a0, a1 = max(int(np.ceil(x0 - 0.5)), 0), min(int(np.floor(x1 - 0.5)), cam.width - 1)
    b0, b1 = max(int(np.ceil(y0 - 0.5)), 0), min(int(np.floor(y1 - 0.5)), cam.height - 1)
    return {(a, b) for a in range(a0, a1 + 1) for b in range(b0, b1 + 1)}


def fd_gradient(p: Params, poses, cam, w_rgb, w_depth, gaussian: int, group: int, comp: int, h: float,
                with_scale: bool = False):
    """Central difference of L = sum(w_rgb rgb) + sum(w_depth depth) over all poses
    with respect to parameter (group, gaussian, comp) (groups: means, log_scales,
    quats, logits, rgb). Returns (gradient, stable), and with `with_scale` also
    the sum over pixels and poses of the magnitudes of the per-pixel central
    differences (the scale of the terms the gradient sums, which bounds what a
    float32 evaluation of that sum can lose to cancellation)."""
    def perturbed(delta):
        q = p.copy()
        arr = q.field(group)
        if arr.ndim == 1:
            arr[gaussian] += delta
        else:
            arr[gaussian, comp] += delta
        return q

    ps = [p, perturbed(h), perturbed(-h)]
    total = [0.0, 0.0, 0.0]
    scale = 0.0
    stable = True
    for pi, pose in enumerate(poses):
        scrs = [project(q, pose, cam) for q in ps]
        if any(s.margin[gaussian] for s in scrs):
            stable = False
        # near the support box edge the float32 rectangle may differ
        for s in scrs:
            if s.visible[gaussian]:
                x0, x1, y0, y1 = s.rect[gaussian]
                fx = (np.array([x0, x1]) - 0.5) % 1.0
                fy = (np.array([y0, y1]) - 0.5) % 1.0
                if np.any(np.minimum(fx, 1 - fx) < M_RECT) or np.any(np.minimum(fy, 1 - fy) < M_RECT):
                    stable = False
        pix = sorted(set().union(*[_touched(s, gaussian, cam) for s in scrs]))
        if not pix:
            continue
        pix = np.array(pix)
        outs = []
        for s in scrs:
            rgb = np.zeros((len(pix), 3))
            dep = np.zeros(len(pix))
            lists, marg = [], False
            for k, (i, j) in enumerate(pix):
                c, d, lst, m = _pixel(s, _candidates(s, i + 0.5, j + 0.5), i + 0.5, j + 0.5)
                rgb[k], dep[k] = c, d
                lists.append(lst)
                marg |= m  # a decision near its threshold anywhere in the pixel moves i's weight
            outs.append((rgb, dep, lists, marg))
        if any(o[3] for o in outs):
            stable = False
        for k in range(len(pix)):
            if not (np.array_equal(outs[0][2][k], outs[1][2][k]) and np.array_equal(outs[0][2][k], outs[2][2][k])):
                stable = False
        wr = w_rgb[pi][:, pix[:, 1], pix[:, 0]].T
        wd = w_depth[pi][pix[:, 1], pix[:, 0]]
        for e in range(3):
            total[e] += float((wr * outs[e][0]).sum() + (wd * outs[e][1]).sum())
        per_pixel = (wr * (outs[1][0] - outs[2][0])).sum(1) + wd * (outs[1][1] - outs[2][1])
        scale += float(np.abs(per_pixel).sum()) / (2 * h)
    if with_scale:
        return (total[1] - total[2]) / (2 * h), stable, scale
    return (total[1] - total[2]) / (2 * h), stable
