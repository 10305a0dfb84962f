"""Front-to-back compositing of colour and depth (oracle; test infrastructure only).

Eq. 1 and Eq. 5 (Sec. III-A) with the footprint of Eq. 2 read as
q_i(x) = o_i * exp(-d_i(x)^2 / 2), d^2 = A dx^2 + 2 B dx dy + C dy^2 (conic of
the screen covariance, dx = x - u_i, dy = y - v_i):

  C(x) = sum_i c_i alpha_i T_i,   D(x) = sum_i z_i alpha_i T_i,
  T_i  = prod_{j<i} (1 - alpha_j)

over the depth-ordered Gaussians, where a Gaussian contributes only if
d^2 <= 9, with alpha = min(0.99, q) and alpha >= float32(1/255). The pixel
stops after the first contributing Gaussian that takes T below 1e-4 (that
layer is included). Background is 0.

Arithmetic is float64 on the float32 screen records. Besides the images this
returns, per pixel, T_final and a margin flag: set when any decision up to the
stop lies within a small distance of its threshold (|d^2 - 9| < 1e-5,
|alpha - 1/255| < 1e-6, |T - 1e-4| < 1e-7), where float32 rounding on the GPU
may legitimately decide the other way.

``render_tiled`` walks the sorted per-tile lists; ``render_bruteforce`` walks
every visible Gaussian for every pixel in (depth bits, index) order, with no
tiles at all. Away from flagged pixels the two agree.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .project import ScreenRecords

ALPHA_MIN = float(np.float32(1.0 / 255.0))
ALPHA_MAX = 0.99
T_MIN = 1e-4
CUTOFF = 9.0
MARGIN_D2 = 1e-5
MARGIN_ALPHA = 1e-6
MARGIN_T = 1e-7


@dataclasses.dataclass
class Render:
    rgb: np.ndarray      # [3,H,W] float64
    depth: np.ndarray    # [H,W]
    t_final: np.ndarray  # [H,W]
    flag: np.ndarray     # [H,W] bool margin flag
    n_contrib: np.ndarray  # [H,W] contributing layers up to the stop
    e_wave: int = 0      # lane-slots under the per-wave culling model (tiled only)


def _composite(u, v, conic, op, rgb, z, px, py):
    """Composite an ordered list (length L) at pixels (px, py) (length M).

    Returns rgb [3,M], depth [M], t_final [M], flag [M], n_contrib [M], stop [M]
    (index of the last list entry processed; L-1 if the pixel never stops).
    """
    L = u.shape[0]
    M = px.shape[0]
    if L == 0:
        z0 = np.zeros(M)
        return (np.zeros((3, M)), z0, np.ones(M), np.zeros(M, bool),
                np.zeros(M, np.int64), np.full(M, -1, np.int64))
    dx = px[None, :] - u.astype(np.float64)[:, None]
    dy = py[None, :] - v.astype(np.float64)[:, None]
    A = conic[:, 0].astype(np.float64)[:, None]
    B = conic[:, 1].astype(np.float64)[:, None]
    Cc = conic[:, 2].astype(np.float64)[:, None]
    d2 = A * dx * dx + 2.0 * B * dx * dy + Cc * dy * dy
    inside = d2 <= CUTOFF
    raw = op.astype(np.float64)[:, None] * np.exp(-0.5 * d2)
    alpha = np.minimum(ALPHA_MAX, raw)
    contrib = inside & (alpha >= ALPHA_MIN)
    a_eff = np.where(contrib, alpha, 0.0)
    t_after = np.cumprod(1.0 - a_eff, axis=0)
    t_before = np.vstack([np.ones((1, M)), t_after[:-1]])
    term = t_after < T_MIN
    any_term = term.any(axis=0)
    stop = np.where(any_term, np.argmax(term, axis=0), L - 1)
    k = np.arange(L)[:, None]
    live = k <= stop[None, :]
    w = np.where(live, a_eff * t_before, 0.0)
    col = np.einsum("lm,lc->cm", w, rgb.astype(np.float64))
    dep = (w * z.astype(np.float64)[:, None]).sum(axis=0)
    t_fin = t_after[stop, np.arange(M)]
    near = (np.abs(d2 - CUTOFF) < MARGIN_D2)
    near |= inside & (np.abs(alpha - ALPHA_MIN) < MARGIN_ALPHA)
    near |= contrib & (np.abs(t_after - T_MIN) < MARGIN_T)
    flag = (near & live).any(axis=0)
    ncon = (contrib & live).sum(axis=0)
    return col, dep, t_fin, flag, ncon, stop


def depth_order(rec: ScreenRecords, idx: np.ndarray) -> np.ndarray:
    """Sort Gaussian indices by (depth bits, index)."""
    zb = rec.z.astype(np.float32).view(np.uint32)[idx]
    return idx[np.lexsort((idx, zb))]


def render_tiled(rec: ScreenRecords, sorted_vals: np.ndarray, ranges: np.ndarray,
                 width: int, height: int, tile_w: int = 16, tile_h: int = 16,
                 wave_w: int = 8, wave_h: int = 8) -> Render:
    """Composite each tile from its sorted list (ranges from ``keys.tile_ranges``).

    ``e_wave`` counts lane-slots of a wave model in which each wave owns a
    wave_w x wave_h block of the tile, skips list entries whose pixel
    rectangle misses its block, and runs until all of its pixels stopped.
    """
    tiles_x = (width + tile_w - 1) // tile_w
    tiles_y = (height + tile_h - 1) // tile_h
    rgb = np.zeros((3, height, width))
    dep = np.zeros((height, width))
    tfin = np.ones((height, width))
    flag = np.zeros((height, width), bool)
    ncon = np.zeros((height, width), np.int64)
    e_wave = 0
    for ty in range(tiles_y):
        for tx in range(tiles_x):
            t = ty * tiles_x + tx
            s, e = ranges[t]
            lst = sorted_vals[s:e].astype(np.int64)
            x0, y0 = tx * tile_w, ty * tile_h
            x1, y1 = min(x0 + tile_w, width), min(y0 + tile_h, height)
            jj, ii = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
            ii = ii.ravel()
            jj = jj.ravel()
            col, d, tf, fl, nc, stop = _composite(
                rec.u[lst], rec.v[lst], rec.conic[lst], rec.opacity[lst], rec.rgb[lst],
                rec.z[lst], ii + 0.5, jj + 0.5)
            rgb[:, jj, ii] = col
            dep[jj, ii] = d
            tfin[jj, ii] = tf
            flag[jj, ii] = fl
            ncon[jj, ii] = nc
            if lst.size:
                r = rec.rect[lst]
                for wy in range(y0, y1, wave_h):
                    for wx in range(x0, x1, wave_w):
                        wx1, wy1 = min(wx + wave_w, x1) - 1, min(wy + wave_h, y1) - 1
                        sel = (ii >= wx) & (ii <= wx1) & (jj >= wy) & (jj <= wy1)
                        wstop = stop[sel].max()
                        hit = ((r[:, 0] <= wx1) & (r[:, 1] >= wx) & (r[:, 2] <= wy1)
                               & (r[:, 3] >= wy))
                        e_wave += 64 * int(hit[: wstop + 1].sum())
    return Render(rgb, dep, tfin, flag, ncon, e_wave)


def render_bruteforce(rec: ScreenRecords, width: int, height: int) -> Render:
    """Every visible Gaussian at every pixel, in (depth bits, index) order; no tiles."""
    idx = depth_order(rec, np.nonzero(rec.visible)[0])
    jj, ii = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    col, d, tf, fl, nc, _ = _composite(rec.u[idx], rec.v[idx], rec.conic[idx],
                                       rec.opacity[idx], rec.rgb[idx], rec.z[idx],
                                       ii + 0.5, jj + 0.5)
    return Render(col.reshape(3, height, width), d.reshape(height, width),
                  tf.reshape(height, width), fl.reshape(height, width),
                  nc.reshape(height, width))


def render_pixels(rec: ScreenRecords, sorted_vals: np.ndarray, ranges: np.ndarray,
                  width: int, pix_i: np.ndarray, pix_j: np.ndarray,
                  tile_w: int = 16, tile_h: int = 16):
    """Composite selected pixels only (for sampled checks at full size).

    Returns rgb [3,M], depth [M], t_final [M], flag [M].
    """
    tiles_x = (width + tile_w - 1) // tile_w
    M = pix_i.shape[0]
    rgb = np.zeros((3, M))
    dep = np.zeros(M)
    tf = np.ones(M)
    fl = np.zeros(M, bool)
    tid = (pix_j // tile_h) * tiles_x + (pix_i // tile_w)
    for t in np.unique(tid):
        sel = np.nonzero(tid == t)[0]
        s, e = ranges[t]
        lst = sorted_vals[s:e].astype(np.int64)
        c, d, t_, f, _, _ = _composite(rec.u[lst], rec.v[lst], rec.conic[lst],
                                       rec.opacity[lst], rec.rgb[lst], rec.z[lst],
                                       pix_i[sel] + 0.5, pix_j[sel] + 0.5)
        rgb[:, sel] = c
        dep[sel] = d
        tf[sel] = t_
        fl[sel] = f
    return rgb, dep, tf, fl
