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

Arithmetic is float64 on the float32 screen records.

Decisions near a threshold. A float32 implementation decides three things per
(pixel, Gaussian) from rounded values: d^2 <= 9, alpha >= 1/255 and T < 1e-4.
Where the exact value lies within the float32 evaluation's error bound of a
threshold, either decision is correct. Per pixel this module returns a margin
flag, set when any decision the pixel reaches lies that close, and
``outcomes`` lists every result the pixel can have when each such decision is
taken either way (the float64 result is one of them). A float32 image is
correct when every unflagged pixel matches the float64 result and every
flagged pixel matches one of its outcomes.

The error bounds (``_exponent_margins``, ``_t_step_error``) are for a float32
evaluation of the base-2 exponent p = log2(o) - log2(e)/2 d^2 as
log2(o) - t1^2 - t2^2, the sum of squares of
  t1 = s (sqrt(A) dx + B / sqrt(A) dy),  t2 = s sqrt(det / A) dy,
  s = sqrt(log2(e) / 2), det = A C - B^2,
with t1 and t2 expanded about a reference point in the pixel's tile, and for
T updated as T - alpha T:
  * each of the factors s sqrt(A), s B / sqrt(A), s sqrt(det / A) is within
    6 units of float32 roundoff (u = 2^-24) of its value: hardware square root
    and reciprocal square root (2u each) and three rounded products;
  * an affine term evaluated about a point of the tile has terms of magnitude
    at most S1 = s (sqrt(A) (|dx| + tw) + |B| / sqrt(A) (|dy| + th)) and
    S2 = s sqrt(det / A) (|dy| + th), so |t1 - t1*| <= 8u S1 and
    |t2 - t2*| <= 8u S2 (factor error plus two rounded fused adds);
  * the exponent adds 2|t1| 8u S1 + 2|t2| 8u S2 + the squares of those, and
    2u (|log2 o| + t1^2 + t2^2) for its two fused adds;
  * the cutoff threshold log2(o) - log2(e)/2 * 9 is one rounded sum of
    float32 constants (2u of its terms); log2(o) cancels between the exponent
    and this threshold;
  * the alpha-floor threshold log2(1/255) is a float32 constant (1u of 8), and
    there log2(o) does not cancel: LOG2_REL of |log2 o| plus LOG2_ABS;
  * per contributing layer, the float32 T picks up a relative error of
    alpha / (1 - alpha) (ln 2 m + EXP2_REL + u) + 2u, with m the exponent's
    margin and EXP2_REL the relative error of the hardware exponential; the
    constants 0.99 and 1e-4 differ from their float32 values by 1e-8 and 3e-8
    relative.
LOG2_REL, LOG2_ABS and EXP2_REL are the hardware log2 and exp2 accuracies
with a factor of 2 to spare: measured exhaustively on MI355X, log2 is within
1 ulp (2u relative) on [2^-9, 1] and exp2 within 1.42u relative on [-9.5, 0].

``render_tiled`` walks the sorted per-tile lists; ``render_bruteforce`` walks
every visible Gaussian for every pixel in (depth bits, index) order, with no
tiles at all. They agree on every pixel both leave unflagged, and each one's
result is among the other's outcomes where either flags.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .project import ScreenRecords

ALPHA_MIN = float(np.float32(1.0 / 255.0))
ALPHA_MAX = 0.99
T_MIN = 1e-4
CUTOFF = 9.0

# float32 error model of the compared implementation (module docstring)
U32 = 2.0 ** -24
S2 = 0.5 / math.log(2.0)          # log2(e) / 2: base-2 exponent per unit of d^2
LOG2_AMIN = math.log2(ALPHA_MIN)
FACTOR_ERR = 8.0                  # units of roundoff in t1, t2 per unit of S1, S2
LOG2_REL = 4.0 * U32
LOG2_ABS = 2.0 ** -26
EXP2_REL = 4.0 * U32
CONST_REL = 1e-8 + 3e-8           # float32(0.99), float32(1e-4) against the exact values
MAX_OUTCOMES = 4096


@dataclasses.dataclass
class Render:
    rgb: np.ndarray      # [3,H,W] float64
    depth: np.ndarray    # [H,W]
    t_final: np.ndarray  # [H,W]
    flag: np.ndarray     # [H,W] bool margin flag
    n_contrib: np.ndarray  # [H,W] contributing layers up to the stop
    e_wave: int = 0      # lane-slots under the per-wave culling model (tiled only)
    # what ``outcomes`` needs: (records, ordered list of a pixel: fn(i, j) -> indices, tile_w, tile_h)
    source: tuple | None = None


def _exponent_margins(dx, dy, A, B, C, op, tile_w, tile_h):
    """(d2, p, m_cut, m_amin): d^2, the exact base-2 exponent log2(o) - S2 d^2 and
    the error bounds (in base-2 exponent units) of the cutoff and alpha-floor
    decisions of a float32 evaluation (module docstring). Broadcasting arrays."""
    d2 = A * dx * dx + 2.0 * B * dx * dy + C * dy * dy
    lo = np.log2(np.maximum(op, 2.0 ** -149))  # (a zero opacity never contributes)
    p = lo - S2 * d2
    s = math.sqrt(S2)
    sa = np.sqrt(np.maximum(A, 1e-300))
    det = np.maximum(A * C - B * B, 0.0)
    f11, f12, f22 = s * sa, s * B / sa, s * np.sqrt(det / np.maximum(A, 1e-300))
    t1 = f11 * dx + f12 * dy
    t2 = f22 * dy
    e1 = FACTOR_ERR * U32 * (f11 * (np.abs(dx) + tile_w) + np.abs(f12) * (np.abs(dy) + tile_h))
    e2 = FACTOR_ERR * U32 * (f22 * (np.abs(dy) + tile_h))
    core = 2.0 * np.abs(t1) * e1 + 2.0 * np.abs(t2) * e2 + e1 * e1 + e2 * e2
    core = core + 2.0 * U32 * (np.abs(lo) + S2 * d2)
    m_cut = core + 2.0 * U32 * (S2 * CUTOFF + np.abs(lo))
    m_amin = core + LOG2_REL * np.abs(lo) + LOG2_ABS + 2.0 * U32 * abs(LOG2_AMIN)
    return d2, p, m_cut, m_amin


def _decisions(d2, alpha, p, m_cut, m_amin):
    """(contrib, may_contrib, may_skip) of the float64 values and the margins:
    contrib is the float64 decision; a float32 implementation may decide
    'contributes' where may_contrib and 'skips' where may_skip."""
    cut = S2 * (d2 - CUTOFF)  # > 0 outside the 3-sigma ellipse, in exponent units
    amin = p - LOG2_AMIN      # >= 0 where o exp(-d^2/2) >= 1/255
    contrib = (d2 <= CUTOFF) & (alpha >= ALPHA_MIN)
    may_contrib = (cut <= m_cut) & (amin >= -m_amin)
    may_skip = (cut > -m_cut) | (amin < m_amin)
    return contrib, may_contrib, may_skip


def _t_step_error(alpha, m_amin):
    """Relative error bound a contributing layer adds to a float32 T."""
    return alpha / (1.0 - alpha) * (math.log(2.0) * m_amin + EXP2_REL + U32) + 2.0 * U32


def _entry_margin_bounds(dxm, dym, A, B, C, op, tile_w, tile_h):
    """Upper bounds over a set of pixels of ``_exponent_margins``' two margins,
    per list entry, from the largest |dx| and |dy| over the set."""
    lo = np.log2(np.maximum(op, 2.0 ** -149))
    s = math.sqrt(S2)
    sa = np.sqrt(np.maximum(A, 1e-300))
    det = np.maximum(A * C - B * B, 0.0)
    f11, f12, f22 = s * sa, np.abs(s * B / sa), s * np.sqrt(det / np.maximum(A, 1e-300))
    t1 = f11 * dxm + f12 * dym
    t2 = f22 * dym
    e1 = FACTOR_ERR * U32 * (f11 * (dxm + tile_w) + f12 * (dym + tile_h))
    e2 = FACTOR_ERR * U32 * (f22 * (dym + tile_h))
    core = 2.0 * t1 * e1 + 2.0 * t2 * e2 + e1 * e1 + e2 * e2 + 2.0 * U32 * (np.abs(lo) + t1 * t1 + t2 * t2)
    m_cut = core + 2.0 * U32 * (S2 * CUTOFF + np.abs(lo))
    m_amin = core + LOG2_REL * np.abs(lo) + LOG2_ABS + 2.0 * U32 * abs(LOG2_AMIN)
    return m_cut, m_amin


def _composite(u, v, conic, op, rgb, z, px, py, tile_w=16, tile_h=16):
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
    u64 = u.astype(np.float64)[:, None]
    v64 = v.astype(np.float64)[:, None]
    dx = px[None, :] - u64
    dy = py[None, :] - v64
    A = conic[:, 0].astype(np.float64)[:, None]
    B = conic[:, 1].astype(np.float64)[:, None]
    Cc = conic[:, 2].astype(np.float64)[:, None]
    o = op.astype(np.float64)[:, None]
    d2 = A * dx * dx + 2.0 * B * dx * dy + Cc * dy * dy
    alpha = np.minimum(ALPHA_MAX, o * np.exp(-0.5 * d2))
    contrib = (d2 <= CUTOFF) & (alpha >= ALPHA_MIN)
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
    ncon = (contrib & live).sum(axis=0)

    # Margin flag. Per entry, bounds of the two exponent margins over these
    # pixels sieve the (entry, pixel) pairs; the exact margins decide on the
    # sieved ones and give the error T picks up at each contribution. A pixel is
    # flagged where a decision up to its latest possible stop lies within its
    # margin, or a termination test within T's error of 1e-4.
    # Only entries a pixel reaches with T above 0.99 T_MIN matter (T's error
    # bound stays far below 1%, asserted).
    alive = t_before >= 0.99 * T_MIN
    Lr = int(np.nonzero(alive.any(axis=1))[0].max()) + 1
    dxm = np.maximum(np.abs(px.min() - u64[:Lr]), np.abs(px.max() - u64[:Lr]))
    dym = np.maximum(np.abs(py.min() - v64[:Lr]), np.abs(py.max() - v64[:Lr]))
    mc_b, ma_b = _entry_margin_bounds(dxm, dym, A[:Lr], B[:Lr], Cc[:Lr], o[:Lr], tile_w, tile_h)
    lo = np.log2(np.maximum(o[:Lr], 2.0 ** -149))
    cut = S2 * (d2[:Lr] - CUTOFF)
    amin = (lo - S2 * d2[:Lr]) - LOG2_AMIN
    li, mi = np.nonzero(alive[:Lr] & (contrib[:Lr] | (np.abs(cut) <= mc_b) | (np.abs(amin) <= ma_b)))
    near = np.zeros((Lr, M), bool)
    step = np.zeros((Lr, M))
    if li.size:
        d2s, ps, mcs, mas = _exponent_margins(dx[li, mi], dy[li, mi], A[li, 0], B[li, 0], Cc[li, 0],
                                              o[li, 0], tile_w, tile_h)
        _, may_c, may_s = _decisions(d2s, alpha[li, mi], ps, mcs, mas)
        near[li, mi] = may_c & may_s
        step[li, mi] = np.where(contrib[li, mi], _t_step_error(alpha[li, mi], mas), 0.0)
    rel = np.cumsum(step, axis=0) + CONST_REL
    assert rel.max() < 1e-2
    c_r, t_r = contrib[:Lr], t_after[:Lr]
    sure_stop = c_r & (t_r < T_MIN * (1.0 - rel))
    stop_hi = np.where(sure_stop.any(axis=0), np.argmax(sure_stop, axis=0), Lr - 1)
    reach = k[:Lr] <= stop_hi[None, :]
    near |= c_r & (np.abs(t_r - T_MIN) <= T_MIN * rel)
    flag = (near & reach).any(axis=0)
    return col, dep, t_fin, flag, ncon, stop


def pixel_outcomes(u, v, conic, op, rgb, z, x, y, tile_w=16, tile_h=16):
    """Every result [n, 5] = (r, g, b, depth, T_final) the pixel at (x, y) can
    have when each decision within its margin is taken either way, for the
    ordered list (u, v, conic, op, rgb, z). Raises if there are more than
    MAX_OUTCOMES."""
    L = u.shape[0]
    if L == 0:
        return np.array([[0.0, 0.0, 0.0, 0.0, 1.0]])
    dx = x - u.astype(np.float64)
    dy = y - v.astype(np.float64)
    o = op.astype(np.float64)
    d2, p, m_cut, m_amin = _exponent_margins(dx, dy, conic[:, 0].astype(np.float64),
                                             conic[:, 1].astype(np.float64),
                                             conic[:, 2].astype(np.float64), o, tile_w, tile_h)
    alpha = np.minimum(ALPHA_MAX, o * np.exp(-0.5 * d2))
    contrib, may_c, may_s = _decisions(d2, alpha, p, m_cut, m_amin)
    step_err = _t_step_error(alpha, m_amin)
    c64 = rgb.astype(np.float64)
    z64 = z.astype(np.float64)
    cand = np.nonzero(may_c)[0]  # the entries that can contribute at all
    out = []
    # depth-first over the branches; a state is (next candidate, decision forced
    # on it or None, T, r, g, b, depth, relative error bound of T)
    stack = [(0, None, 1.0, 0.0, 0.0, 0.0, 0.0, CONST_REL)]
    while stack:
        pos, force, T, r, g, b, d, rel = stack.pop()
        while pos < cand.size:
            kk = cand[pos]
            if force is None:
                take = bool(contrib[kk])
                if may_s[kk]:  # near its threshold: the other decision is valid too
                    stack.append((pos, not take, T, r, g, b, d, rel))
            else:
                take = force
                force = None
            pos += 1
            if not take:
                continue
            w = alpha[kk] * T
            r += c64[kk, 0] * w
            g += c64[kk, 1] * w
            b += c64[kk, 2] * w
            d += z64[kk] * w
            T = T * (1.0 - alpha[kk])
            rel += step_err[kk]
            if T < T_MIN * (1.0 - rel):   # stops on either side
                break
            if T < T_MIN * (1.0 + rel):   # may stop here, or go on
                out.append((r, g, b, d, T))
        out.append((r, g, b, d, T))
        if len(out) > MAX_OUTCOMES:
            raise RuntimeError("more than MAX_OUTCOMES outcomes for one pixel")
    return np.array(out)


def outcomes(render: Render, i: int, j: int) -> np.ndarray:
    """``pixel_outcomes`` of pixel (i, j) of a render from this module."""
    rec, list_of, tw, th = render.source
    lst = list_of(i, j)
    return pixel_outcomes(rec.u[lst], rec.v[lst], rec.conic[lst], rec.opacity[lst], rec.rgb[lst],
                          rec.z[lst], i + 0.5, j + 0.5, tw, th)


def depth_order(rec: ScreenRecords, idx: np.ndarray) -> np.ndarray:
    """Sort Gaussian indices by (depth bits, index)."""
    zb = rec.z.astype(np.float32).view(np.uint32)[idx]
    return idx[np.lexsort((idx, zb))]


def _tile_list_fn(sorted_vals, ranges, width, tile_w, tile_h):
    tiles_x = (width + tile_w - 1) // tile_w

    def list_of(i, j):
        s, e = ranges[(j // tile_h) * tiles_x + (i // tile_w)]
        return sorted_vals[s:e].astype(np.int64)
    return list_of


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
                rec.z[lst], ii + 0.5, jj + 0.5, tile_w, tile_h)
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
    return Render(rgb, dep, tfin, flag, ncon, e_wave,
                  (rec, _tile_list_fn(sorted_vals, ranges, width, tile_w, tile_h), tile_w, tile_h))


def render_bruteforce(rec: ScreenRecords, width: int, height: int,
                      tile_w: int = 16, tile_h: int = 16) -> Render:
    """Every visible Gaussian at every pixel, in (depth bits, index) order; no
    tiles (tile_w, tile_h only size the float32 margins)."""
    idx = depth_order(rec, np.nonzero(rec.visible)[0])
    jj, ii = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    col, d, tf, fl, nc, _ = _composite(rec.u[idx], rec.v[idx], rec.conic[idx],
                                       rec.opacity[idx], rec.rgb[idx], rec.z[idx],
                                       ii + 0.5, jj + 0.5, tile_w, tile_h)
    return Render(col.reshape(3, height, width), d.reshape(height, width),
                  tf.reshape(height, width), fl.reshape(height, width),
                  nc.reshape(height, width), 0, (rec, lambda i, j: idx, tile_w, tile_h))


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
                                       pix_i[sel] + 0.5, pix_j[sel] + 0.5, tile_w, tile_h)
        rgb[:, sel] = c
        dep[sel] = d
        tf[sel] = t_
        fl[sel] = f
    return rgb, dep, tf, fl
