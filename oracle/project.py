"""EWA projection of 3D Gaussians for one camera pose (oracle; test infrastructure only).

Sec. III-A, Eq. 3 and Eq. 4. For world-to-camera pose W_t = [R_w | t_w] and
intrinsics (fx, fy, cx, cy):

  t      = R_w mu + t_w                       (camera-space mean)
  m(mu)  = (fx t_x/t_z + cx, fy t_y/t_z + cy)  (Eq. 4, pixel units)
  J      = d m / d t, a 2x3 matrix             (Jacobian of Eq. 4)
  Sigma' = (J R_w) Sigma (J R_w)^T + eps I     (Eq. 3, top-left 2x2 kept)

then the inverse (the conic used by the footprint of Eq. 2), the 3-sigma
pixel rectangle and the tile rectangle.

Float32, fixed operation order (written out term by term below):
  cull a Gaussian with any non-finite mean, covariance, opacity or colour entry
  t_k  = ((Rw[k,0]*mu_x + Rw[k,1]*mu_y) + Rw[k,2]*mu_z) + tw[k]; cull unless t_z > 0.2
  xt   = t_x / t_z, yt = t_y / t_z; lim_x = 1.3 * ((0.5*W) / fx), lim_y alike;
  xc   = clamp(xt, -lim_x, lim_x), yc alike (used in J only)
  J00  = fx / t_z, J02 = -(fx*xc) / t_z, J11 = fy / t_z, J12 = -(fy*yc) / t_z
  T0j  = J00*Rw[0,j] + J02*Rw[2,j];  T1j = J11*Rw[1,j] + J12*Rw[2,j]
  U_ij = (T_i0*S_0j + T_i1*S_1j) + T_i2*S_2j
  a    = ((U00*T00 + U01*T01) + U02*T02) + eps
  b    = (U00*T10 + U01*T11) + U02*T12
  c    = ((U10*T10 + U11*T11) + U12*T12) + eps
  det  = a*c - b*b; cull unless det > 0; conic = (c/det, (-b)/det, a/det)
  rx   = 3*sqrt(a), ry = 3*sqrt(c); u = fx*xt + cx, v = fy*yt + cy
  cull if any of u, v, rx, ry, conic is not finite
  i0 = max(ceil((u - rx) - 0.5), 0), i1 = min(floor((u + rx) - 0.5), W-1), j0/j1 alike
  cull if i0 > i1 or j0 > j1; tile rect = [i0 // tw, i1 // tw] x [j0 // th, j1 // th]

Pixel i is sampled at i + 0.5, so [i0, i1] is exactly the set of pixel columns
whose centre lies within rx of u; rx = 3 sqrt(a) is the horizontal half-width
of the ellipse d^2 = 9 of covariance [[a, b], [b, c]].
"""
from __future__ import annotations

import dataclasses

import numpy as np

F = np.float32

# Readings of constants the paper leaves open (defaults; see the package docstring).
EPS_DILATE = F(0.3)
Z_NEAR = F(0.2)
JAC_CLAMP = F(1.3)


@dataclasses.dataclass
class ScreenRecords:
    """Per-Gaussian screen-space records for one pose (float32 unless noted)."""
    visible: np.ndarray  # [N] bool
    u: np.ndarray
    v: np.ndarray
    z: np.ndarray        # camera-space depth t_z
    conic: np.ndarray    # [N,3] (A, B, C): d^2 = A dx^2 + 2 B dx dy + C dy^2
    cov2d: np.ndarray    # [N,3] (a, b, c) dilated screen covariance
    rx: np.ndarray
    ry: np.ndarray
    rect: np.ndarray     # [N,4] int64 pixel rectangle (i0, i1, j0, j1), -1 if culled
    tile_rect: np.ndarray  # [N,4] int64 (tx0, tx1, ty0, ty1), -1 if culled
    opacity: np.ndarray
    rgb: np.ndarray      # [N,3]

    @property
    def n_tiles(self) -> np.ndarray:
        tr = self.tile_rect
        n = (tr[:, 1] - tr[:, 0] + 1) * (tr[:, 3] - tr[:, 2] + 1)
        return np.where(self.visible, n, 0)


def nonfinite(mu: np.ndarray, cov6: np.ndarray, opacity: np.ndarray, rgb: np.ndarray) -> np.ndarray:
    """[N] bool: Gaussians with a non-finite mean, covariance entry, opacity or
    colour channel. Such a Gaussian is culled at every pose (and counted)."""
    with np.errstate(all="ignore"):
        ok = (np.isfinite(np.asarray(mu, F)).all(1) & np.isfinite(np.asarray(cov6, F)).all(1)
              & np.isfinite(np.asarray(opacity, F)) & np.isfinite(np.asarray(rgb, F)).all(1))
    return ~ok


def preprocess(mu: np.ndarray, cov6: np.ndarray, opacity: np.ndarray, rgb: np.ndarray,
               pose: np.ndarray, width: int, height: int, fx: float, fy: float,
               cx: float, cy: float, tile_w: int = 16, tile_h: int = 16,
               eps: float = EPS_DILATE, z_near: float = Z_NEAR,
               jac_clamp: float = JAC_CLAMP) -> ScreenRecords:
    """Eq. 3-4 for one pose over all Gaussians (float32, order as in the module docstring)."""
    mu = np.asarray(mu, dtype=F)
    s = np.asarray(cov6, dtype=F)
    pose = np.asarray(pose, dtype=F)
    fx, fy, cx, cy = F(fx), F(fy), F(cx), F(cy)
    eps, z_near, jac_clamp = F(eps), F(z_near), F(jac_clamp)
    rw = pose[:, :3]
    tw = pose[:, 3]
    n = mu.shape[0]

    def tcomp(k):
        return ((rw[k, 0] * mu[:, 0] + rw[k, 1] * mu[:, 1]) + rw[k, 2] * mu[:, 2]) + tw[k]

    tx, ty, tz = tcomp(0), tcomp(1), tcomp(2)
    with np.errstate(all="ignore"):
        vis = tz > z_near
        vis &= ~nonfinite(mu, s, opacity, rgb)
        xt = tx / tz
        yt = ty / tz
        lim_x = jac_clamp * ((F(0.5) * F(width)) / fx)
        lim_y = jac_clamp * ((F(0.5) * F(height)) / fy)
        xc = np.minimum(np.maximum(xt, -lim_x), lim_x)
        yc = np.minimum(np.maximum(yt, -lim_y), lim_y)
        j00 = fx / tz
        j02 = -(fx * xc) / tz
        j11 = fy / tz
        j12 = -(fy * yc) / tz
        t0 = [j00 * rw[0, j] + j02 * rw[2, j] for j in range(3)]
        t1 = [j11 * rw[1, j] + j12 * rw[2, j] for j in range(3)]
        # Sigma_ij from the 6 unique entries (00,01,02,11,12,22)
        S = [[s[:, 0], s[:, 1], s[:, 2]], [s[:, 1], s[:, 3], s[:, 4]], [s[:, 2], s[:, 4], s[:, 5]]]

        def urow(t):
            return [(t[0] * S[0][j] + t[1] * S[1][j]) + t[2] * S[2][j] for j in range(3)]

        u0 = urow(t0)
        u1 = urow(t1)
        a = ((u0[0] * t0[0] + u0[1] * t0[1]) + u0[2] * t0[2]) + eps
        b = (u0[0] * t1[0] + u0[1] * t1[1]) + u0[2] * t1[2]
        c = ((u1[0] * t1[0] + u1[1] * t1[1]) + u1[2] * t1[2]) + eps
        det = a * c - b * b
        vis &= det > 0
        ca = c / det
        cb = (-b) / det
        cc = a / det
        rx = F(3.0) * np.sqrt(a)
        ry = F(3.0) * np.sqrt(c)
        u = fx * xt + cx
        v = fy * yt + cy
        fin = (np.isfinite(u) & np.isfinite(v) & np.isfinite(rx) & np.isfinite(ry)
               & np.isfinite(ca) & np.isfinite(cb) & np.isfinite(cc))
        vis &= fin
        half = F(0.5)
        i0f = np.maximum(np.ceil((u - rx) - half), F(0.0))
        i1f = np.minimum(np.floor((u + rx) - half), F(width - 1))
        j0f = np.maximum(np.ceil((v - ry) - half), F(0.0))
        j1f = np.minimum(np.floor((v + ry) - half), F(height - 1))
        vis &= (i0f <= i1f) & (j0f <= j1f)
    rect = np.full((n, 4), -1, dtype=np.int64)
    rect[vis, 0] = i0f[vis].astype(np.int64)
    rect[vis, 1] = i1f[vis].astype(np.int64)
    rect[vis, 2] = j0f[vis].astype(np.int64)
    rect[vis, 3] = j1f[vis].astype(np.int64)
    trect = np.full((n, 4), -1, dtype=np.int64)
    trect[vis, 0] = rect[vis, 0] // tile_w
    trect[vis, 1] = rect[vis, 1] // tile_w
    trect[vis, 2] = rect[vis, 2] // tile_h
    trect[vis, 3] = rect[vis, 3] // tile_h
    return ScreenRecords(vis, u, v, tz, np.stack([ca, cb, cc], 1), np.stack([a, b, c], 1),
                         rx, ry, rect, trect, np.asarray(opacity, dtype=F),
                         np.asarray(rgb, dtype=F))
