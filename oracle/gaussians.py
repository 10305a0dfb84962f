"""Gaussian parameters to 3D covariance (oracle; test infrastructure only).

Sec. III-A: each Gaussian has a covariance Sigma = R S S^T R^T with
S = diag(s_x, s_y, s_z) and R = q2R([r_w, r_x, r_y, r_z]). The colour is plain
RGB without spherical harmonics (Sec. III-B2).

Everything here is IEEE float32 in a fixed operation order:
  n  = sqrt(((w*w + x*x) + y*y) + z*z);   q <- q / n  (per component)
  R  = textbook unit-quaternion rotation matrix, each entry evaluated exactly
       as written below, left to right
  M  = R * diag(s)   (M_ij = R_ij * s_j)
  Sigma_ij = (M_i0*M_j0 + M_i1*M_j1) + M_i2*M_j2   for ij in 00,01,02,11,12,22
"""
from __future__ import annotations

import numpy as np

F = np.float32
ONE = F(1.0)
TWO = F(2.0)


def normalise_quat(q: np.ndarray) -> np.ndarray:
    """Unit quaternion, (w, x, y, z) order, float32 [N,4]."""
    q = np.asarray(q, dtype=F)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    n = np.sqrt(((w * w + x * x) + y * y) + z * z)
    return np.stack([w / n, x / n, y / n, z / n], axis=1)


def quat_to_rot(qn: np.ndarray) -> np.ndarray:
    """q2R of Sec. III-A for unit quaternions (w first); float32 [N,3,3]."""
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    r = np.empty((qn.shape[0], 3, 3), dtype=F)
    r[:, 0, 0] = ONE - TWO * (y * y + z * z)
    r[:, 0, 1] = TWO * (x * y - w * z)
    r[:, 0, 2] = TWO * (x * z + w * y)
    r[:, 1, 0] = TWO * (x * y + w * z)
    r[:, 1, 1] = ONE - TWO * (x * x + z * z)
    r[:, 1, 2] = TWO * (y * z - w * x)
    r[:, 2, 0] = TWO * (x * z - w * y)
    r[:, 2, 1] = TWO * (y * z + w * x)
    r[:, 2, 2] = ONE - TWO * (x * x + y * y)
    return r


def covariance(scales: np.ndarray, quats: np.ndarray) -> np.ndarray:
    """Sigma = R S S^T R^T; returns the 6 unique entries (00,01,02,11,12,22), f32 [N,6]."""
    s = np.asarray(scales, dtype=F)
    r = quat_to_rot(normalise_quat(quats))
    m = r * s[:, None, :]  # M_ij = R_ij * s_j

    def ent(i, j):
        return (m[:, i, 0] * m[:, j, 0] + m[:, i, 1] * m[:, j, 1]) + m[:, i, 2] * m[:, j, 2]

    return np.stack([ent(0, 0), ent(0, 1), ent(0, 2), ent(1, 1), ent(1, 2), ent(2, 2)], axis=1)


def full_cov(c6: np.ndarray) -> np.ndarray:
    """[N,6] unique entries -> symmetric [N,3,3] (same dtype)."""
    c = np.empty((c6.shape[0], 3, 3), dtype=c6.dtype)
    c[:, 0, 0] = c6[:, 0]
    c[:, 0, 1] = c[:, 1, 0] = c6[:, 1]
    c[:, 0, 2] = c[:, 2, 0] = c6[:, 2]
    c[:, 1, 1] = c6[:, 3]
    c[:, 1, 2] = c[:, 2, 1] = c6[:, 4]
    c[:, 2, 2] = c6[:, 5]
    return c
