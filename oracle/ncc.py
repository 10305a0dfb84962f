"""Normalised cross-correlation (oracle; test infrastructure only).

Eq. 10 (Sec. III-C1): NCC(I_q, I_G) = sum (I_q - mean_q)(I_G - mean_G) /
(sqrt(sum (I_q - mean_q)^2) * sqrt(sum (I_G - mean_G)^2)), summed over all
pixels. Images are reduced to grey with 0.299 R + 0.587 G + 0.114 B first;
if either image has zero variance the score is 0. Float64, two passes.
"""
from __future__ import annotations

import numpy as np


def grey(rgb: np.ndarray) -> np.ndarray:
    """[...,3,H,W] -> [...,H,W] float64."""
    x = np.asarray(rgb, dtype=np.float64)
    return 0.299 * x[..., 0, :, :] + 0.587 * x[..., 1, :, :] + 0.114 * x[..., 2, :, :]


def ncc_grey(q: np.ndarray, g: np.ndarray) -> float:
    q = np.asarray(q, dtype=np.float64).ravel()
    g = np.asarray(g, dtype=np.float64).ravel()
    qc = q - q.mean()
    gc = g - g.mean()
    sq = np.sum(qc * qc)
    sg = np.sum(gc * gc)
    if sq == 0.0 or sg == 0.0:
        return 0.0
    return float(np.sum(qc * gc) / (np.sqrt(sq) * np.sqrt(sg)))


def ncc(query_rgb: np.ndarray, renders_rgb: np.ndarray) -> np.ndarray:
    """query [3,H,W], renders [P,3,H,W] -> scores [P] float64."""
    q = grey(query_rgb)
    r = grey(renders_rgb)
    return np.array([ncc_grey(q, r[p]) for p in range(r.shape[0])])
