"""Pins for the oracle's NCC (Eq. 10): Pearson correlation, identities, bounds."""
import numpy as np
import pytest

import workloads as W
from oracle import ncc


def test_equals_numpy_corrcoef():
    imgs = W.random_images(0, 6, 37, 53)
    g = ncc.grey(imgs)
    s = ncc.ncc(imgs[0], imgs)
    for p in range(6):
        ref = np.corrcoef(g[0].ravel(), g[p].ravel())[0, 1]
        assert abs(s[p] - ref) < 1e-12
    assert abs(s[0] - 1.0) < 1e-12


def test_grey_weights_bt601():
    x = np.zeros((3, 1, 3))
    x[0, 0, 0] = 1
    x[1, 0, 1] = 1
    x[2, 0, 2] = 1
    assert np.allclose(ncc.grey(x)[0], [0.299, 0.587, 0.114])


@pytest.mark.parametrize("a,b", [(2.5, 0.3), (0.01, -4.0), (-1.7, 0.2)])
def test_affine_invariance_and_sign(a, b):
    q, r = W.random_images(1, 2, 24, 40)
    base = ncc.ncc(q, r[None])[0]
    aff = ncc.ncc(q, (a * r.astype(np.float64) + b)[None])[0]
    assert abs(aff - np.sign(a) * base) < 1e-10


def test_symmetry_and_bounds():
    imgs = W.random_images(2, 5, 16, 16)
    for i in range(5):
        for j in range(5):
            sij = ncc.ncc(imgs[i], imgs[j][None])[0]
            sji = ncc.ncc(imgs[j], imgs[i][None])[0]
            assert abs(sij - sji) < 1e-12 and -1 - 1e-12 <= sij <= 1 + 1e-12


def test_constant_image_scores_zero():
    q = W.random_images(3, 1, 8, 8)[0]
    const = np.full((1, 3, 8, 8), 0.37, np.float32)
    assert ncc.ncc(q, const)[0] == 0.0
    assert ncc.ncc(const[0], q[None])[0] == 0.0


def test_hand_example():
    # grey values q = [1, 2, 3, 4] and g = [2, 1, 4, 3]: centred (-1.5,-0.5,0.5,1.5) and
    # (-0.5,-1.5,1.5,0.5); sum of products 0.75+0.75+0.75+0.75 = 3; both sums of squares 5 -> 0.6
    q = np.zeros((3, 2, 2))
    g = np.zeros((1, 3, 2, 2))
    q[:] = np.array([[1, 2], [3, 4]], float)
    g[0, :] = np.array([[2, 1], [4, 3]], float)
    assert abs(ncc.ncc(q, g)[0] - 0.6) < 1e-12
