"""Learned candidate scorer (oracle; test infrastructure only).

The paper prunes its candidate poses before the expensive comparison
(Sec. III-C1 renders and compares every candidate; Sec. IV explores only part
of the space). This module is the plain statement of the learned pruning
network: a small CNN that maps (low-resolution render, low-resolution query)
to a predicted NCC, trained by mean squared error against the full-resolution
NCC of Eq. 10. Everything is float64 NumPy with explicit loops over the nine
taps; the GPU version runs the same network in bfloat16 with float32
accumulation.

Input of one candidate: two channels, the BT.601 grey of the render and the
4x4-mean-pooled grey of the query, each standardised to zero mean and unit
variance over its pixels (a constant image becomes all zeros).

Network (NHWC activations, 'same' 3x3 convolutions with zero padding 1):
  conv 2->32 stride 2, ReLU; conv 32->64 stride 1, ReLU; conv 64->64 stride 2,
  ReLU; conv 64->128 stride 1, ReLU; conv 128->128 stride 2, ReLU;
  global average pool; linear 128->128, ReLU; linear 128->1.
Output size of a stride-s convolution of n pixels: (n - 1) // s + 1.

Parameters, one flat float32 vector in this order:
  per conv layer: W[c_out][3][3][c_in] then b[c_out];
  fc1: W[128][128] (out, in) then b[128]; fc2: W[128] then b[1].

With ``bf16=True`` the forward and backward round to bfloat16 (round to nearest,
ties to even) exactly where the GPU stores bfloat16: the weights of the conv
layers, the network input, every conv layer's output, and the gradient of
every conv layer's output. The sums themselves stay float64.
"""
from __future__ import annotations

import numpy as np

CHANNELS = [2, 32, 64, 64, 128, 128]
STRIDES = [2, 1, 2, 1, 2]
HIDDEN = 128


def param_shapes():
    shapes = []
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        shapes += [(co, 3, 3, ci), (co,)]
    shapes += [(HIDDEN, CHANNELS[-1]), (HIDDEN,), (HIDDEN,), (1,)]
    return shapes


def n_params() -> int:
    return int(sum(np.prod(s) for s in param_shapes()))


def unflatten(flat):
    flat = np.asarray(flat)
    out, o = [], 0
    for s in param_shapes():
        k = int(np.prod(s))
        out.append(flat[o:o + k].reshape(s))
        o += k
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def bf16_round(x):
    """Round to bfloat16 (8 significant bits), nearest, ties to even; returned as
    float64. Inputs are first rounded to float32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    r = np.where(np.isnan(f), u, r)  # NaN stays NaN
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def out_size(n: int, stride: int) -> int:
    return (n - 1) // stride + 1


def conv3x3(x, w, b, stride):
    """x [N, H, W, Ci], w [Co, 3, 3, Ci], b [Co] -> [N, Ho, Wo, Co]; zero padding 1."""
    N, H, W, Ci = x.shape
    Ho, Wo = out_size(H, stride), out_size(W, stride)
    xp = np.zeros((N, H + 2, W + 2, Ci))
    xp[:, 1:H + 1, 1:W + 1] = x
    y = np.zeros((N, Ho, Wo, w.shape[0]))
    for kh in range(3):
        for kw in range(3):
            patch = xp[:, kh:kh + stride * (Ho - 1) + 1:stride, kw:kw + stride * (Wo - 1) + 1:stride, :]
            y += patch @ w[:, kh, kw, :].T
    return y + b


def conv3x3_backward(x, w, dy, stride):
    """Gradients of conv3x3 w.r.t. x, w and b, given dy [N, Ho, Wo, Co]."""
    N, H, W, Ci = x.shape
    Ho, Wo = dy.shape[1], dy.shape[2]
    xp = np.zeros((N, H + 2, W + 2, Ci))
    xp[:, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w, dtype=np.float64)
    for kh in range(3):
        for kw in range(3):
            sl = (slice(None), slice(kh, kh + stride * (Ho - 1) + 1, stride),
                  slice(kw, kw + stride * (Wo - 1) + 1, stride), slice(None))
            patch = xp[sl]
            dw[:, kh, kw, :] = np.einsum("nhwo,nhwi->oi", dy, patch)
            dxp[sl] += dy @ w[:, kh, kw, :]
    return dxp[:, 1:H + 1, 1:W + 1], dw, dy.sum(axis=(0, 1, 2))


def standardise(img):
    """Zero mean, unit variance over all pixels (float64). A constant image (all
    pixels equal) gives zeros; this is decided by equality, since the rounded
    mean of equal values need not equal them."""
    img = np.asarray(img, dtype=np.float64)
    if np.all(img == img.flat[0]):
        return np.zeros_like(img)
    c = img - img.mean()
    return c / np.sqrt((c * c).mean())


def grey(rgb):
    rgb = np.asarray(rgb, dtype=np.float64)
    return 0.299 * rgb[0] + 0.587 * rgb[1] + 0.114 * rgb[2]


def pool_grey(rgb, f: int = 4):
    """f x f mean pooling of the BT.601 grey of a [3, H, W] image; H, W multiples of f."""
    g = grey(rgb)
    H, W = g.shape
    return g.reshape(H // f, f, W // f, f).mean(axis=(1, 3))


def inputs(render_rgb, query_pooled):
    """Network input of B candidates: renders [B, 3, h, w], query grey [h, w] -> [B, h, w, 2]."""
    q = standardise(query_pooled)
    B = render_rgb.shape[0]
    x = np.empty((B,) + q.shape + (2,))
    for i in range(B):
        x[i, :, :, 0] = standardise(grey(render_rgb[i]))
        x[i, :, :, 1] = q
    return x


def forward(params, x, bf16: bool = False):
    """Predicted scores [B] and the cache the backward pass needs."""
    p = unflatten(params)
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    acts = [rnd(x)]
    for l, s in enumerate(STRIDES):
        y = conv3x3(acts[-1], rnd(p[2 * l]), p[2 * l + 1], s)
        acts.append(rnd(np.maximum(y, 0.0)))
    g = acts[-1].mean(axis=(1, 2))
    w1, b1, w2, b2 = p[10], p[11], p[12], p[13]
    h = np.maximum(g @ w1.T + b1, 0.0)
    score = h @ w2 + b2[0]
    return score, (acts, g, h)


def loss_and_grads(params, x, labels, bf16: bool = False):
    """MSE = mean((score - label)^2) and its gradient w.r.t. the flat parameters."""
    p = unflatten(params)
    score, (acts, g, h) = forward(params, x, bf16)
    rnd = bf16_round if bf16 else (lambda a: a)
    B = x.shape[0]
    r = score - np.asarray(labels, dtype=np.float64)
    loss = float((r * r).mean())
    ds = 2.0 * r / B
    w1, w2 = p[10], p[12]
    dw2 = h.T @ ds
    db2 = np.array([ds.sum()])
    dh = np.outer(ds, w2) * (h > 0)
    dw1 = dh.T @ g
    db1 = dh.sum(axis=0)
    dg = dh @ w1
    a5 = acts[-1]
    dy = np.broadcast_to(dg[:, None, None, :] / (a5.shape[1] * a5.shape[2]), a5.shape) * (a5 > 0)
    grads = [None] * 10
    for l in reversed(range(5)):
        dy = rnd(dy)
        dx, dw, db = conv3x3_backward(acts[l], rnd(p[2 * l]), dy, STRIDES[l])
        grads[2 * l], grads[2 * l + 1] = dw, db
        if l > 0:
            dy = dx * (acts[l] > 0)
    return loss, flatten(grads + [dw1, db1, dw2, db2])


def decay_mask():
    """1.0 for the entries that weight decay applies to (weights), 0.0 for biases."""
    return flatten([np.full(s, 1.0 if len(s) > 1 or i == len(param_shapes()) - 2 else 0.0)
                    for i, s in enumerate(param_shapes())])


def adamw_step(params, grads, m, v, t, lr, beta1, beta2, eps, weight_decay):
    """One AdamW step (Adam moments with bias correction, weight decay decoupled
    from the gradient and applied to weights only); t counts this step from 1.
    Returns new (params, m, v), float64."""
    p = np.asarray(params, dtype=np.float64)
    g = np.asarray(grads, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    p = p - lr * weight_decay * decay_mask() * p - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v
