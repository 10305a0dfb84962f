"""Pins of the learned-scorer oracle: convolution against brute force and
identities, gradients against central differences, bfloat16 rounding against a
library conversion and hand cases."""
import numpy as np
import pytest

import workloads as W
from oracle import scorer as S


def _conv_brute(x, w, b, s):
    N, H, Wd, Ci = x.shape
    Co = w.shape[0]
    Ho, Wo = S.out_size(H, s), S.out_size(Wd, s)
    y = np.zeros((N, Ho, Wo, Co))
    for n in range(N):
        for oy in range(Ho):
            for ox in range(Wo):
                for kh in range(3):
                    for kw in range(3):
                        iy, ix = oy * s - 1 + kh, ox * s - 1 + kw
                        if 0 <= iy < H and 0 <= ix < Wd:
                            y[n, oy, ox] += w[:, kh, kw, :] @ x[n, iy, ix]
    return y + b


@pytest.mark.parametrize("s,H,Wd", [(1, 5, 7), (2, 5, 7), (2, 6, 4), (1, 1, 1), (2, 1, 3)])
def test_conv_equals_brute_force(s, H, Wd):
    rng = np.random.default_rng(H * 10 + Wd + s)
    x = rng.normal(size=(2, H, Wd, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    assert np.allclose(S.conv3x3(x, w, b, s), _conv_brute(x, w, b, s))


def test_conv_delta_kernel_is_identity_or_subsampling():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(1, 6, 9, 2))
    w = np.zeros((2, 3, 3, 2))
    w[0, 1, 1, 0] = w[1, 1, 1, 1] = 1.0
    assert np.allclose(S.conv3x3(x, w, np.zeros(2), 1), x)
    assert np.allclose(S.conv3x3(x, w, np.zeros(2), 2), x[:, ::2, ::2])


@pytest.mark.parametrize("s", [1, 2])
def test_conv_backward_matches_central_differences(s):
    rng = np.random.default_rng(7 + s)
    x = rng.normal(size=(2, 5, 6, 3))
    w = rng.normal(size=(2, 3, 3, 3))
    b = rng.normal(size=2)
    dy = rng.normal(size=S.conv3x3(x, w, b, s).shape)
    f = lambda x_, w_, b_: float((S.conv3x3(x_, w_, b_, s) * dy).sum())
    dx, dw, db = S.conv3x3_backward(x, w, dy, s)
    h = 1e-6
    for arr, grad in ((x, dx), (w, dw), (b, db)):
        for _ in range(12):
            i = tuple(rng.integers(0, n) for n in arr.shape)
            a0 = arr[i]
            arr[i] = a0 + h
            fp = f(x, w, b)
            arr[i] = a0 - h
            fm = f(x, w, b)
            arr[i] = a0
            assert abs((fp - fm) / (2 * h) - grad[i]) < 1e-6 * max(1.0, abs(grad[i]))


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(11)
    params = W.scorer_params(5).astype(np.float64)
    params += rng.normal(0, 0.01, params.size)  # non-zero biases
    x = rng.normal(size=(3, 13, 22, 2))
    labels = rng.uniform(-1, 1, 3)
    loss, g = S.loss_and_grads(params, x, labels)
    h = 1e-6
    idx = rng.choice(params.size, 60, replace=False)
    idx = np.concatenate([idx, [params.size - 1, params.size - 2, 0, 608]])  # fc2 b, fc2 w, conv1, conv2
    for i in idx:
        p = params.copy()
        p[i] += h
        lp, _ = S.loss_and_grads(p, x, labels)
        p[i] -= 2 * h
        lm, _ = S.loss_and_grads(p, x, labels)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_parameter_layout():
    assert S.n_params() == 294113 == W.scorer_params(0).size
    parts = S.unflatten(np.arange(S.n_params()))
    assert [p.shape for p in parts] == S.param_shapes()
    assert np.array_equal(S.flatten(parts), np.arange(S.n_params()))


def test_bf16_round_hand_cases_and_library():
    # 1 + 2^-8 is half-way between 1 and 1 + 2^-7: ties go to the even mantissa (1)
    assert S.bf16_round(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 * 2^-8 is half-way between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert S.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert S.bf16_round(-2.5) == -2.5 and np.isnan(S.bf16_round(np.nan))
    import torch
    x = np.random.default_rng(2).normal(size=10000).astype(np.float32) * 10.0 ** np.random.default_rng(3).integers(-8, 8, 10000)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16_round(x), ref)


def test_standardise_pool_and_inputs():
    rng = np.random.default_rng(4)
    img = rng.normal(3.0, 2.0, (8, 12))
    z = S.standardise(img)
    assert abs(z.mean()) < 1e-12 and abs((z * z).mean() - 1) < 1e-12
    assert np.all(S.standardise(np.full((4, 4), 7.0)) == 0)
    # grey of a constant colour has a full 53-bit mantissa; its rounded mean differs from it
    assert np.all(S.standardise(S.grey(np.full((3, 94, 352), 0.25, np.float32))) == 0)
    rgb = rng.uniform(0, 1, (3, 8, 12))
    g = 0.299 * rgb[0] + 0.587 * rgb[1] + 0.114 * rgb[2]
    assert np.allclose(S.pool_grey(rgb, 4)[1, 2], g[4:8, 8:12].mean())
    x = S.inputs(rng.uniform(0, 1, (2, 3, 2, 3)), rng.uniform(0, 1, (2, 3)))
    assert x.shape == (2, 2, 3, 2) and np.allclose(x[0, :, :, 1], x[1, :, :, 1])


def test_forward_shapes_and_pooling():
    rng = np.random.default_rng(9)
    x = rng.normal(size=(2, 94, 352, 2))
    score, (acts, g, h) = S.forward(W.scorer_params(1), x)
    assert [a.shape[1:3] for a in acts] == [(94, 352), (47, 176), (47, 176), (24, 88), (24, 88), (12, 44)]
    assert score.shape == (2,) and np.allclose(g, acts[-1].mean(axis=(1, 2)))


def test_adamw_first_step_closed_form_and_constant_gradient():
    rng = np.random.default_rng(12)
    n = S.n_params()
    p = rng.normal(size=n)
    g = rng.normal(size=n)
    lr, eps = 1e-3, 1e-8
    m = v = np.zeros(n)
    step = lr * g / (np.abs(g) + eps)  # bias-corrected moments are g and g^2
    for t in (1, 2, 3):  # a constant gradient gives the same step every time
        p_new, m, v = S.adamw_step(p, g, m, v, t, lr, 0.9, 0.999, eps, 0.0)
        assert np.allclose(p - p_new, step, rtol=1e-9, atol=1e-15)
        p = p_new


def test_adamw_weight_decay_only_on_weights():
    n = S.n_params()
    p = np.full(n, 2.0)
    p_new, _, _ = S.adamw_step(p, np.zeros(n), np.zeros(n), np.zeros(n), 1, 0.1, 0.9, 0.999, 1e-8, 0.5)
    parts = S.unflatten(p_new)
    for i, q in enumerate(parts):
        bias = i % 2 == 1 and i != 12  # conv biases, b1, b2 (index 12 is the fc2 weight vector)
        assert np.all(q == (2.0 if bias else 2.0 * (1 - 0.1 * 0.5))), i


def test_adamw_matches_torch():
    import torch
    rng = np.random.default_rng(13)
    n = S.n_params()
    p0 = rng.normal(size=n)
    grads = [rng.normal(size=n) for _ in range(3)]
    mask = S.decay_mask().astype(bool)
    tw = torch.tensor(p0[mask], dtype=torch.float64, requires_grad=True)
    tb = torch.tensor(p0[~mask], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([{"params": [tw], "weight_decay": 0.01}, {"params": [tb], "weight_decay": 0.0}],
                            lr=3e-3, betas=(0.8, 0.95), eps=1e-6)
    p, m, v = p0, np.zeros(n), np.zeros(n)
    for t, g in enumerate(grads, 1):
        tw.grad = torch.tensor(g[mask])
        tb.grad = torch.tensor(g[~mask])
        opt.step()
        p, m, v = S.adamw_step(p, g, m, v, t, 3e-3, 0.8, 0.95, 1e-6, 0.01)
    assert np.allclose(p[mask], tw.detach().numpy(), rtol=0, atol=1e-12)
    assert np.allclose(p[~mask], tb.detach().numpy(), rtol=0, atol=1e-12)
