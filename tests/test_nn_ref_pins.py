"""Pins of the FP64 upscaler reference (oracle/nn_ref.py).

The paper has no learned part, so these pin the reference with mathematics
(identities, central finite differences) and with independent library
routines (torch CPU float64 conv2d, pixel_shuffle, interpolate, Adam).
"""
import math

import numpy as np
import pytest
import torch

from oracle import nn_ref as nr


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_matches_torch_conv2d():
    x = rnd((2, 7, 9, 5), 0)
    w = rnd((4, 3, 3, 5), 1)
    b = rnd(4, 2)
    y = nr.conv3x3(x, w, b)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2),
                                     torch.from_numpy(w).permute(0, 3, 1, 2),
                                     torch.from_numpy(b), padding=1)
    np.testing.assert_allclose(y, ref.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)


def test_conv_delta_kernels():
    x = rnd((1, 6, 5, 3), 3)
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, 1, 1, c] = 1.0
    np.testing.assert_array_equal(nr.conv3x3(x, w), x)
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, 0, 0, c] = 1.0       # output (i, j) reads input (i-1, j-1)
    y = nr.conv3x3(x, w)
    np.testing.assert_array_equal(y[:, 1:, 1:], x[:, :-1, :-1])
    assert np.all(y[:, 0] == 0) and np.all(y[:, :, 0] == 0)


def _fd(f, x, v, eps=1e-6):
    return (f(x + eps * v) - f(x - eps * v)) / (2 * eps)


def test_conv_gradients_finite_differences():
    x = rnd((2, 5, 6, 3), 4)
    w = rnd((2, 3, 3, 3), 5)
    b = rnd(2, 6)
    R = rnd((2, 5, 6, 2), 7)
    f = lambda x_, w_=w, b_=b: float((nr.conv3x3(x_, w_, b_) * R).sum())
    dx = nr.conv3x3_bwd_data(R, w)
    dw, db = nr.conv3x3_bwd_weight(x, R)
    for s in range(3):
        V = rnd(x.shape, 10 + s)
        assert (dx * V).sum() == pytest.approx(_fd(f, x, V), rel=1e-7)
        Vw = rnd(w.shape, 20 + s)
        assert (dw * Vw).sum() == pytest.approx(_fd(lambda w_: f(x, w_), w, Vw), rel=1e-7)
        Vb = rnd(b.shape, 30 + s)
        assert (db * Vb).sum() == pytest.approx(_fd(lambda b_: f(x, w, b_), b, Vb), rel=1e-7)


def test_pixel_shuffle_matches_torch_and_inverts():
    a = rnd((2, 3, 5, 48), 8)
    o = nr.pixel_shuffle(a)
    ref = torch.nn.functional.pixel_shuffle(torch.from_numpy(a).permute(0, 3, 1, 2), 4)
    np.testing.assert_array_equal(o, ref.permute(0, 2, 3, 1).numpy())
    np.testing.assert_array_equal(nr.pixel_unshuffle(o), a)


def test_bilinear_matches_torch_interpolate():
    a = rnd((2, 5, 7, 3), 9)
    up = nr.bilinear_up(a)
    ref = torch.nn.functional.interpolate(torch.from_numpy(a).permute(0, 3, 1, 2),
                                          scale_factor=4, mode="bilinear", align_corners=False)
    np.testing.assert_allclose(up, ref.permute(0, 2, 3, 1).numpy(), rtol=1e-13, atol=1e-13)
    # a constant field stays constant
    np.testing.assert_allclose(nr.bilinear_up(np.full((1, 3, 4, 1), 2.5)), 2.5)


def test_head_and_loss_gradient():
    conv6 = rnd((1, 3, 4, 48), 11) * 0.1
    L_low = np.abs(rnd((1, 3, 4, 3), 12))
    target = np.random.default_rng(13).uniform(0, 1, (1, 12, 16, 3))

    def f(c6):
        L, I = nr.head(c6, L_low)
        return nr.mse(I, target)

    L, I = nr.head(conv6, L_low)
    g = nr.head_backward(L, I, target)
    for s in range(3):
        V = rnd(conv6.shape, 40 + s)
        assert (g * V).sum() == pytest.approx(_fd(f, conv6, V), rel=1e-6)


def test_head_clamps_negative_optical_depth():
    # a residual that drives L below zero gives L = 0, I = 0 and no gradient
    conv6 = np.zeros((1, 1, 2, 48))
    conv6[0, 0, 0, :] = -5.0
    L_low = np.full((1, 1, 2, 3), 1.0)
    L, I = nr.head(conv6, L_low)
    assert np.all(L[:, :, :4] == 0.0) and np.all(I[:, :, :4] == 0.0)
    assert np.all(L[:, :, 4:] == 1.0)
    g = nr.head_backward(L, I, np.full(I.shape, 0.5))
    assert np.all(g[0, 0, 0] == 0.0) and np.all(g[0, 0, 1] != 0.0)


def test_pack_input_features():
    la = np.array([[[[0.0, 1.0, np.e - 1.0]]]])
    cc = np.array([[[3]]])
    np.testing.assert_allclose(nr.pack_input(la, cc)[0, 0, 0], [0.0, np.log(2.0), 1.0,
                                                               np.log(4.0)], rtol=1e-15)


def test_network_backward_finite_differences():
    params = nr.init_params(seed=1, scale_last=1.0)
    g = np.random.default_rng(14)
    x = g.uniform(0, 1, (1, 4, 5, 4))
    L_low = x[..., :3]
    target = g.uniform(0, 1, (1, 16, 20, 3))
    acts, L, I = nr.forward(params, x, L_low)
    grads = nr.backward(params, acts, L, I, target)

    def loss_with(k, which, val):
        ps = [(w.copy(), b.copy()) for w, b in params]
        w, b = ps[k]
        if which == 0:
            ps[k] = (val, b)
        else:
            ps[k] = (w, val)
        _, _, I2 = nr.forward(ps, x, L_low)
        return nr.mse(I2, target)

    for k in (0, 3, 5):
        for which in (0, 1):
            p = params[k][which]
            V = rnd(p.shape, 50 + 2 * k + which)
            an = (grads[k][which] * V).sum()
            num = _fd(lambda val: loss_with(k, which, val), p, V, eps=1e-6)
            assert an == pytest.approx(num, rel=2e-5, abs=1e-12), (k, which)


def test_adam_matches_torch():
    p0 = rnd(20, 15)
    grads = [rnd(20, 16 + t) for t in range(3)]
    p, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    for t, gr in enumerate(grads, start=1):
        nr.adam_step(p, gr, m, v, t, lr=1e-2)
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for gr in grads:
        opt.zero_grad()
        tp.grad = torch.from_numpy(gr)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_consistency_metric():
    L_low = np.abs(rnd((1, 4, 5, 3), 17))
    # a prediction equal to the low-res value on each central 2x2 block
    full = np.repeat(np.repeat(L_low, 4, axis=1), 4, axis=2)
    assert nr.consistency(full, L_low) == 0.0
    full2 = full.copy()
    full2[:, 1::4, 1::4] += 0.4       # one of four central pixels per block
    d = np.expm1(-L_low) - np.expm1(-(L_low + 0.1))
    assert nr.consistency(full2, L_low) == pytest.approx(math.sqrt(np.mean(d * d)), rel=1e-12)


def test_region_consistency_metric():
    g = np.random.default_rng(23)
    h, w = 10, 13                       # ragged: regions of 4 low pixels leave 2 and 1
    L_low = g.uniform(0, 2, (h, w, 3))
    L_full = g.uniform(0, 2, (4 * h, 4 * w, 3))
    # one region covering the image is the whole-frame metric
    one = nr.region_consistency(L_full, L_low, 4 * 16)
    assert one.shape == (1,)
    assert one[0] == pytest.approx(nr.consistency(L_full[None], L_low[None]), rel=1e-12)
    # regions of 4 low pixels: row-major, ceil(13/4) x ceil(10/4) = 4 x 3,
    # and the pixel-weighted mean of their squares is the frame's
    m = nr.region_consistency(L_full, L_low, 16)
    assert m.shape == (12,)
    npx = np.array([min(4, h - y) * min(4, w - x) for y in range(0, h, 4) for x in range(0, w, 4)])
    assert npx.sum() == h * w
    assert math.sqrt(float((m * m * npx).sum()) / (h * w)) == pytest.approx(
        nr.consistency(L_full[None], L_low[None]), rel=1e-12)
    # constant images: every region is |exp(-b) - exp(-a)|
    a, b = 0.3, 1.1
    m2 = nr.region_consistency(np.full((4 * h, 4 * w, 3), a), np.full((h, w, 3), b), 8)
    assert np.allclose(m2, abs(math.exp(-b) - math.exp(-a)), rtol=1e-14)
    # a change inside one region moves that region only (region (1, 2) of
    # 4x4 low pixels holds low pixel (5, 9))
    L2 = L_low.copy()
    L2[5, 9] += 0.5
    m3 = nr.region_consistency(L_full, L2, 16)
    changed = np.nonzero(m3 != m)[0]
    assert list(changed) == [1 * 4 + 2]


def test_param_count_and_flops():
    n = sum(co * 9 * ci + co for ci, co, _ in nr.LAYERS)
    assert n == 52048
    flops = sum(2 * 9 * ci * co * 512 * 512 for ci, co, _ in nr.LAYERS)
    assert abs(flops / 1e9 - 27.2) < 0.1
