"""Upscaler kernels (BF16 matrix-core convolutions with FP32 accumulation,
head, loss, Adam, consistency) against the FP64 reference oracle/nn_ref.py.

Inputs are rounded to bf16 first and the reference runs on exactly those
values in float64, so the only differences are the kernels' FP32
accumulation and, for bf16 outputs, the final rounding:
  |y - ref| <= 2e-5 * S (+ 2^-8 |ref| for bf16 outputs),
with S = sum of the absolute values of the terms (bias included); 2e-5
exceeds K * 2^-24 for the largest term count K = 9 * 48 + 1 used here.
"""
import math

import numpy as np
import pytest

from oracle import nn_ref as nr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1309_1114_amd import nn as nnmod
    return nnmod


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def dev_bf16(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).cuda()


def dev_f32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def host(t):
    import torch
    return t.float().cpu().numpy().astype(np.float64)


def check(got, ref, scale, bf16_out):
    tol = 2e-5 * scale + (2.0 ** -8) * np.abs(ref) * bf16_out + 1e-30
    bad = np.abs(got - ref) > tol
    assert not bad.any(), (int(bad.sum()), float(np.abs(got - ref).max()))


SHAPES = [(4, 32), (32, 32), (32, 48), (48, 32)]


@pytest.mark.parametrize("cin,cout", SHAPES)
@pytest.mark.parametrize("out_f32", [0, 1])
def test_conv_fwd(nn, cin, cout, out_f32):
    g = np.random.default_rng(cin * 100 + cout + out_f32)
    n, h, w = 2, 19, 37                     # several 16 x 16 tiles and ragged tails
    x = bf16(g.standard_normal((n, h, w, cin)))
    wt = bf16(g.standard_normal((cout, 3, 3, cin)) * 0.2)
    b = g.standard_normal(cout).astype(np.float32).astype(np.float64)
    relu = cout != 48
    y = nn.conv3x3_fwd(dev_bf16(x), dev_bf16(wt), dev_f32(b), relu=relu, out_f32=bool(out_f32))
    ref = nr.conv3x3(x, wt, b)
    scale = nr.conv3x3(np.abs(x), np.abs(wt), np.abs(b))
    if relu:
        ref = np.maximum(ref, 0.0)
    check(host(y), ref, scale, 0 if out_f32 else 1)


def test_conv_fwd_mask_and_no_bias(nn):
    # the data-gradient form: input masked by a ReLU output, no bias
    g = np.random.default_rng(7)
    n, h, w = 1, 33, 17
    dy = bf16(g.standard_normal((n, h, w, 32)))
    act = bf16(np.maximum(g.standard_normal((n, h, w, 32)), 0.0))
    wt = bf16(g.standard_normal((32, 3, 3, 32)) * 0.2)
    y = nn.conv3x3_fwd(dev_bf16(dy), dev_bf16(wt), mask=dev_bf16(act), relu=False, out_f32=True)
    d = dy * (act > 0)
    check(host(y), nr.conv3x3(d, wt), nr.conv3x3(np.abs(d), np.abs(wt)), 0)


@pytest.mark.parametrize("cin,cout", [(32, 32), (32, 48)])
def test_data_gradient_via_flipped_weights(nn, cin, cout):
    g = np.random.default_rng(11 + cout)
    n, h, w = 2, 21, 18
    dy = bf16(g.standard_normal((n, h, w, cout)))
    wt = bf16(g.standard_normal((cout, 3, 3, cin)) * 0.2)
    wflip = nn.flip_weights(dev_bf16(wt))
    assert np.array_equal(host(wflip), np.transpose(wt[:, ::-1, ::-1, :], (3, 1, 2, 0)))
    dx = nn.conv3x3_fwd(dev_bf16(dy), wflip, relu=False, out_f32=True)
    ref = nr.conv3x3_bwd_data(dy, wt)
    scale = nr.conv3x3_bwd_data(np.abs(dy), np.abs(wt))
    check(host(dx), ref, scale, 0)


@pytest.mark.parametrize("cin,cout", [(4, 32), (32, 32), (32, 48)])
@pytest.mark.parametrize("masked", [False, True])
def test_conv_bwd_weight(nn, cin, cout, masked):
    import torch
    g = np.random.default_rng(cin + cout + 5 * masked)
    n, h, w = 2, 27, 35                     # 8 x 16 tiles with ragged tails
    x = bf16(g.standard_normal((n, h, w, cin)))
    dy = bf16(g.standard_normal((n, h, w, cout)))
    act = bf16(np.maximum(g.standard_normal((n, h, w, cout)), 0.0)) if masked else None
    d = dy * (act > 0) if masked else dy
    dw = torch.full((cout, 3, 3, cin), 0.5, device="cuda")    # accumulates
    db = torch.full((cout,), -0.25, device="cuda")
    nn.conv3x3_bwd_weight(dev_bf16(x), dev_bf16(dy), dw, db,
                          mask=dev_bf16(act) if masked else None)
    rdw, rdb = nr.conv3x3_bwd_weight(x, d)
    sdw, sdb = nr.conv3x3_bwd_weight(np.abs(x), np.abs(d))
    check(host(dw), rdw + 0.5, sdw + 0.5, 0)
    check(host(db), rdb - 0.25, sdb + 0.25, 0)


def test_pack_input(nn):
    import torch
    g = np.random.default_rng(3)
    la = g.uniform(0, 5, (2, 9, 13, 3)).astype(np.float32)
    cc = g.integers(0, 1000, (2, 9, 13)).astype(np.int32)
    x = nn.pack_input(dev_f32(la), torch.from_numpy(cc).cuda())
    ref = nr.pack_input(la.astype(np.float64), cc)
    got = host(x)
    # log1p in FP32 then one bf16 rounding
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * ref + 1e-6)


def test_head_loss_and_gradient(nn):
    import torch
    g = np.random.default_rng(4)
    n, h, w = 2, 5, 7
    # large enough that the clamp at L = 0 is active on part of the image
    conv6 = (g.standard_normal((n, h, w, 48)) * 1.5).astype(np.float32).astype(np.float64)
    L_low = g.uniform(0, 3, (n, h, w, 3)).astype(np.float32).astype(np.float64)
    target = g.uniform(0, 1, (n, 4 * h, 4 * w, 3)).astype(np.float32).astype(np.float64)
    loss = torch.full((1,), 2.0, device="cuda")
    dconv6 = torch.empty((n, h, w, 48), dtype=torch.bfloat16, device="cuda")
    L_full = torch.empty((n, 4 * h, 4 * w, 3), device="cuda")
    rgb = nn.head(dev_f32(conv6), dev_f32(L_low), L_full=L_full, target=dev_f32(target),
                  loss_sum=loss, dconv6=dconv6)
    L, I = nr.head(conv6, L_low)
    assert (L == 0).mean() > 0.05
    assert np.abs(host(L_full) - L).max() <= 1e-5 * (1 + np.abs(L)).max()
    assert np.abs(host(rgb) - I).max() <= 2e-6
    assert host(loss)[0] == pytest.approx(2.0 + float(((I - target) ** 2).sum()), rel=1e-5)
    gref = nr.head_backward(L, I, target)
    got = host(dconv6)
    assert np.all(np.abs(got - gref) <= 2.0 ** -8 * np.abs(gref) + 1e-6 * np.abs(gref).max())


def test_adam_steps(nn):
    import torch
    g = np.random.default_rng(5)
    p0 = g.standard_normal(1000)
    grads = [g.standard_normal(1000) for _ in range(3)]
    p, m, v = p0.copy(), np.zeros(1000), np.zeros(1000)
    P, M, V = dev_f32(p0), torch.zeros(1000, device="cuda"), torch.zeros(1000, device="cuda")
    for t, gr in enumerate(grads, start=1):
        nr.adam_step(p, gr, m, v, t, lr=1e-2)
        nn.adam(P, dev_f32(gr), M, V, t, lr=1e-2)
    assert np.abs(host(P) - p).max() <= 1e-5


def test_to_bf16(nn):
    a = np.random.default_rng(6).standard_normal(4097).astype(np.float32)
    assert np.array_equal(host(nn.to_bf16(dev_f32(a))), bf16(a))


def test_consistency(nn):
    import torch
    g = np.random.default_rng(8)
    L_low = g.uniform(0, 2, (2, 6, 9, 3)).astype(np.float32).astype(np.float64)
    L_full = g.uniform(0, 2, (2, 24, 36, 3)).astype(np.float32).astype(np.float64)
    s = torch.zeros(1, device="cuda")
    nn.consistency(dev_f32(L_full), dev_f32(L_low), s)
    rms = math.sqrt(host(s)[0] / L_low.size)
    assert rms == pytest.approx(nr.consistency(L_full, L_low), rel=1e-5)


@pytest.mark.parametrize("h,w,region", [(32, 32, 64), (20, 27, 64), (16, 16, 16)])
def test_region_check(nn, h, w, region):
    """Per-region metric, mask and marked count against nn_ref; a NaN in
    one region marks it whatever theta."""
    import torch
    g = np.random.default_rng(h * w + region)
    L_low = g.uniform(0, 2, (1, h, w, 3)).astype(np.float32).astype(np.float64)
    L_full = g.uniform(0, 2, (1, 4 * h, 4 * w, 3)).astype(np.float32).astype(np.float64)
    L_full[0, 5, 6, 1] = np.nan                          # region 0
    ref = nr.region_consistency(L_full[0], L_low[0], region)
    nreg = ref.size
    theta = float(np.nanmedian(ref))
    mask = torch.full((nreg,), 7, dtype=torch.uint8, device="cuda")
    metric = torch.zeros(nreg, device="cuda")
    nm = torch.full((1,), 3, dtype=torch.int32, device="cuda")   # accumulated
    nn.region_check(dev_f32(L_full), dev_f32(L_low), region, theta, mask, nm, metric=metric)
    torch.cuda.synchronize()
    got = host(metric)
    assert np.isnan(got[0]) and np.isnan(ref[0])
    np.testing.assert_allclose(got[1:], ref[1:], rtol=1e-5)
    want = ~(ref <= theta)
    near = np.abs(ref - theta) <= 1e-5 * theta
    m = mask.cpu().numpy().astype(bool)
    assert np.array_equal(m[~near], want[~near]) and m[0]
    assert int(nm.item()) == 3 + int(m.sum())


def test_relu_passes_nan(nn):
    # a NaN weight must reach the output (the fallback test relies on it)
    x = np.ones((1, 4, 4, 32))
    wt = np.zeros((32, 3, 3, 32))
    wt[0, 1, 1, 0] = np.nan
    y = host(nn.conv3x3_fwd(dev_bf16(x), dev_bf16(wt), relu=True, out_f32=True))
    assert np.isnan(y[..., 0]).all() and not np.isnan(y[..., 1:]).any()


def test_errors(nn):
    import torch
    from paper_1309_1114_amd import splotch
    x = torch.zeros((1, 4, 4, 32), dtype=torch.bfloat16, device="cuda")
    w = torch.zeros((40, 3, 3, 32), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(splotch.SplotchError) as ei:
        nn.conv3x3_fwd(x, w)
    assert ei.value.status == splotch.ERR_UNSUPPORTED
    w2 = torch.zeros((48, 3, 3, 48), dtype=torch.bfloat16, device="cuda")
    x2 = torch.zeros((1, 4, 4, 48), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(splotch.SplotchError):
        nn.conv3x3_fwd(x2, w2)


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def bf16_storage_reference(params, x, L_low, target):
    """The FP64 reference with values rounded where the GPU path stores
    them: bf16 activations and data gradients, FP32 last layer output."""
    acts = [x]
    a = x
    for (w, b), (_, _, relu) in zip(params, nr.LAYERS):
        z = nr.conv3x3(a, w, b)
        a = bf16(np.maximum(z, 0.0)) if relu else _f32(z)
        acts.append(a)
    L, I = nr.head(acts[-1], L_low)
    g = bf16(nr.head_backward(L, I, target))
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        d = g * (acts[k + 1] > 0) if nr.LAYERS[k][2] else g
        grads[k] = nr.conv3x3_bwd_weight(acts[k], d)
        if k > 0:
            g = bf16(nr.conv3x3_bwd_data(d, params[k][0]))
    return grads, nr.mse(I, target)


def _network_case():
    params = nr.init_params(seed=3, scale_last=1.0)
    params = [(bf16(w), _f32(b + 0.01)) for w, b in params]
    g = np.random.default_rng(9)
    n, h, w = 2, 12, 20
    x = bf16(np.concatenate([g.uniform(0, 2, (n, h, w, 3)), g.uniform(0, 3, (n, h, w, 1))], -1))
    target = _f32(g.uniform(0, 1, (n, 4 * h, 4 * w, 3)))
    return params, x, _f32(x[..., :3]), target


def _gpu_gradients(params, x, L_low, target):
    from paper_1309_1114_amd.upscaler import Upscaler
    up = Upscaler(params=params)
    loss = up.train_step(dev_bf16(x), dev_f32(L_low), dev_f32(target), apply=False)
    return up.gradients(), loss


def _compare(ref, got, rel_max, cos_min):
    for k, ((rdw, rdb), (gdw, gdb)) in enumerate(zip(ref, got)):
        for r, gg in ((rdw, gdw), (rdb, gdb)):
            gg = gg.astype(np.float64)
            rel = np.linalg.norm(gg - r) / np.linalg.norm(r)
            cos = float((gg * r).sum() / (np.linalg.norm(gg) * np.linalg.norm(r)))
            assert rel <= rel_max and cos >= cos_min, (k, rel, cos)


def test_network_gradients_match_bf16_storage_reference(nn):
    """Full forward/backward through the GPU kernels against the FP64
    reference rounded at the GPU's storage points: the kernels differ only by
    FP32 accumulation order, so per layer the relative L2 error is <= 1e-3."""
    params, x, L_low, target = _network_case()
    got, loss = _gpu_gradients(params, x, L_low, target)
    ref, ref_loss = bf16_storage_reference(params, x, L_low, target)
    assert loss == pytest.approx(ref_loss, rel=1e-4)
    _compare(ref, got, 1e-3, 0.999999)


def test_network_gradients_match_reference(nn):
    """The same against the pure FP64 reference.  bf16 storage of
    activations and gradients (relative rounding 2^-9 at each of 11
    convolutions, amplified by cancellation in the sums) leaves a few
    percent: per layer relative L2 error <= 8e-2 and cosine >= 0.997."""
    params, x, L_low, target = _network_case()
    got, loss = _gpu_gradients(params, x, L_low, target)
    acts, L, I = nr.forward(params, x, L_low)
    ref = nr.backward(params, acts, L, I, target)
    assert loss == pytest.approx(nr.mse(I, target), rel=1e-2)
    _compare(ref, got, 8e-2, 0.997)
