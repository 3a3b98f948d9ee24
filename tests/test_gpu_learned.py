"""The learned serving path: the one-call network equals the kernel-by-kernel
network, the fallback returns exactly the plain full-resolution render, and
the trained weights gain over the path without the network (bilinear
upsampling of the same low-resolution render)."""
import math

import numpy as np
import pytest

from paper_1309_1114_amd import configs, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1309_1114_amd import splotch
    R = splotch.Renderer(0)
    cm = torch.from_numpy(synth.ramp_colormap()).cuda()
    yield R, cm
    R.close()


def small_scene(seed=20000, n=300_000, side=256, accum=0):
    """A C5-style frame at reduced size; accum=1 (int64) makes renders
    bitwise reproducible, so a fallback frame can be compared exactly."""
    from dataclasses import replace
    parts = synth.nbody_like_device(n, seed)
    cam = configs.c5_camera(seed, 0, side)
    prm = replace(configs.c5_params(side), accum=accum)
    return parts, cam, prm


def test_fused_upscale_equals_kernel_by_kernel(env):
    import torch
    from paper_1309_1114_amd import nn
    from paper_1309_1114_amd.upscaler import Upscaler
    R, cm = env
    up = Upscaler(seed=4)
    parts, cam, prm = small_scene()
    h = w = 64
    lc = synth.Camera(**{**cam.__dict__, "width": w, "height": h})
    la = torch.empty((1, h, w, 3), device="cuda")
    cc = torch.empty((1, h, w), dtype=torch.int32, device="cuda")
    R.render(parts, lc, cm, prm, log_accum=la[0], center_count=cc[0])
    x = nn.pack_input(la, cc)
    Lf1 = torch.empty((1, 4 * h, 4 * w, 3), device="cuda")
    rgb1 = up.forward(x, la, L_full=Lf1).clone()
    s1 = torch.zeros(1, device="cuda")
    nn.consistency(Lf1, la, s1)
    rgb2 = torch.empty_like(rgb1)
    Lf2 = torch.empty_like(Lf1)
    s2 = torch.full((1,), 123.0, device="cuda")     # the call overwrites it
    nn.upscale(up.weights_struct, la, cc, rgb2, L_full=Lf2, check=s2)
    torch.cuda.synchronize()
    assert torch.equal(rgb1, rgb2) and torch.equal(Lf1, Lf2)
    # the kernel-by-kernel sum uses atomics (any order), the fused one a
    # fixed order: equal to FP32 rounding, and the fused one reproducible
    assert float(s2) == pytest.approx(float(s1), rel=1e-5)
    s3 = torch.zeros(1, device="cuda")
    nn.upscale(up.weights_struct, la, cc, rgb2, L_full=Lf2, check=s3)
    torch.cuda.synchronize()
    assert float(s3) == float(s2)
    # a workspace one byte short is refused before any launch
    need = nn.upscale_workspace_size(1, h, w)
    with pytest.raises(Exception):
        nn.upscale(up.weights_struct, la, cc, rgb2, workspace=torch.empty(need - 1, dtype=torch.uint8,
                                                                         device="cuda"))


@pytest.mark.parametrize("theta,expect_fallback", [(-math.inf, True), (math.inf, False)])
def test_threshold_decides_fallback(env, theta, expect_fallback):
    import torch
    from paper_1309_1114_amd.upscaler import LearnedRenderer, Upscaler
    R, cm = env
    parts, cam, prm = small_scene(seed=20001, accum=1)
    LR = LearnedRenderer(R, Upscaler(seed=1), theta)
    out = LR.render(parts, cam, cm, prm)
    plain = R.render(parts, cam, cm, prm)
    torch.cuda.synchronize()
    assert LR.fallback == expect_fallback and math.isfinite(LR.metric) and LR.metric > 0
    assert LR.fallback_fraction == (1.0 if expect_fallback else 0.0)
    assert torch.equal(out, plain) == expect_fallback


def test_region_fallback_replaces_marked_regions(env):
    """A threshold between the regions' metrics: the marked regions hold the
    plain render bit for bit (int64), the others the network's image."""
    import torch
    from paper_1309_1114_amd import nn
    from paper_1309_1114_amd.upscaler import LearnedRenderer, Upscaler
    R, cm = env
    parts, cam, prm = small_scene(seed=20003, accum=1)
    up = Upscaler(seed=3)
    probe = LearnedRenderer(R, up, math.inf)
    net = probe.render(parts, cam, cm, prm).clone()
    metric = up._bufs[("region_metric", (probe.n_regions(cam),), torch.float32)].cpu().numpy()
    theta = float(np.median(metric))
    LR = LearnedRenderer(R, up, theta)
    out = LR.render(parts, cam, cm, prm)
    plain = R.render(parts, cam, cm, prm)
    torch.cuda.synchronize()
    marked = ~(metric <= theta)
    assert 0 < marked.sum() < marked.size
    assert LR.fallback_fraction == pytest.approx(marked.mean())
    side = cam.width // 64
    pm = np.repeat(np.repeat(marked.reshape(side, side), 64, 0), 64, 1)
    pm = torch.from_numpy(pm).cuda()
    assert torch.equal(out[pm], plain[pm]) and torch.equal(out[~pm], net[~pm])


def test_nan_weights_fall_back_to_the_plain_render(env):
    import torch
    from paper_1309_1114_amd.upscaler import LearnedRenderer, Upscaler, he_init
    R, cm = env
    params = he_init(2)
    params[2][0][0, 1, 1, 0] = np.nan
    LR = LearnedRenderer(R, Upscaler(params=params), theta=math.inf)
    parts, cam, prm = small_scene(seed=20002, accum=1)
    out = LR.render(parts, cam, cm, prm)
    plain = R.render(parts, cam, cm, prm)
    torch.cuda.synchronize()
    assert math.isnan(LR.metric) and LR.fallback
    assert torch.equal(out, plain)


def test_trained_network_beats_bilinear_on_heldout_frames(env):
    """Committed weights on three held-out C5 frames (2e7 particles,
    2048^2 from 512^2): the network's PSNR against the plain full render
    exceeds that of bilinear upsampling of the same low-resolution optical
    depth on every frame."""
    from paper_1309_1114_amd import c5
    from paper_1309_1114_amd.upscaler import Upscaler, default_weights_path
    R, cm = env
    up = Upscaler.load(default_weights_path())
    rows = c5.evaluate(R, up, cm, list(configs.C5_HELDOUT_SEEDS)[:3])
    for r in rows:
        assert r["psnr_net"] > r["psnr_bilinear"] + 0.2, r


def test_training_resumes_where_it_stopped(tmp_path):
    """Six training steps in one run, and a run of the same six-step
    schedule stopped after three, its checkpoint loaded and trained on: the
    checkpoint restores weights, moments and step
    exactly, the same crops are drawn (equal sampler states in the two
    step-6 checkpoints), and the weights agree.  The weight gradients sum
    with float atomics, and Adam turns a gradient near zero into a step of
    about lr whatever its size, so a few weights may differ by up to
    2 lr per step; the typical (median) weight agrees far more closely, as
    it does not when the resumed run draws other crops."""
    import json
    from types import SimpleNamespace

    import torch
    from paper_1309_1114_amd import c5
    from paper_1309_1114_amd.upscaler import SCALE, Upscaler
    g = torch.Generator(device="cpu").manual_seed(5)
    low, n = 48, 4
    pairs = SimpleNamespace(
        P=n,
        x=torch.rand((n, low, low, 4), generator=g).to(torch.bfloat16).cuda(),
        L=torch.rand((n, low, low, 3), generator=g).cuda(),
        t=torch.rand((n, SCALE * low, SCALE * low, 3), generator=g).cuda())
    lr = 2e-3
    kw = dict(batch=2, crop=24, lr=lr, seed=3, log_every=1000, ckpt_every=3)
    a = Upscaler(seed=1)
    c5.train(a, pairs, 6, ckpt=str(tmp_path / "a.npz"), **kw)
    b = Upscaler(seed=1)
    c5.train(b, pairs, 6, ckpt=str(tmp_path / "b3.npz"), until=3, **kw)
    r = Upscaler.load(str(tmp_path / "b3.npz"))
    assert b.step == r.step == 3
    for name in ("P", "M", "V"):
        assert torch.equal(getattr(b, name), getattr(r, name)), name
    c5.train(r, pairs, 6, ckpt=str(tmp_path / "r.npz"), rng_state=c5.checkpoint_rng_state(r),
             **kw)
    assert a.step == r.step == 6
    za, zr = np.load(tmp_path / "a.npz"), np.load(tmp_path / "r.npz")
    assert json.loads(str(za["meta_rng_state"])) == json.loads(str(zr["meta_rng_state"]))
    assert int(za["step"]) == int(zr["step"]) == 6
    d = np.abs(za["P"] - zr["P"])
    assert d.max() <= 2 * 6 * lr * 1.01, d.max()
    # a resumed run without the sampler state draws other crops
    w = Upscaler.load(str(tmp_path / "b3.npz"))
    c5.train(w, pairs, 6, ckpt=str(tmp_path / "w.npz"), **dict(kw, seed=4))
    dw = np.abs(za["P"] - np.load(tmp_path / "w.npz")["P"])
    assert float(np.median(d)) <= 1e-6, float(np.median(d))
    assert float(np.median(dw)) > 100 * max(float(np.median(d)), 1e-9), float(np.median(dw))
