"""The allocation-free render (splotch_render_noalloc) against splotch_render.

Both entry points are called through the C ABI on the same device inputs.
The allocation-free call takes its workspace from the library's fixed
per-device scratch, so consecutive calls share it: each case renders twice
in a row, the second time a smaller input, and compares both with the
workspace-taking render.  int64 images must be bit-identical; FP32 images
must agree within max|dI| <= 1e-5 (and with the FP64 oracle within the same
bound where it is run).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle
from paper_1309_1114_amd import splotch, synth
from paper_1309_1114_amd.synth import Camera, Params

pytestmark = pytest.mark.gpu
TOL = 1e-5
CMAP = synth.ramp_colormap()
SCRATCH = 512 << 20


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    r = splotch.Renderer(0)
    yield r
    r.close()


def _outs(cam, fill):
    import torch
    H, W = cam.height, cam.width
    return (torch.full((H, W, 3), fill, dtype=torch.float32, device="cuda:0"),
            torch.full((H, W, 3), fill, dtype=torch.float32, device="cuda:0"),
            torch.full((H, W), -1, dtype=torch.int32, device="cuda:0"))


def _both(R, parts, cam, prm):
    """(workspace render, allocation-free render) of the same inputs, each
    as host arrays (I, L, count), and the allocation-free call's stats."""
    import torch
    cm = torch.from_numpy(CMAP).cuda()
    a = _outs(cam, 7.0)
    R.render(parts, cam, cm, prm, rgb=a[0], log_accum=a[1], center_count=a[2])
    b = _outs(cam, -3.0)
    R.render_noalloc(parts, cam, cm, prm, rgb=b[0], log_accum=b[1], center_count=b[2])
    torch.cuda.synchronize()
    st = R.stats()
    return [t.cpu().numpy() for t in a], [t.cpu().numpy() for t in b], st


def _compare(a, b, accum):
    if accum == splotch.ACCUM_INT64:
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    else:
        err = float(np.abs(a[0].astype(np.float64) - b[0]).max())
        assert err <= TOL, f"max|dI| = {err:.3e}"
        assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("accum", [splotch.ACCUM_FP32, splotch.ACCUM_INT64])
def test_noalloc_equals_render_two_calls(R, accum):
    """A 131072-particle 512x512 frame, then a 20000-particle 160x120 frame
    in the same scratch: both equal splotch_render's images; the FP32 ones
    also match the oracle."""
    prm = Params(brightness=(0.02,) * 4, accum=accum)
    cases = [(synth.uniform_cube(131072, seed=0), Camera(width=512, height=512)),
             (synth.uniform_cube(20000, seed=5), Camera(width=160, height=120))]
    for ps, cam in cases:
        print(f"noalloc: n={ps.n} {cam.width}x{cam.height} accum={accum}", flush=True)
        a, b, st = _both(R, splotch.to_device(ps), cam, prm)
        assert st["passes"] == 1
        _compare(a, b, accum)
        if accum == splotch.ACCUM_FP32:
            ref = oracle.render(ps, cam, CMAP, prm)
            err = float(np.abs(b[0].astype(np.float64) - ref["I"]).max())
            assert err <= TOL, f"oracle max|dI| = {err:.3e}"


@pytest.mark.parametrize("accum", [splotch.ACCUM_FP32, splotch.ACCUM_INT64])
def test_noalloc_chunked_set(R, accum):
    """3e6 clustered particles at 1024x1024 need more than the fixed
    scratch for one pass: the allocation-free call renders them in several
    chunks and still equals the one-pass render; then a small set reuses
    the scratch."""
    import torch
    parts = synth.nbody_like_device(3_000_000, 41)
    cam = Camera(width=1024, height=1024)
    b = 0.05
    prm = Params(brightness=(b,) * 4, fixed_sigma_frac=(0.0, 1.0 / 1024, 0.0, 0.0), accum=accum)
    need = R.workspace_size(splotch.particles_struct(parts), cam, prm)
    assert need > SCRATCH
    print(f"noalloc chunked: accum={accum} one-pass workspace {need / 2**20:.0f} MiB", flush=True)
    a, bb, st = _both(R, parts, cam, prm)
    assert st["passes"] > 1
    _compare(a, bb, accum)
    small = {k: (None if v is None else v[:50000].contiguous()) for k, v in parts.items()}
    cam2 = Camera(width=640, height=480)
    a, bb, st = _both(R, small, cam2, prm)
    assert st["passes"] == 1
    _compare(a, bb, accum)
    del parts
    torch.cuda.empty_cache()


def test_noalloc_rejects_an_image_beyond_the_scratch(R):
    """8192x8192 in int64 mode needs 1.5 GiB of optical-depth planes: the
    call fails before any launch and leaves the outputs untouched."""
    import torch
    ps = synth.uniform_cube(1000, seed=3)
    cam = Camera(width=8192, height=8192)
    prm = Params(accum=splotch.ACCUM_INT64)
    rgb = torch.full((8192, 8192, 3), 7.0, dtype=torch.float32, device="cuda:0")
    with pytest.raises(splotch.SplotchError) as e:
        R.render_noalloc(splotch.to_device(ps), cam, torch.from_numpy(CMAP).cuda(), prm, rgb=rgb)
    assert e.value.status == splotch.ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((rgb == 7.0).all())
    del rgb
    torch.cuda.empty_cache()


def test_noalloc_ordered_transfer_unsupported(R):
    import torch
    ps = synth.uniform_cube(1000, seed=3)
    cam = Camera(width=64, height=64)
    prm = Params(absorption=(0.01,) * 4, transfer=1)
    rgb = torch.full((64, 64, 3), 7.0, dtype=torch.float32, device="cuda:0")
    with pytest.raises(splotch.SplotchError) as e:
        R.render_noalloc(splotch.to_device(ps), cam, torch.from_numpy(CMAP).cuda(), prm, rgb=rgb)
    assert e.value.status == splotch.ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((rgb == 7.0).all())
