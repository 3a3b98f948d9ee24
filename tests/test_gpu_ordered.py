"""GPU parity of the ordered render (emission and absorption independent).

The HIP path (depth sort, per-tile entry lists, front-to-back compositing)
is compared with the FP64 oracle's per-pixel sorted compositing on the same
seeded inputs: max|dI| <= 1e-5.  Per-particle coefficients stay <= 0.05 (the
FP32 screen-position budget), density supplies the optical depth.  The
result must be bit-identical from run to run; a different number of passes
regroups the associative merge of a tile's work items, so it agrees to
rounding (1e-6).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle
from paper_1309_1114_amd import splotch, synth
from paper_1309_1114_amd.synth import Camera, Params
from scenes import lattice_camera, lattice_scene

pytestmark = pytest.mark.gpu
TOL = 1e-5
CMAP = synth.ramp_colormap()
CAM = Camera(eye=(0.5, 0.5, -1.5), target=(0.5, 0.5, 0.5), fov_deg=45.0, width=121, height=91)
# species 0 (sigma 1.5 px): emits 2.5 times what it absorbs; species 1
# (sigma 1 px): dust, absorbs only.  About 1200 samples per pixel.
PRM = Params(chi=3.0, brightness=(0.05, 0.0, 0.0, 0.0), absorption=(0.02, 0.05, 0.0, 0.0),
             fixed_sigma_frac=(1.5 / 121, 1.0 / 121, 0.0, 0.0), transfer=1)


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    r = splotch.Renderer(0)
    yield r
    r.close()


@pytest.fixture(scope="module")
def scene():
    return synth.nbody_like(300_001, seed=31)


def render(R, ps, cam, prm, cmap=CMAP, want_L=False, ws_bytes=None):
    import torch
    parts = splotch.to_device(ps)
    cm = None if cmap is None else torch.from_numpy(np.ascontiguousarray(cmap)).cuda()
    rgb = torch.full((cam.height, cam.width, 3), 7.0, device="cuda:0")
    la = torch.empty_like(rgb) if want_L else None
    kw = {}
    if ws_bytes is not None:
        kw = dict(workspace=torch.empty(ws_bytes, dtype=torch.uint8, device="cuda:0"),
                  workspace_bytes=ws_bytes)
    R.render(parts, cam, cm, prm, rgb=rgb, log_accum=la, **kw)
    torch.cuda.synchronize()
    out = dict(I=rgb.cpu().numpy(), stats=R.stats())
    if want_L:
        out["L"] = la.cpu().numpy()
    return out


def test_ordered_parity_with_oracle(R, scene):
    ref = oracle.render(scene, CAM, CMAP, PRM)
    assert 0.2 < float(np.median(ref["L"][..., 1])) < 5.0
    assert ref["I"].max() > 0.3
    gpu = render(R, scene, CAM, PRM, want_L=True)
    err = np.abs(gpu["I"].astype(np.float64) - ref["I"]).max()
    assert err <= TOL, err
    errL = np.abs(gpu["L"].astype(np.float64) - ref["L"]).max() / max(1.0, ref["L"].max())
    assert errL <= TOL, errL
    assert gpu["stats"]["n_input"] == scene.n
    assert gpu["stats"]["n_active"] == ref["active"]
    assert gpu["stats"]["passes"] == 1
    # the order matters here: the order-free image of the same emission differs
    ea = oracle.render(scene, CAM, CMAP, replace(PRM, transfer=0))
    assert np.abs(ea["I"] - ref["I"]).max() > 100 * TOL


@pytest.mark.parametrize("scale", [0.1, 20.0])
def test_ordered_series_and_expm1_paths_match_the_oracle(R, scene, scale):
    """Absorption scaled so that every record takes the short series of
    (1 - exp(-t))/t (scale 0.1: all coefficients below 2^-7), or so that the
    central samples of most records need expm1 (scale 20: t up to 1)."""
    prm = replace(PRM, brightness=tuple(scale * b for b in PRM.brightness),
                  absorption=tuple(scale * a for a in PRM.absorption))
    sub = synth.ParticleSet(*[None if a is None else a[:60_000] for a in
                              (scene.x, scene.y, scene.z, scene.h, scene.intensity,
                               scene.scalar, scene.species)])
    ref = oracle.render(sub, CAM, CMAP, prm)
    gpu = render(R, sub, CAM, prm, want_L=True)
    err = np.abs(gpu["I"].astype(np.float64) - ref["I"]).max()
    assert err <= TOL, err
    errL = np.abs(gpu["L"].astype(np.float64) - ref["L"]).max() / max(1.0, ref["L"].max())
    assert errL <= TOL, errL
    assert ref["I"].max() > 0.05


def test_ordered_run_to_run_bit_exact_and_passes(R, scene):
    import torch
    full = render(R, scene, CAM, PRM)
    again = render(R, scene, CAM, PRM)
    assert np.array_equal(full["I"], again["I"])
    # a workspace far below the queried size: many passes, the same image
    need = R.workspace_size(splotch.particles_struct(splotch.to_device(scene)), CAM, PRM)
    small = need - (15 << 20)
    out = render(R, scene, CAM, PRM, ws_bytes=small)
    assert out["stats"]["passes"] >= 3, out["stats"]["passes"]
    assert np.abs(out["I"].astype(np.float64) - full["I"]).max() <= 1e-6
    again = render(R, scene, CAM, PRM, ws_bytes=small)
    assert np.array_equal(out["I"], again["I"])
    torch.cuda.synchronize()


def test_ordered_equal_coefficients_match_the_order_free_render(R, scene):
    eq = replace(PRM, brightness=(0.05, 0.05, 0, 0), absorption=(0.05, 0.05, 0, 0))
    a = render(R, scene, CAM, eq)
    b = render(R, scene, CAM, replace(eq, transfer=0))
    assert np.abs(a["I"].astype(np.float64) - b["I"]).max() <= TOL


def test_ordered_disk_edges_count(R):
    # chi = 1: a sample on the disk's rim weighs e^-1 of the peak, so a
    # record wrongly skipped by a wave (its quadrant test) would show far
    # above the tolerance (dropping the outermost ring of every disk, chi
    # 0.97, moves every pixel past it).  64 x 48 pixels, fixed sigmas of 1.5
    # and 2.5 pixels, rims across quadrant and tile borders; lattice
    # positions keep every pixel centre 1/8 px^2 away from every rim, so
    # the in-disk decisions are exact on both sides, and nine depths give
    # many equal depths, ordered by index.
    W, H = 64, 48
    ps, _, _ = lattice_scene(60_001, W, H, seed=35, n_species=2)
    cam = lattice_camera(W, H)
    prm = replace(PRM, chi=1.0, fixed_sigma_frac=(1.5 / W, 2.5 / W, 0.0, 0.0))
    ref = oracle.render(ps, cam, CMAP, prm)
    assert ref["I"].max() > 0.3
    gpu = render(R, ps, cam, prm)
    assert np.abs(gpu["I"].astype(np.float64) - ref["I"]).max() <= TOL
    assert gpu["stats"]["n_active"] == ref["active"]


def test_ordered_vector_colour(R):
    ps = synth.nbody_like(200_003, seed=32)
    v = np.random.default_rng(32).normal(0.0, 0.8, size=(3, ps.n)).astype(np.float32)
    ps.vx, ps.vy, ps.vz = v
    ps.scalar = None
    prm = replace(PRM, colour_mode=1, scalar_min=-1.0, scalar_max=1.0)
    ref = oracle.render(ps, CAM, None, prm)
    gpu = render(R, ps, CAM, prm, cmap=None)
    assert np.abs(gpu["I"].astype(np.float64) - ref["I"]).max() <= TOL


def test_ordered_empty_and_invisible(R):
    e = np.zeros(0, np.float32)
    empty = synth.ParticleSet(e, e, e, e, e, e, None)
    out = render(R, empty, CAM, PRM)
    assert float(np.abs(out["I"]).max()) == 0.0
    ps = synth.uniform_cube(1000, seed=3)
    behind = replace(ps, z=(ps.z - np.float32(5.0)).astype(np.float32))
    out = render(R, behind, CAM, PRM)
    assert float(np.abs(out["I"]).max()) == 0.0 and out["stats"]["n_active"] == 0


def test_ordered_error_paths(R):
    import torch
    ps = synth.uniform_cube(100, seed=1)
    parts = splotch.to_device(ps)
    cm = torch.from_numpy(CMAP).cuda()
    rgb = torch.full((32, 32, 3), 7.0, device="cuda:0")
    cam = Camera(width=32, height=32)
    cases = [
        (replace(PRM, accum=1), splotch.ERR_UNSUPPORTED),
        (replace(PRM, absorption=(-1.0, 0, 0, 0)), splotch.ERR_INVALID_ARG),
        (replace(PRM, absorption=(float("nan"), 0, 0, 0)), splotch.ERR_INVALID_ARG),
        (replace(PRM, transfer=2), splotch.ERR_INVALID_ARG),
    ]
    for prm, code in cases:
        with pytest.raises(splotch.SplotchError) as ei:
            R.render(parts, cam, cm, prm, rgb=rgb)
        assert ei.value.status == code, prm
    jobs = R.make_jobs([dict(parts=parts, cam=cam, cmap=cm, prm=PRM, rgb=rgb)])
    with pytest.raises(splotch.SplotchError) as ei:
        R.render_batched(jobs)
    assert ei.value.status == splotch.ERR_UNSUPPORTED
    # nor streamed from host memory, nor autotuned
    with pytest.raises(splotch.SplotchError) as ei:
        R.render_streamed(splotch.to_host(ps, pinned=False), cam, cm, PRM, chunk=64, rgb=rgb)
    assert ei.value.status == splotch.ERR_UNSUPPORTED
    with pytest.raises(splotch.SplotchError) as ei:
        R.autotune(parts, cam, cm, PRM, rgb)
    assert ei.value.status == splotch.ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((rgb == 7.0).all())


def test_ordered_oblique_camera_with_depth_ties(R):
    """An oblique camera gives depths with full double mantissas (the sort
    maps them to 32 bits with a loss of precision and reorders the runs of
    equal 32-bit keys by the full depth); every tenth particle is doubled
    with another species at the same position, so equal depths must be
    taken in index order as the oracle takes them."""
    base = synth.nbody_like(150_000, seed=32)
    sel = np.arange(0, base.n, 10)
    cat = lambda a, b: np.concatenate([a, b])
    sp = base.species if base.species is not None else np.zeros(base.n, np.uint8)
    ps = synth.ParticleSet(cat(base.x, base.x[sel]), cat(base.y, base.y[sel]),
                           cat(base.z, base.z[sel]), cat(base.h, base.h[sel]),
                           cat(base.intensity, base.intensity[sel]),
                           cat(base.scalar, 1.0 - base.scalar[sel]),
                           cat(sp, (1 - np.minimum(sp[sel], 1)).astype(np.uint8)))
    cam = Camera(eye=(1.9, 1.3, -1.1), target=(0.45, 0.55, 0.5), fov_deg=40.0, width=127,
                 height=95)
    ref = oracle.render(ps, cam, CMAP, PRM)
    out = render(R, ps, cam, PRM)
    err = np.abs(out["I"].astype(np.float64) - ref["I"]).max()
    assert ref["I"].max() > 0.05 and err <= TOL, err


def test_ordered_screen_filling_particles_with_minimal_workspace(R):
    """Five particles cover the whole 1152x1088 image (4896 tiles of 16
    pixels each) beside 3000 small ones.  With the smallest workspace the
    call accepts, a pass holds fewer entries than one such particle has:
    its entries run over several passes.  The image equals the one-pass
    render to rounding and the oracle within 1e-5."""
    import torch
    g = np.random.default_rng(37)
    small = synth.uniform_cube(3000, seed=37)
    n_big = 5
    f32 = lambda a: np.asarray(a, np.float32)
    ps = synth.ParticleSet(
        f32(np.concatenate([0.5 + 0.02 * g.standard_normal(n_big), small.x])),
        f32(np.concatenate([0.5 + 0.02 * g.standard_normal(n_big), small.y])),
        f32(np.concatenate([-1.0 + 0.1 * np.arange(n_big), small.z])),
        f32(np.concatenate([np.full(n_big, 0.5), small.h])),
        f32(np.ones(n_big + small.n)),
        f32(np.concatenate([g.random(n_big), small.scalar])),
        np.zeros(n_big + small.n, np.uint8))
    cam = Camera(width=1152, height=1088, fov_deg=40.0)
    prm = replace(PRM, brightness=(0.03,) * 4, absorption=(0.02,) * 4, fixed_sigma_frac=(0.0,) * 4)
    full = render(R, ps, cam, prm)
    assert full["stats"]["passes"] == 1
    parts = splotch.to_device(ps)
    need = R.workspace_size(splotch.particles_struct(parts), cam, prm)
    cm = torch.from_numpy(CMAP).cuda()
    rgb = torch.empty((cam.height, cam.width, 3), device="cuda:0")
    lo, hi = 1 << 20, need            # the smallest accepted size, to 64 KiB
    while hi - lo > (64 << 10):
        mid = (lo + hi) // 2 // 256 * 256
        try:
            R.render(parts, cam, cm, prm, rgb=rgb, workspace=torch.empty(mid, dtype=torch.uint8,
                                                                          device="cuda:0"),
                     workspace_bytes=mid)
            hi = mid
        except splotch.SplotchError as e:
            assert e.status == splotch.ERR_WORKSPACE
            lo = mid
        torch.cuda.synchronize()
    out = render(R, ps, cam, prm, ws_bytes=hi)
    assert out["stats"]["passes"] >= 2, out["stats"]["passes"]
    assert np.abs(out["I"].astype(np.float64) - full["I"]).max() <= 1e-6
    ref = oracle.render(ps, cam, CMAP, prm)
    assert ref["I"].min() > 0.0
    assert np.abs(out["I"].astype(np.float64) - ref["I"]).max() <= TOL


def test_ordered_depth_order_finer_than_the_32_bit_keys(R):
    """400 particles stacked on one spot at depths 1.5 + k * 2e-12 (distinct
    doubles, nearer with every index) and a few far behind them at depth
    1e4: the sort maps the depth bits to 32 bits by dropping the low 24, so
    the stack falls into one or two runs of equal keys whose order comes
    from the dropped bits alone (every neighbour pair is out of index
    order).  The composite must follow the exact depths, as the oracle's
    per-pixel sort does."""
    n_stack, n_far = 400, 8
    k = np.arange(n_stack)
    f32 = lambda a: np.asarray(a, np.float32)
    z = np.concatenate([(n_stack - k) * 2e-12, np.full(n_far, 1.0e4)])
    assert len(np.unique(f32(z))) == n_stack + 1
    n = n_stack + n_far
    # emitters and dust alternate along the stack (one emission-to-absorption
    # ratio for all would make the composite order-free)
    ps = synth.ParticleSet(
        f32(np.full(n, 0.5)), f32(np.full(n, 0.5)), f32(z), f32(np.full(n, 0.002)),
        f32(np.ones(n)), f32(np.concatenate([k / n_stack, np.full(n_far, 0.5)])),
        np.concatenate([k % 2, np.zeros(n_far, np.int64)]).astype(np.uint8))
    prm = PRM
    ref = oracle.render(ps, CAM, CMAP, prm)
    out = render(R, ps, CAM, prm)
    err = np.abs(out["I"].astype(np.float64) - ref["I"]).max()
    assert ref["I"].max() > 0.2 and err <= TOL, err
    # the stack's order shows: the same particles taken back to front by index
    rev = synth.ParticleSet(ps.x, ps.y, f32(np.concatenate([k * 2e-12 + 2e-12, z[n_stack:]])),
                            ps.h, ps.intensity, ps.scalar, ps.species)
    other = oracle.render(rev, CAM, CMAP, prm)
    assert np.abs(other["I"] - ref["I"]).max() > 100 * TOL


def test_ordered_long_run_below_the_32_bit_keys(R):
    """20000 particles on one spot, all in one run of equal 32-bit sort keys
    and in reverse depth order by index (depths 1.5 + k * 1e-13, with a far
    particle stretching the key range): the run is put in order by the
    dropped key bits with work that grows as m log m, and the composite
    still follows the exact depths."""
    n_stack = 20000
    k = np.arange(n_stack)
    f32 = lambda a: np.asarray(a, np.float32)
    z = np.concatenate([(n_stack - k) * 1e-13, [1.0e4]])
    assert len(np.unique(f32(z))) == n_stack + 1
    n = n_stack + 1
    ps = synth.ParticleSet(
        f32(np.full(n, 0.5)), f32(np.full(n, 0.5)), f32(z), f32(np.full(n, 0.002)),
        f32(np.ones(n)), f32(np.concatenate([(k % 97) / 97.0, [0.5]])),
        np.concatenate([k % 2, [0]]).astype(np.uint8))
    prm = replace(PRM, brightness=(0.002, 0.0, 0.0, 0.0), absorption=(0.001, 0.002, 0.0, 0.0))
    ref = oracle.render(ps, CAM, CMAP, prm)
    out = render(R, ps, CAM, prm)
    err = np.abs(out["I"].astype(np.float64) - ref["I"]).max()
    assert ref["I"].max() > 0.05 and err <= TOL, err
