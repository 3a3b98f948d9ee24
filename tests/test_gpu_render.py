"""GPU parity of the HIP render path against the FP64 oracle.

Every render goes through the C ABI (libsplotch.so via the ctypes binding).
FP32 accumulation must match the oracle within max|dI| <= 1e-5 on the [0,1]
image; the int64 fixed-point mode must match the oracle within the same
bound and be bit-identical across runs, schedules and particle orders.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle
from paper_1309_1114_amd import configs, splotch, synth
from paper_1309_1114_amd.synth import Camera, Params, ParticleSet
from scenes import lattice_camera, lattice_scene

pytestmark = pytest.mark.gpu
TOL = 1e-5
CMAP = synth.ramp_colormap()


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    r = splotch.Renderer(0)
    yield r
    r.close()


def gpu_render(R, ps, cam, prm, want_L=False, want_count=False, cmap=CMAP, ws_bytes=None,
               check_stats=True):
    import torch
    dev = "cuda:0"
    parts = splotch.to_device(ps, dev)
    cm = None if cmap is None else torch.from_numpy(np.ascontiguousarray(cmap, np.float32)).to(dev)
    H, W = cam.height, cam.width
    rgb = torch.full((H, W, 3), 7.0, dtype=torch.float32, device=dev)
    la = torch.empty((H, W, 3), dtype=torch.float32, device=dev) if want_L else None
    cc = torch.empty((H, W), dtype=torch.int32, device=dev) if want_count else None
    kw = {}
    if ws_bytes is not None:
        kw = dict(workspace=torch.empty(ws_bytes, dtype=torch.uint8, device=dev),
                  workspace_bytes=ws_bytes)
    R.render(parts, cam, cm, prm, rgb=rgb, log_accum=la, center_count=cc, **kw)
    torch.cuda.synchronize()
    out = dict(I=rgb.cpu().numpy(), stats=R.stats(check=check_stats))
    if want_L:
        out["L"] = la.cpu().numpy()
    if want_count:
        out["count"] = cc.cpu().numpy()
    return out


def assert_parity(gpu, ref, tol=TOL):
    err = np.abs(gpu["I"].astype(np.float64) - ref["I"]).max()
    assert err <= tol, f"max|dI| = {err:.3e} > {tol}"
    return err


def brightness_for(ps, cam, prm, target=0.7, **kw):
    """Brightness giving median green optical depth `target` (test input)."""
    one = replace(prm, brightness=(1.0,) * 4)
    L = oracle.render(ps, cam, CMAP, one, want_image=False, **kw)["L"]
    return target / float(np.median(L[..., 1][L[..., 1] > 0]))


# ---------------------------------------------------------------------------
# Config 1: uniform cube, 131072 particles, 512x512.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1():
    ps, cam, prm = configs.c1()
    ref = oracle.render(ps, cam, CMAP, prm, want_count=True)
    return ps, cam, prm, ref


def test_c1_fp32_parity(R, c1):
    ps, cam, prm, ref = c1
    out = gpu_render(R, ps, cam, prm, want_L=True, want_count=True)
    assert_parity(out, ref)
    assert np.abs(out["L"] - ref["L"]).max() <= 1e-5 * (1 + ref["L"].max())
    st = out["stats"]
    assert st["n_input"] == ps.n
    assert abs(st["n_active"] - ref["active"]) <= 2
    assert out["count"].sum() == ref["count"].sum()
    assert (out["count"] != ref["count"]).mean() < 1e-4


def test_c1_int64_parity_and_run_to_run(R, c1):
    ps, cam, prm, ref = c1
    p64 = replace(prm, accum=1)
    a = gpu_render(R, ps, cam, p64)
    b = gpu_render(R, ps, cam, p64)
    assert_parity(a, ref)
    assert np.array_equal(a["I"].view(np.uint32), b["I"].view(np.uint32))


@pytest.mark.parametrize("knobs", [
    dict(tile=8, halo=0, max_clip_tiles=1, chunk=32),
    dict(tile=16, halo=4, max_clip_tiles=2, chunk=64),
    dict(tile=32, halo=8, max_clip_tiles=4, chunk=1024),
    dict(tile=64, halo=4, max_clip_tiles=16, chunk=4096),
    dict(tile=32, halo=0, max_clip_tiles=64, chunk=256),
    dict(tile=16, halo=16, max_clip_tiles=1, chunk=8191),
])
def test_int64_bit_exact_across_schedules(R, c1, knobs):
    ps, cam, prm, ref = c1
    base = gpu_render(R, ps, cam, replace(prm, accum=1))
    other = gpu_render(R, ps, cam, replace(prm, accum=1, **knobs))
    assert np.array_equal(base["I"].view(np.uint32), other["I"].view(np.uint32)), knobs


def test_int64_bit_exact_under_permutation(R, c1):
    ps, cam, prm, ref = c1
    perm = np.random.default_rng(7).permutation(ps.n)
    a = gpu_render(R, ps, cam, replace(prm, accum=1))
    b = gpu_render(R, ps.subset(perm), cam, replace(prm, accum=1))
    assert np.array_equal(a["I"].view(np.uint32), b["I"].view(np.uint32))


@pytest.mark.parametrize("knobs", [dict(tile=8, halo=0, max_clip_tiles=1),
                                   dict(tile=64, halo=4, max_clip_tiles=64)])
def test_fp32_parity_other_schedules(R, c1, knobs):
    ps, cam, prm, ref = c1
    assert_parity(gpu_render(R, ps, cam, replace(prm, **knobs)), ref)


# ---------------------------------------------------------------------------
# Ragged sizes, degenerate inputs.
# ---------------------------------------------------------------------------
def test_ragged_image_and_particle_tail(R):
    ps = synth.uniform_cube(50001, seed=3)
    cam = Camera(width=333, height=197, fov_deg=50.0)
    prm = Params(chi=3.0, brightness=(0.03,) * 4)
    ref = oracle.render(ps, cam, CMAP, prm)
    assert_parity(gpu_render(R, ps, cam, prm), ref)
    assert_parity(gpu_render(R, ps, cam, replace(prm, accum=1, tile=16)), ref)


@pytest.fixture(scope="module")
def rims():
    # chi = 1: a sample on a disk's rim weighs e^-1 of its particle's peak,
    # so a sample dropped or added at a disk's edge (segment bounds, halo and
    # clip borders, the large pass) shows far above the tolerance (dropping
    # the outermost ring of every disk, chi 0.97, moves 98% of these pixels
    # past it).  Lattice positions keep every pixel centre 1/8 px^2 away from
    # every rim, so the in-disk decisions are exact on both sides: with
    # random positions a centre within FP32 rounding of a rim (|d^2 - R^2|
    # about 1e-6 R^2) flips one whole sample.
    W, H = 256, 192
    ps, _, _ = lattice_scene(100_001, W, H, seed=36)
    cam = lattice_camera(W, H)
    prm = Params(chi=1.0, brightness=(0.01,) * 4,
                 fixed_sigma_frac=(2.5 / W, 1.5 / W, 6.0 / W, 0.0))
    return ps, cam, prm, oracle.render(ps, cam, CMAP, prm)


@pytest.mark.parametrize("knobs", [dict(), dict(tile=8, halo=0, max_clip_tiles=1),
                                   dict(tile=16, halo=4, max_clip_tiles=2),
                                   dict(tile=64, halo=4, max_clip_tiles=64)])
def test_small_chi_rims(R, rims, knobs):
    ps, cam, prm, ref = rims
    assert ref["I"].max() > 0.2
    assert_parity(gpu_render(R, ps, cam, replace(prm, **knobs)), ref)
    assert_parity(gpu_render(R, ps, cam, replace(prm, accum=1, **knobs)), ref)


def test_single_particle_closed_form(R):
    # eye at the origin looking down +z: X = 36, Y = 22, sigma = 2, R = 6
    cam = Camera(eye=(0.0, 0.0, 0.0), target=(0.0, 0.0, 1.0), up=(0, 1, 0), fov_deg=90.0,
                 width=64, height=48)
    f1 = lambda v: np.array([v], np.float32)
    ps = ParticleSet(f1(-0.25), f1(0.125), f1(2.0), f1(0.125), f1(0.75), f1(0.25),
                     np.zeros(1, np.uint8))
    prm = Params(chi=3.0, brightness=(0.5, 0, 0, 0))
    out = gpu_render(R, ps, cam, prm, want_L=True)
    i = np.arange(64) + 0.5
    j = np.arange(48) + 0.5
    d2 = (i[None, :] - 36.0) ** 2 + (j[:, None] - 22.0) ** 2
    e = np.where(d2 <= 36.0, np.exp(-d2 / 4.0), 0.0)
    u = 0.25 * 255                          # palette position 63.75
    m = int(math.floor(u))
    t = u - m
    col = (1 - t) * CMAP[m].astype(np.float64) + t * CMAP[m + 1].astype(np.float64)
    exp_L = e[..., None] * (0.5 * 0.75 * col)[None, None, :]
    assert np.abs(out["L"] - exp_L).max() <= 1e-6 * exp_L.max()
    assert np.all(out["L"][d2 > 36.0] == 0.0)


def test_empty_and_invisible(R):
    cam = Camera(width=100, height=60)
    e = np.zeros(0, np.float32)
    empty = ParticleSet(e, e, e, e, e, e, None)
    out = gpu_render(R, empty, cam, Params())
    assert np.all(out["I"] == 0.0) and out["stats"]["n_active"] == 0
    ps = synth.uniform_cube(1000, seed=1)
    behind = ParticleSet(ps.x, ps.y, ps.z - np.float32(3.0), ps.h, ps.intensity, ps.scalar,
                         ps.species)
    out = gpu_render(R, behind, cam, Params(brightness=(1.0,) * 4))
    assert np.all(out["I"] == 0.0) and out["stats"]["n_active"] == 0


@pytest.mark.parametrize("accum", [0, 1])
def test_footprints_between_pixel_centres(R, accum):
    """Particles centred 1/64 px right of and below pixel corners, so that
    the nearest pixel centre is 0.685 px away.  With R = 0.6 px no pixel
    centre lies in the disk: nothing is drawn, yet each particle whose
    centre is in the image counts once at the pixel holding it.  With
    R = 0.75 px the four nearest centres (0.685 to 0.729 px) are drawn."""
    W, H, n = 64, 48, 3000
    rng = np.random.default_rng(17)
    X = rng.integers(-2, W + 3, n) + 1.0 / 64.0
    Y = rng.integers(-2, H + 3, n) + 1.0 / 64.0
    z = rng.choice([1.0, 2.0, 4.0], n)
    f = W / 2.0
    x = ((W / 2.0 - X) * z / f).astype(np.float32)
    y = ((H / 2.0 - Y) * z / f).astype(np.float32)
    assert np.array_equal(x.astype(np.float64), (W / 2.0 - X) * z / f)
    assert np.array_equal(y.astype(np.float64), (H / 2.0 - Y) * z / f)
    f32 = lambda a: np.asarray(a, np.float32)
    ps = ParticleSet(x, y, f32(z), f32(np.full(n, 0.01)), f32(np.ones(n)),
                     f32(rng.uniform(0.0, 1.0, n)), None)
    cam = lattice_camera(W, H)
    inside = (X >= 0) & (X < W) & (Y >= 0) & (Y < H)
    want = np.zeros((H, W), np.int64)
    np.add.at(want, (np.floor(Y[inside]).astype(int), np.floor(X[inside]).astype(int)), 1)
    for sigma, b, draws in ((0.2, 0.05, False), (0.25, 100.0, True)):
        prm = Params(chi=3.0, brightness=(b,) * 4, fixed_sigma_frac=(sigma / W,) * 4,
                     accum=accum)
        ref = oracle.render(ps, cam, CMAP, prm, want_count=True)
        assert np.array_equal(ref["count"], want)
        out = gpu_render(R, ps, cam, prm, want_count=True)
        assert np.array_equal(out["count"], want)
        assert_parity(out, ref)
        if draws:
            assert ref["I"].max() > 0.01
        else:
            assert ref["I"].max() == 0.0 and float(np.abs(out["I"]).max()) == 0.0


def test_infinite_coefficient_stays_inside_its_disk(R):
    """A particle of infinite intensity (it goes to the large pass) among
    ordinary ones: its disk resolves to I = 1 and every other pixel matches
    the oracle, finite (its infinite coefficient never meets a pixel outside
    the disk, not even with a zero weight)."""
    ps = synth.uniform_cube(3000, seed=9)
    ps.intensity[0] = np.inf
    ps.h[0] = 0.05          # a disk of about 15 px
    cam = Camera(width=160, height=120)
    prm = Params(chi=3.0, brightness=(0.02,) * 4)
    ref = oracle.render(ps, cam, CMAP, prm)
    out = gpu_render(R, ps, cam, prm, check_stats=False)
    assert out["stats"]["n_large"] >= 1
    hot = ~np.isfinite(ref["L"]).all(axis=2)
    assert 0 < hot.sum() < hot.size // 2
    assert np.all(out["I"][hot] == 1.0)
    cold = ~hot
    assert np.all(np.isfinite(out["I"][cold]))
    assert np.abs(out["I"][cold].astype(np.float64) - ref["I"][cold]).max() <= 1e-5


def test_one_pixel_image_and_huge_particle(R):
    ps = synth.uniform_cube(2000, seed=4)
    for W, H in ((1, 1), (1, 37), (53, 1)):
        cam = Camera(width=W, height=H, fov_deg=30.0)
        prm = Params(brightness=(0.01,) * 4)
        assert_parity(gpu_render(R, ps, cam, prm), oracle.render(ps, cam, CMAP, prm))
    # one particle filling the whole screen (large path only)
    f1 = lambda v: np.array([v], np.float32)
    big = ParticleSet(f1(0.5), f1(0.5), f1(0.0), f1(0.4), f1(1.0), f1(0.5), None)
    cam = Camera(width=300, height=200)
    prm = Params(brightness=(0.5,) * 4)
    out = gpu_render(R, big, cam, prm)
    assert out["stats"]["n_large"] == 1
    assert_parity(out, oracle.render(big, cam, CMAP, prm))


# ---------------------------------------------------------------------------
# Config 3 slice (large footprints) and config 2 slice (clustered, 1080p).
# ---------------------------------------------------------------------------
def test_c3_slice_large_footprints(R):
    ps = synth.pareto_cube(200_000, seed=2)
    cam = Camera(eye=(0.5, 0.5, 0.5), target=(0.5, 0.5, 1.0), fov_deg=90.0,
                 width=512, height=512)
    prm = Params(chi=3.0)
    prm = replace(prm, brightness=(brightness_for(ps, cam, prm),) * 4)
    ref = oracle.render(ps, cam, CMAP, prm)
    out = gpu_render(R, ps, cam, prm)
    assert out["stats"]["n_large"] > 100
    assert_parity(out, ref)
    out64 = gpu_render(R, ps, cam, replace(prm, accum=1))
    assert_parity(out64, ref)


def test_c2_slice_1080p(R):
    # a 2e6-particle slice of the N-body-like set with the per-particle
    # optical depth of the full 1e8 workload (its calibrated brightness)
    ps = synth.nbody_like(2_000_000, seed=1)
    cam = Camera(eye=(0.5, 0.5, -1.5), target=(0.5, 0.5, 0.5), fov_deg=45.0,
                 width=1920, height=1080)
    prm = configs.c2_params(1920)
    ref = oracle.render(ps, cam, CMAP, prm, want_count=True)
    out = gpu_render(R, ps, cam, prm, want_count=True)
    assert_parity(out, ref)
    assert abs(out["stats"]["n_active"] - ref["active"]) <= 10
    assert_parity(gpu_render(R, ps, cam, replace(prm, accum=1)), ref)


def test_dense_stack_parity(R):
    # thousands of particles piled on a few pixels: many terms per pixel,
    # optical depth of order one
    g = np.random.default_rng(11)
    n = 20000
    ps = ParticleSet((0.5 + 0.002 * g.standard_normal(n)).astype(np.float32),
                     (0.5 + 0.002 * g.standard_normal(n)).astype(np.float32),
                     (0.5 + 0.01 * g.standard_normal(n)).astype(np.float32),
                     np.full(n, 0.003, np.float32), np.ones(n, np.float32),
                     g.uniform(0, 1, n).astype(np.float32), np.zeros(n, np.uint8))
    cam = Camera(width=256, height=256)
    prm = Params(brightness=(1e-3,) * 4)
    ref = oracle.render(ps, cam, CMAP, prm)
    assert ref["L"].max() > 1.0
    assert_parity(gpu_render(R, ps, cam, prm), ref)
    assert_parity(gpu_render(R, ps, cam, replace(prm, accum=1)), ref)


# ---------------------------------------------------------------------------
# Workspace chunking, errors, overflow.
# ---------------------------------------------------------------------------
def test_small_workspace_gives_same_image(R):
    ps = synth.uniform_cube(300_000, seed=6)
    cam = Camera(width=256, height=256)
    prm = Params(brightness=(0.01,) * 4, accum=1)
    full = gpu_render(R, ps, cam, prm)
    need = R.workspace_size(splotch.particles_struct(splotch.to_device(ps)), cam, prm)
    small = gpu_render(R, ps, cam, prm, ws_bytes=need // 3)
    assert small["stats"]["passes"] > 1
    assert np.array_equal(full["I"].view(np.uint32), small["I"].view(np.uint32))


def test_error_paths_leave_outputs_untouched(R):
    import torch
    ps = synth.uniform_cube(100, seed=1)
    parts = splotch.to_device(ps)
    cm = torch.from_numpy(CMAP).cuda()
    good = Camera(width=32, height=32)
    rgb = torch.full((32, 32, 3), 7.0, device="cuda:0")
    bad_cases = [
        (replace(good, fov_deg=180.0), Params(), splotch.ERR_INVALID_ARG),
        (replace(good, fov_deg=0.0), Params(), splotch.ERR_INVALID_ARG),
        (replace(good, z_near=0.0), Params(), splotch.ERR_INVALID_ARG),
        (replace(good, target=good.eye), Params(), splotch.ERR_INVALID_ARG),
        (replace(good, up=(0.0, 0.0, 1.0), target=(0.5, 0.5, 0.5), eye=(0.5, 0.5, -1.0)),
         Params(), splotch.ERR_INVALID_ARG),
        (good, Params(chi=0.0), splotch.ERR_INVALID_ARG),
        (good, Params(accum=1, frac_bits=60), splotch.ERR_INVALID_ARG),
        (good, Params(accum=2), splotch.ERR_INVALID_ARG),
        (good, Params(tile=12), splotch.ERR_INVALID_ARG),
        (good, Params(max_clip_tiles=65), splotch.ERR_INVALID_ARG),
        (good, Params(scalar_min=1.0, scalar_max=1.0), splotch.ERR_INVALID_ARG),
        (good, Params(colour_mode=2), splotch.ERR_INVALID_ARG),
        # records per work item: 32..8191 (the item's int64 sums cannot overflow)
        (good, Params(chunk=8192), splotch.ERR_INVALID_ARG),
        (good, Params(chunk=31), splotch.ERR_INVALID_ARG),
        # the vector mode needs vx, vy, vz (absent here) and no log10
        (good, Params(colour_mode=1), splotch.ERR_INVALID_ARG),
    ]
    for cam, prm, code in bad_cases:
        with pytest.raises(splotch.SplotchError) as ei:
            R.render(parts, cam, cm, prm, rgb=rgb)
        assert ei.value.status == code, (cam, prm)
    # colormap with one entry, and none in the palette mode
    for bad_cm in (cm[:1], None):
        with pytest.raises(splotch.SplotchError) as ei:
            R.render(parts, good, bad_cm, Params(), rgb=rgb)
        assert ei.value.status == splotch.ERR_INVALID_ARG
    vparts = dict(parts, vx=parts["x"], vy=parts["y"], vz=parts["z"])
    with pytest.raises(splotch.SplotchError) as ei:
        R.render(vparts, good, None, Params(colour_mode=1, scalar_log10=1, scalar_min=0.1),
                 rgb=rgb)
    assert ei.value.status == splotch.ERR_INVALID_ARG
    # workspace below the minimum, and misaligned
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(splotch.SplotchError) as ei:
        R.render(parts, good, cm, Params(), rgb=rgb, workspace=ws, workspace_bytes=1024)
    assert ei.value.status == splotch.ERR_WORKSPACE
    with pytest.raises(splotch.SplotchError) as ei:
        R.render(parts, good, cm, Params(), rgb=rgb, workspace=ws[1:], workspace_bytes=1 << 19)
    assert ei.value.status == splotch.ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((rgb == 7.0).all())


def _stack(n, tau0):
    f = lambda v: np.full(n, v, np.float32)
    # n identical particles at the image centre of the axis camera
    return ParticleSet(f(0.0), f(0.0), f(2.0), f(0.125), f(tau0), f(1.0), None)


@pytest.mark.parametrize("n,tau0", [(150, 1.0), (1, 100.0)])
def test_int64_overflow_is_reported(R, n, tau0):
    # frac_bits 56 leaves L < 128: 150 unit terms overflow the sum, a single
    # term of 100 overflows the quantiser
    cam = Camera(eye=(0.0, 0.0, 0.0), target=(0.0, 0.0, 1.0), fov_deg=90.0, width=64,
                 height=48)
    prm = Params(brightness=(1.0,) * 4, accum=1, frac_bits=56)
    out = gpu_render(R, _stack(n, tau0), cam, prm, check_stats=False)
    assert out["stats"]["overflow"] == 1
    with pytest.raises(splotch.SplotchError) as ei:
        R.stats()
    assert ei.value.status == splotch.ERR_OVERFLOW
    ok = gpu_render(R, _stack(100, 1.0), cam, prm)
    assert ok["stats"]["overflow"] == 0


def _pileup(n, tau0, jitter=0.0, seed=0):
    # n particles whose centres fall in the one pixel (36, 22) of the axis
    # camera: screen position (36.5 + u, 22.5 + v), u, v in [0, jitter), at
    # depth 2 with sigma 0.5 px (f = 32: X = 32 - 16 x, Y = 24 - 16 y); with
    # no jitter every centre is the pixel centre, where the weight is 1
    g = np.random.default_rng(seed)
    d = g.uniform(0, jitter, (2, n)) if jitter else np.zeros((2, n))
    x = (-(4.5 + d[0]) / 16.0).astype(np.float32)
    y = ((1.5 - d[1]) / 16.0).astype(np.float32)
    f = lambda v: np.full(n, v, np.float32)
    scalar = g.uniform(0, 1, n).astype(np.float32) if jitter else f(1.0)
    return ParticleSet(x, y, f(2.0), f(1.0 / 32.0), f(tau0), scalar, None)


AXIS_CAM = Camera(eye=(0.0, 0.0, 0.0), target=(0.0, 0.0, 1.0), fov_deg=90.0, width=64,
                  height=48)


@pytest.mark.parametrize("accum", [0, 1])
def test_pileup_on_one_pixel(R, accum):
    # 1e5 particles in one pixel: every one of them adds to the same few
    # pixels (one LDS word per channel takes every add of a work item)
    ps = _pileup(100_000, 1.0, jitter=0.5, seed=3)
    prm = Params(chi=3.0, brightness=(2e-5,) * 4, accum=accum)
    ref = oracle.render(ps, AXIS_CAM, CMAP, prm)
    assert ref["L"].max() > 0.3
    out = gpu_render(R, ps, AXIS_CAM, prm)
    assert_parity(out, ref)
    assert out["stats"]["n_active"] == ps.n and out["stats"]["overflow"] == 0
    if accum:
        other = gpu_render(R, ps, AXIS_CAM, replace(prm, tile=8, halo=0, chunk=8191))
        assert np.array_equal(out["I"].view(np.uint32), other["I"].view(np.uint32))


def test_int64_item_sums_at_the_chunk_cap(R):
    # terms just below 2^50 (tau 1000 at 40 fractional bits, at the tile
    # splat's limit): 8191 of them fill a work item's LDS word to 0.98 of
    # 2^63 without overflowing it; the image sum of 20000 of them leaves the
    # int64 range, which only the checked addition into the plane can see
    ps = _pileup(20_000, 1000.0)
    prm = Params(chi=3.0, brightness=(1.0, 0, 0, 0), accum=1, frac_bits=40, chunk=8191,
                 tile=16, halo=4)
    out = gpu_render(R, ps, AXIS_CAM, prm, check_stats=False)
    assert out["stats"]["n_large"] == 0          # drawn by the tile splat
    assert out["stats"]["overflow"] == 1
    # 8000 of them: sum 8000 * 1000 * 2^40 < 2^63, exact, no flag
    ok = gpu_render(R, _pileup(8000, 1000.0), AXIS_CAM, replace(prm, chunk=4096),
                    want_L=True, check_stats=False)
    assert ok["stats"]["overflow"] == 0
    assert ok["L"][22, 36, 0] == pytest.approx(8000 * 1000.0 * float(CMAP[255, 0]), rel=1e-6)


@pytest.mark.parametrize("eye_z", [-6.0, -1.5, 0.2])
def test_radius_statistics(R, eye_z):
    """The radius histogram and mean radius R0 of the active particles (the
    zoom-test quantities) against the oracle's projection: r = chi * sigma,
    active = in front of the camera with a footprint box meeting the image."""
    ps = synth.nbody_like(400_000, seed=7)
    cam = Camera(eye=(0.5, 0.5, eye_z), target=(0.5, 0.5, 0.5), fov_deg=45.0,
                 width=512, height=512)
    prm = Params(chi=3.0, brightness=(0.01,) * 4)
    assert sum(gpu_render(R, ps, cam, prm)["stats"]["radius_hist"]) == 0   # off by default
    R.set_radius_stats(True)
    try:
        st = gpu_render(R, ps, cam, prm)["stats"]
    finally:
        R.set_radius_stats(False)
    pr = oracle.project(ps, cam, prm)
    r = prm.chi * pr["sigma"]
    with np.errstate(invalid="ignore"):
        act = ((pr["depth"] > cam.z_near) & (r > 0)
               & (np.ceil(pr["X"] + r - 0.5) >= 0) & (np.floor(pr["X"] - r - 0.5) <= cam.width - 1)
               & (np.ceil(pr["Y"] + r - 0.5) >= 0) & (np.floor(pr["Y"] - r - 0.5) <= cam.height - 1))
    ra = r[act]
    hist = np.histogram(ra, bins=[0, 2, 4, 8, 16, np.inf])[0]
    # FP32 projection against FP64: a few particles may sit on a bin edge
    assert abs(st["n_active"] - act.sum()) <= 3
    assert sum(st["radius_hist"]) == st["n_active"]
    assert np.abs(np.array(st["radius_hist"]) - hist).max() <= 3 + 1e-5 * act.sum()
    assert st["radius_mean"] == pytest.approx(ra.mean(), rel=1e-5)


@pytest.mark.parametrize("pinned", [True, False])
def test_streamed_from_host_equals_device_render(R, pinned):
    """Particles in host memory, copied in chunks while the previous chunk
    renders: int64 image identical to the device render, FP32 within the
    oracle tolerance; ragged last chunk, one chunk, and an empty set."""
    import torch
    ps = synth.nbody_like(300_001, seed=11)
    cam = Camera(eye=(0.5, 0.5, -1.5), target=(0.5, 0.5, 0.5), fov_deg=45.0,
                 width=400, height=300)
    prm = Params(brightness=(0.01,) * 4, fixed_sigma_frac=(0.0, 1.0 / 400, 0.0, 0.0))
    cm = torch.from_numpy(CMAP).cuda()
    host = splotch.to_host(ps, pinned=pinned)
    p64 = replace(prm, accum=1)
    dev = R.render(splotch.to_device(ps), cam, cm, p64)
    for chunk in (70_000, 300_001, 10**9):
        out = R.render_streamed(host, cam, cm, p64, chunk=chunk)
        torch.cuda.synchronize()
        assert torch.equal(out, dev), chunk
        assert R.stats()["n_input"] == ps.n
    ref = oracle.render(ps, cam, CMAP, prm)
    out = R.render_streamed(host, cam, cm, prm, chunk=65_536)
    torch.cuda.synchronize()
    assert np.abs(out.cpu().numpy().astype(np.float64) - ref["I"]).max() <= TOL
    empty = {k: v[:0] for k, v in host.items()}
    out = R.render_streamed(empty, cam, cm, prm, chunk=1000)
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0


# ---------------------------------------------------------------------------
# Screen-plane prefilter: the anti-aliased coarse render the upscaler reads.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def coarse():
    """A clustered set at 256x256 with dark matter at a quarter pixel (a
    scaled-down low-resolution frame of the upscaler), prefilter 0.5 px."""
    ps = synth.nbody_like(1_000_000, seed=12)
    cam = Camera(width=256, height=256)
    # peak depth per particle <= 0.02 (the FP32 error budget of the
    # projection, which grows as 1/sigma for these narrow footprints)
    prm = Params(chi=3.0, brightness=(0.02,) * 4, fixed_sigma_frac=(0.0, 0.25 / 256, 0.0, 0.0),
                 prefilter=0.5)
    return ps, cam, prm, oracle.render(ps, cam, CMAP, prm, want_count=True)


def test_prefilter_parity(R, coarse):
    ps, cam, prm, ref = coarse
    assert ref["I"].max() > 0.3
    out = gpu_render(R, ps, cam, prm, want_L=True, want_count=True)
    assert_parity(out, ref)
    # centre counts: a projected centre within float rounding of a pixel
    # edge (about 1.5e-5 px at 256 px) may land in the neighbouring pixel;
    # at most one particle in 10^4 moves
    assert out["count"].sum() == ref["count"].sum()
    assert np.abs(out["count"] - ref["count"]).sum() <= 2e-4 * ps.n
    assert_parity(gpu_render(R, ps, cam, replace(prm, accum=1)), ref)
    # the filter changes the image: without it the quarter-pixel particles
    # are point-sampled
    plain = oracle.render(ps, cam, CMAP, replace(prm, prefilter=0.0))
    assert np.abs(plain["I"] - ref["I"]).max() > 0.05


@pytest.mark.parametrize("knobs", [dict(tile=8, halo=0, max_clip_tiles=1, chunk=64),
                                   dict(tile=64, halo=4, max_clip_tiles=64, chunk=4096)])
def test_prefilter_int64_bit_exact_across_schedules(R, coarse, knobs):
    ps, cam, prm, ref = coarse
    base = gpu_render(R, ps, cam, replace(prm, accum=1))
    other = gpu_render(R, ps, cam, replace(prm, accum=1, **knobs))
    assert np.array_equal(base["I"].view(np.uint32), other["I"].view(np.uint32)), knobs


def test_prefilter_ordered_parity(R, coarse):
    ps, cam, prm, _ = coarse
    b = prm.brightness[0]
    op = replace(prm, transfer=1, brightness=(b, 0.0, 0.0, 0.0), absorption=(0.5 * b, b, 0.0, 0.0))
    assert_parity(gpu_render(R, ps, cam, op), oracle.render(ps, cam, CMAP, op))


# ---------------------------------------------------------------------------
# Region masks: only the marked regions are drawn and written.
# ---------------------------------------------------------------------------
def masked_render(R, ps, cam, prm, mask, region, fill=7.0):
    import torch
    dev = "cuda:0"
    H, W = cam.height, cam.width
    rgb = torch.full((H, W, 3), fill, dtype=torch.float32, device=dev)
    la = torch.full((H, W, 3), fill, dtype=torch.float32, device=dev)
    m = torch.from_numpy(np.ascontiguousarray(mask, np.uint8)).to(dev)
    R.render(splotch.to_device(ps, dev), cam, torch.from_numpy(CMAP).to(dev), prm, rgb=rgb,
             log_accum=la, region_mask=m, region_size=region)
    torch.cuda.synchronize()
    return rgb.cpu().numpy(), la.cpu().numpy()


def pixel_mask(mask, region, W, H):
    m = np.repeat(np.repeat(np.asarray(mask, bool).reshape(-(-H // region), -(-W // region)),
                            region, 0), region, 1)
    return m[:H, :W]


@pytest.mark.parametrize("region,knobs", [(64, dict()), (16, dict(tile=32)),
                                          (128, dict(tile=16, halo=4)), (8, dict(tile=64))])
def test_region_mask_draws_only_marked_regions(R, c1, region, knobs):
    """int64: marked pixels equal the unmasked render bit for bit, the
    others keep their previous contents; FP32: marked pixels match the
    oracle."""
    ps, cam, prm, ref = c1
    W, H = cam.width, cam.height
    nreg = (-(-W // region)) * (-(-H // region))
    mask = (np.random.default_rng(region).random(nreg) < 0.35).astype(np.uint8)
    mask[0] = 1
    pm = pixel_mask(mask, region, W, H)
    p64 = replace(prm, accum=1, **knobs)
    full = gpu_render(R, ps, cam, p64, want_L=True)
    rgb, la = masked_render(R, ps, cam, p64, mask, region)
    assert np.array_equal(rgb[pm].view(np.uint32), full["I"][pm].view(np.uint32))
    assert np.array_equal(la[pm].view(np.uint32), full["L"][pm].view(np.uint32))
    assert np.all(rgb[~pm] == 7.0) and np.all(la[~pm] == 7.0)
    rgb32, _ = masked_render(R, ps, cam, replace(prm, **knobs), mask, region)
    err = np.abs(rgb32[pm].astype(np.float64) - ref["I"][pm]).max()
    assert err <= TOL and np.all(rgb32[~pm] == 7.0)


def test_region_mask_large_footprints_and_all_or_none(R):
    """Screen-filling particles (the large pass) under a mask; a mask with
    every region marked is the whole render, one with none writes
    nothing."""
    ps = synth.pareto_cube(30000, seed=5)
    cam = Camera(eye=(0.5, 0.5, 0.5), target=(0.5, 0.5, 1.0), fov_deg=90.0, width=256,
                 height=192)
    prm = Params(chi=3.0, brightness=(0.002,) * 4, accum=1, max_clip_tiles=2)
    full = gpu_render(R, ps, cam, prm)
    assert full["stats"]["n_large"] > 0
    region = 32
    nreg = (256 // 32) * (192 // 32)
    mask = (np.arange(nreg) % 3 == 0).astype(np.uint8)
    pm = pixel_mask(mask, region, 256, 192)
    rgb, _ = masked_render(R, ps, cam, prm, mask, region)
    assert np.array_equal(rgb[pm].view(np.uint32), full["I"][pm].view(np.uint32))
    assert np.all(rgb[~pm] == 7.0)
    rgb, _ = masked_render(R, ps, cam, prm, np.ones(nreg, np.uint8), region)
    assert np.array_equal(rgb.view(np.uint32), full["I"].view(np.uint32))
    rgb, _ = masked_render(R, ps, cam, prm, np.zeros(nreg, np.uint8), region)
    assert np.all(rgb == 7.0)


def test_region_mask_errors(R):
    import torch
    ps = synth.uniform_cube(1000, seed=2)
    cam = Camera(width=64, height=64)
    parts = splotch.to_device(ps)
    cm = torch.from_numpy(CMAP).cuda()
    m = torch.ones(4, dtype=torch.uint8, device="cuda")
    rgb = torch.full((64, 64, 3), 7.0, device="cuda")
    cc = torch.zeros((64, 64), dtype=torch.int32, device="cuda")
    for kw, status in ((dict(region_size=48), splotch.ERR_INVALID_ARG),
                       (dict(region_size=32, center_count=cc), splotch.ERR_INVALID_ARG)):
        with pytest.raises(splotch.SplotchError) as e:
            R.render(parts, cam, cm, Params(), rgb=rgb, region_mask=m, **kw)
        assert e.value.status == status
    with pytest.raises(splotch.SplotchError) as e:
        R.render(parts, cam, cm, Params(absorption=(0.01,) * 4, transfer=1), rgb=rgb,
                 region_mask=m, region_size=32)
    assert e.value.status == splotch.ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((rgb == 7.0).all())


# ---------------------------------------------------------------------------
# Colour by vector: the three colour channels from (vx, vy, vz).
# ---------------------------------------------------------------------------
def vector_set(n, seed):
    """N-body-like set with velocity-like components, about a third of
    them outside [-1, 1] so the clamp is exercised; no scalar."""
    ps = synth.nbody_like(n, seed=seed)
    v = np.random.default_rng(seed).normal(0.0, 0.8, size=(3, n)).astype(np.float32)
    ps.vx, ps.vy, ps.vz = v[0], v[1], v[2]
    ps.scalar = None
    return ps


# per-particle tau0 <= 0.05: a float32 screen position carries ~1e-5 px of
# rounding, which moves a 1-px Gaussian's terms by ~2e-5 of tau0 (the FP32
# error budget); density, not brightness, gives the optical depth
VEC_CAM = Camera(eye=(0.5, 0.5, -1.5), target=(0.5, 0.5, 0.5), fov_deg=45.0,
                 width=161, height=121)
VEC_PRM = Params(chi=3.0, brightness=(0.05,) * 4, fixed_sigma_frac=(0.0, 1.0 / 161, 0.0, 0.0),
                 scalar_min=-1.0, scalar_max=1.0, colour_mode=1)


def test_vector_colour_parity_and_schedules(R):
    ps = vector_set(300_001, seed=21)
    ref = oracle.render(ps, VEC_CAM, None, VEC_PRM)
    assert 0.2 < float(np.median(ref["L"][..., 1])) < 5.0
    gpu = gpu_render(R, ps, VEC_CAM, VEC_PRM, cmap=None, want_L=True)
    assert_parity(gpu, ref)
    assert gpu["stats"]["n_input"] == ps.n
    runs = []
    for knobs in (dict(tile=16, halo=0, max_clip_tiles=1), dict(tile=64, halo=4, max_clip_tiles=16)):
        out = gpu_render(R, ps, VEC_CAM, replace(VEC_PRM, accum=1, **knobs), cmap=None)
        assert_parity(out, ref)
        runs.append(out["I"])
    assert np.array_equal(runs[0], runs[1])
    # a palette passed in this mode is not read
    out = gpu_render(R, ps, VEC_CAM, replace(VEC_PRM, accum=1, tile=16, halo=0,
                                             max_clip_tiles=1), cmap=CMAP)
    assert np.array_equal(out["I"], runs[0])


def test_vector_colour_streamed_equals_device(R):
    import torch
    ps = vector_set(50_003, seed=22)
    prm = replace(VEC_PRM, accum=1)
    dev = R.render(splotch.to_device(ps), VEC_CAM, None, prm)
    host = splotch.to_host(ps, pinned=True)
    assert "scalar" not in host and "vx" in host
    for chunk in (12_345, 10**9):
        out = R.render_streamed(host, VEC_CAM, None, prm, chunk=chunk)
        torch.cuda.synchronize()
        assert torch.equal(out, dev), chunk


def test_palette_sizes(R, c1):
    # a two-entry palette and one of 2000 entries (the scatter pass reads
    # palettes of more than 1024 entries from global memory, smaller ones
    # from LDS): parity with the oracle either way
    ps, cam, prm, _ = c1
    t = np.linspace(0.0, 1.0, 2000, dtype=np.float64)
    big = np.stack([0.5 + 0.5 * np.sin(7 * t), t, 1.0 - t ** 2], axis=1).astype(np.float32)
    two = np.array([[0.1, 0.9, 0.3], [0.8, 0.2, 0.6]], np.float32)
    for cmap in (two, big):
        ref = oracle.render(ps, cam, cmap, prm)
        gpu = gpu_render(R, ps, cam, prm, cmap=cmap)
        assert_parity(gpu, ref)


def test_exact_sample_count(R, c1):
    """The samples the kernels draw (Eq. 6's beta R0^2 term) against the
    oracle's exact count; FP32 and FP64 may take a centre within rounding of
    a rim on different sides, a few in a million.  The count is the same for
    every schedule (every kernel takes the same decision per sample)."""
    ps, cam, prm, ref = c1
    assert gpu_render(R, ps, cam, prm)["stats"]["n_samples"] == -1    # off by default
    R.set_sample_count(True)
    try:
        a = gpu_render(R, ps, cam, prm)["stats"]["n_samples"]
        b = gpu_render(R, ps, cam, replace(prm, tile=8, halo=0, max_clip_tiles=1,
                                            accum=1))["stats"]["n_samples"]
        c = gpu_render(R, ps, cam, replace(prm, tile=64, halo=4, max_clip_tiles=64,
                                            chunk=256))["stats"]["n_samples"]
    finally:
        R.set_sample_count(False)
    assert a == b == c
    assert abs(a - ref["samples"]) <= 1e-5 * ref["samples"] + 10, (a, ref["samples"])
    # a slice of the clustered 1e8 workload at 1080p, and the large pass
    for ps2, cam2, prm2 in (
            (synth.nbody_like(1_000_000, seed=1),
             Camera(eye=(0.5, 0.5, -1.5), target=(0.5, 0.5, 0.5), fov_deg=45.0,
                    width=1920, height=1080), configs.c2_params(1920)),
            (synth.pareto_cube(50_000, seed=2),
             Camera(eye=(0.5, 0.5, 0.5), target=(0.5, 0.5, 1.0), fov_deg=90.0,
                    width=400, height=400), Params(brightness=(0.001,) * 4))):
        ref2 = oracle.render(ps2, cam2, CMAP, prm2, want_image=False)
        R.set_sample_count(True)
        try:
            st = gpu_render(R, ps2, cam2, prm2)["stats"]
        finally:
            R.set_sample_count(False)
        assert abs(st["n_samples"] - ref2["samples"]) <= 1e-5 * ref2["samples"] + 10, \
            (st["n_samples"], ref2["samples"])
