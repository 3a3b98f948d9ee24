"""Batched render (one launch sequence, graph-captured and replayed) and the
autotuner, through the C ABI.

Each job of a batch must give the image splotch_render gives for it (int64
mode: bit for bit) and match the FP64 oracle within 1e-5 (FP32 mode).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle
from paper_1309_1114_amd import splotch, synth
from paper_1309_1114_amd.synth import Camera, Params

pytestmark = pytest.mark.gpu
CMAP = synth.ramp_colormap()


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    r = splotch.Renderer(0)
    yield r
    r.close()


def uneven_jobs(seed=0, accum=0):
    """Particle sets of uneven sizes at uneven resolutions (config 4b in
    miniature: sizes log-uniform in [1e3, 3e5], sides in [48, 640])."""
    g = np.random.default_rng(seed)
    jobs = []
    for j in range(6):
        n = int(np.exp(g.uniform(np.log(1e3), np.log(3e5))))
        side = int(8 * round(np.exp(g.uniform(np.log(48), np.log(640))) / 8))
        ps = synth.nbody_like(n, seed=500 + j) if j % 2 else synth.uniform_cube(n, seed=500 + j)
        cam = Camera(width=side, height=max(8, side * 3 // 4), fov_deg=float(g.uniform(30, 60)))
        prm = Params(brightness=(float(3e2 / n),) * 4, accum=accum,
                     fixed_sigma_frac=(0.0, 1.0 / side, 0.0, 0.0))
        jobs.append((ps, cam, prm))
    return jobs


def device_specs(jobs):
    import torch
    cm = torch.from_numpy(CMAP).cuda()
    specs = []
    for ps, cam, prm in jobs:
        specs.append(dict(parts=splotch.to_device(ps), cam=cam, cmap=cm, prm=prm,
                          rgb=torch.full((cam.height, cam.width, 3), 7.0, device="cuda:0")))
    return specs


def single(R, spec):
    import torch
    out = torch.empty_like(spec["rgb"])
    R.render(spec["parts"], spec["cam"], spec["cmap"], spec["prm"], rgb=out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_batch_equals_single_int64(R):
    import torch
    specs = device_specs(uneven_jobs(seed=1, accum=1))
    jobs = R.make_jobs(specs)
    R.render_batched(jobs)
    torch.cuda.synchronize()
    st = R.stats()
    assert st["n_input"] == sum(s["parts"]["x"].numel() for s in specs)
    for s in specs:
        assert np.array_equal(s["rgb"].cpu().numpy().view(np.uint32), single(R, s).view(np.uint32))


def test_batch_fp32_matches_oracle(R):
    import torch
    jobs = uneven_jobs(seed=2, accum=0)
    specs = device_specs(jobs)
    R.render_batched(R.make_jobs(specs))
    torch.cuda.synchronize()
    for (ps, cam, prm), s in zip(jobs, specs):
        ref = oracle.render(ps, cam, CMAP, prm)
        err = np.abs(s["rgb"].cpu().numpy().astype(np.float64) - ref["I"]).max()
        assert err <= 1e-5, (cam.width, ps.n, err)


def test_graph_replays_match_eager(R):
    # the same batch shape replayed with new cameras and particle data, with
    # eager work and synchronisations between the replays
    import torch
    base = uneven_jobs(seed=3, accum=1)
    specs = device_specs(base)
    ws_bytes = R.batch_workspace_size(R.make_jobs(specs))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda:0")
    for rep in range(4):
        for k, s in enumerate(specs):
            s["cam"] = replace(s["cam"], eye=(0.5 + 0.1 * rep, 0.5, -1.5 + 0.05 * k))
            s["parts"]["z"].add_(0.01)          # eager work on the same buffers
        torch.cuda.synchronize()
        R.render_batched(R.make_jobs(specs), workspace=ws, workspace_bytes=ws_bytes)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda:0").sum().item()
        for s in specs:
            got = s["rgb"].cpu().numpy()
            assert np.array_equal(got.view(np.uint32), single(R, s).view(np.uint32)), rep


def test_orbit_views_batch(R):
    # config 4a in miniature: 8 orbit views of one particle set
    import torch
    ps = synth.nbody_like(100_000, seed=3)
    cams = synth.orbit_cameras(8, width=160, height=160)
    prm = Params(brightness=(0.01,) * 4, accum=1, fixed_sigma_frac=(0.0, 1.0 / 160, 0.0, 0.0))
    parts = splotch.to_device(ps)
    cm = torch.from_numpy(CMAP).cuda()
    specs = [dict(parts=parts, cam=c, cmap=cm, prm=prm,
                  rgb=torch.empty((160, 160, 3), device="cuda:0")) for c in cams]
    R.render_batched(R.make_jobs(specs))
    torch.cuda.synchronize()
    for s in specs:
        assert np.array_equal(s["rgb"].cpu().numpy().view(np.uint32), single(R, s).view(np.uint32))
    ref = oracle.render(ps, cams[3], CMAP, replace(prm, accum=0))
    assert np.abs(specs[3]["rgb"].cpu().numpy() - ref["I"]).max() <= 1e-5


def test_batch_errors(R):
    import torch
    specs = device_specs(uneven_jobs(seed=4))
    specs[2]["prm"] = replace(specs[2]["prm"], accum=1)
    with pytest.raises(splotch.SplotchError) as ei:
        R.render_batched(R.make_jobs(specs))
    assert ei.value.status == splotch.ERR_INVALID_ARG
    specs[2]["prm"] = replace(specs[2]["prm"], accum=0)
    jobs = R.make_jobs(specs)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    for s in specs:
        s["rgb"].fill_(7.0)
    with pytest.raises(splotch.SplotchError) as ei:     # below any job's minimum
        R.render_batched(jobs, workspace=ws, workspace_bytes=1 << 20)
    assert ei.value.status == splotch.ERR_WORKSPACE
    torch.cuda.synchronize()
    assert all(bool((s["rgb"] == 7.0).all()) for s in specs)


@pytest.mark.parametrize("mode", ["quarter", "half_largest_job"])
def test_batch_in_groups_equals_whole_batch(R, mode):
    """A quarter of the batch's workspace draws it in groups of jobs; half
    of the largest job's own need leaves that job to be drawn in particle
    chunks.  Both give the whole batch's int64 images bit for bit and the
    same counters."""
    import torch
    specs = device_specs(uneven_jobs(seed=5, accum=1))
    jobs = R.make_jobs(specs)
    need = R.batch_workspace_size(jobs)
    largest = max(R.workspace_size(splotch.particles_struct(s["parts"]), s["cam"], s["prm"])
                  for s in specs)
    frac = 0.25 if mode == "quarter" else max(largest // 2, 48 << 20) / need
    R.render_batched(jobs)
    torch.cuda.synchronize()
    whole = [s["rgb"].cpu().numpy().copy() for s in specs]
    st_whole = R.stats()
    for s in specs:
        s["rgb"].fill_(7.0)
    small = (int(need * frac) + 255) // 256 * 256
    ws = torch.empty(small, dtype=torch.uint8, device="cuda:0")
    R.render_batched(R.make_jobs(specs), workspace=ws, workspace_bytes=small)
    torch.cuda.synchronize()
    st = R.stats()
    for s, w in zip(specs, whole):
        assert np.array_equal(s["rgb"].cpu().numpy().view(np.uint32), w.view(np.uint32))
    assert st["passes"] > 1
    for k in ("n_input", "n_active"):
        assert st[k] == st_whole[k], k


def test_autotune_is_result_neutral(R, tmp_path):
    import torch
    ps = synth.uniform_cube(131072, seed=0)
    cam = Camera(width=512, height=512)
    prm = Params(brightness=(0.02,) * 4, accum=1)
    parts = splotch.to_device(ps)
    cm = torch.from_numpy(CMAP).cuda()
    rgb = torch.empty((512, 512, 3), device="cuda:0")
    default = R.render(parts, cam, cm, prm, rgb=torch.empty_like(rgb)).cpu().numpy()
    best, ms = R.autotune(parts, cam, cm, prm, rgb)
    assert best.tile in (16, 32, 64) and ms > 0
    tuned = R.render(parts, cam, cm, prm, rgb=torch.empty_like(rgb))   # knobs from the cache
    torch.cuda.synchronize()
    st = R.stats()
    assert (st["tile"], st["halo"], st["max_clip_tiles"], st["chunk"]) == \
        (best.tile, best.halo, best.max_clip_tiles, best.chunk)
    assert np.array_equal(default.view(np.uint32), tuned.cpu().numpy().view(np.uint32))
    path = tmp_path / "tune.json"
    R.tune_save(path)
    R2 = splotch.Renderer(0)
    try:
        R2.tune_load(path)
        R2.render(parts, cam, cm, prm, rgb=torch.empty_like(rgb))
        torch.cuda.synchronize()
        assert R2.stats()["tile"] == best.tile
    finally:
        R2.close()


def test_radius_stats_toggle_between_replays(R):
    # the radius statistics choose a variant of the counting kernel on the
    # host, so a captured batch must not be replayed across a toggle
    import torch
    specs = device_specs(uneven_jobs(seed=3))
    jobs = R.make_jobs(specs)
    need = R.batch_workspace_size(jobs)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    sums = []
    for on in (False, True, True, False):
        R.set_radius_stats(on)
        try:
            R.render_batched(jobs, workspace=ws, workspace_bytes=need)
            torch.cuda.synchronize()
            st = R.stats()
        finally:
            R.set_radius_stats(False)
        sums.append((sum(st["radius_hist"]), st["n_active"]))
    assert sums[0][0] == 0 and sums[3][0] == 0
    assert sums[1][0] == sums[1][1] > 0 and sums[2] == sums[1]
