"""Benchmark of the plain render path on one MI355X.

A step is one complete render (transform, binning, large-footprint pass,
tile splat, resolve) of the whole particle set, with the particles already
resident in HBM.  Default workload: 1e8 N-body-like particles at 1920x1080
(FP32 accumulation).  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload c2|c2_4k|c1|c3]
                    [--n N] [--accum fp32|int64] [--cpu-seconds S] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mparticles/s & frames/s (1e8 particles, 1080p); learned vs plain at PSNR>=40dB"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# operations of one (particle, pixel) sample: two offsets (2 adds, 2 subs),
# dy*dy, one fma (2), the exponent scale (1 mul), exp2 (1), three colour
# products and three accumulations
FLOPS_PER_SAMPLE = 14
# bytes the transform must read per particle: x, y, z, h, intensity, scalar
# (float32) and species (uint8)
BYTES_PER_PARTICLE = 25
COUNT_BYTES_PER_PARTICLE = 17   # x, y, z, h, species (the key needs no colour)
RECORD_BYTES = 32


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name, n):
    from paper_1309_1114_amd import configs, synth
    if name == "c1":
        ps, cam, prm = configs.c1()
        desc = "C1 uniform cube 131072 particles 512x512 plain render"
    elif name in ("c2", "c2_4k"):
        W, H = (1920, 1080) if name == "c2" else (4096, 4096)
        ps, cam, prm = configs.c2(n=n or 100_000_000, width=W, height=H)
        desc = f"C2 N-body-like {ps.n:.0e} particles {W}x{H} plain render"
    elif name == "c3":
        ps, cam, prm = configs.c3(n=n or 10_000_000)
        desc = f"C3 large-footprint stress {ps.n:.0e} particles 2048x2048 plain render"
    else:
        raise SystemExit(f"unknown workload {name}")
    return ps, cam, prm, desc


def cpu_baseline(ps, cam, prm, cmap, seconds):
    """The FP64 oracle on the host cores, on a leading sample of the
    (randomly ordered) particle set sized to take about `seconds`."""
    from oracle import oracle
    n = ps.n
    probe = min(n, 200_000)
    t0 = time.perf_counter()
    r = oracle.render(ps.subset(slice(0, probe)), cam, cmap, prm, want_image=False)
    dt = time.perf_counter() - t0
    ns = min(n, max(probe, int(probe * seconds / max(dt, 1e-3))))
    if ns > probe:
        t0 = time.perf_counter()
        r = oracle.render(ps.subset(slice(0, ns)), cam, cmap, prm, want_image=False)
        dt = time.perf_counter() - t0
    return dict(value=ns / dt / 1e6, unit="Mparticles/s", cores=r["threads"], kind="oracle",
                sample=f"first {ns} of {n} particles (random order), same camera and image",
                seconds=round(dt, 3), samples_in_sample=r["samples"], n_sample=ns)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--accum", default="fp32", choices=["fp32", "int64"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this renderer is measured per GPU "
              "(multi-GPU sharding is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from dataclasses import replace
    from paper_1309_1114_amd import splotch, synth

    t0 = time.perf_counter()
    ps, cam, prm, desc = workload(args.workload, args.n)
    if args.accum == "int64":
        prm = replace(prm, accum=1)
    cmap = synth.ramp_colormap()
    log(f"generated {desc} in {time.perf_counter() - t0:.1f} s")

    dev = "cuda:0"
    parts = splotch.to_device(ps, dev)
    cm = torch.from_numpy(cmap).to(dev)
    R = splotch.Renderer(0)
    rgb = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device=dev)
    ws_bytes = R.workspace_size(splotch.particles_struct(parts), cam, prm)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    log(f"device inputs {sum(v.numel() * v.element_size() for v in parts.values() if v is not None) / 1e9:.2f} GB, "
        f"workspace {ws_bytes / 1e9:.2f} GB")

    def step():
        R.render(parts, cam, cm, prm, rgb=rgb, workspace=ws, workspace_bytes=ws_bytes)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")

    # timed region: exactly `steps` renders
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    log(f"timed {args.steps} renders: {ms:.3f} ms/render")
    st = R.stats()

    # per-stage GPU times (HIP events on the render stream, separate loop)
    R.set_timing(True)
    for _ in range(args.steps):
        step()
    stage_ms, nt = R.stage_times()
    R.set_timing(False)
    stage_ms = {k: v / max(nt, 1) for k, v in stage_ms.items()}
    log("stage ms: " + ", ".join(f"{k} {v:.3f}" for k, v in stage_ms.items()))

    base = None
    if not args.no_cpu:
        base = cpu_baseline(ps, cam, prm, cmap, args.cpu_seconds)
        log(f"cpu baseline: {base['value']:.2f} Mparticles/s on {base['cores']} threads")

    n = ps.n
    # samples of the whole frame, scaled from the oracle's exact count on its sample
    samples = None
    if base:
        samples = base["samples_in_sample"] * n / base["n_sample"]

    kern = {}
    kern["k_count"] = dict(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS,
                           work=n * COUNT_BYTES_PER_PARTICLE / 1e9, ms=stage_ms["count"])
    kern["k_scatter"] = dict(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS,
                             work=(n * BYTES_PER_PARTICLE + st["n_entries"] * RECORD_BYTES) / 1e9,
                             ms=stage_ms["scatter"])
    if samples is not None:
        kern["k_splat"] = dict(bound="alu", unit="TFLOP/s", peak=FP32_PEAK_TFLOPS,
                               work=samples * FLOPS_PER_SAMPLE / 1e12,
                               ms=stage_ms["splat"] + stage_ms["large"])
    dom_name = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom_name]
    achieved = d["work"] / (d["ms"] / 1e3)
    roofline = dict(kernel=dom_name, bound=d["bound"], achieved=round(achieved, 3),
                    peak=d["peak"], unit=d["unit"], frac=round(achieved / d["peak"], 5),
                    traffic=None)
    others = {k: dict(bound=v["bound"], achieved=round(v["work"] / (v["ms"] / 1e3), 3),
                      unit=v["unit"], ms=round(v["ms"], 4)) for k, v in kern.items()}

    out = {
        "metric": METRIC,
        "value": round(n / (ms / 1e3) / 1e6, 3),
        "unit": "Mparticles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "frames_per_s": round(1e3 / ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prm.accum == 0 else "int64",
        "data": "synthetic",
        "config": {"workload": desc, "n_particles": n, "width": cam.width,
                   "height": cam.height, "accum": args.accum, "chi": prm.chi,
                   "brightness": prm.brightness[0], "tile": st["tile"], "halo": st["halo"],
                   "max_clip_tiles": st["max_clip_tiles"], "chunk": st["chunk"]},
        "roofline": roofline,
        "kernels": others,
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "counts": {"active": st["n_active"], "entries": st["n_entries"],
                   "large": st["n_large"], "items": st["n_items"],
                   "samples_est": None if samples is None else int(samples)},
        "cpu_baseline": None if base is None else {k: base[k] for k in
                                                  ("value", "unit", "cores", "kind", "sample")},
    }
    print(json.dumps(out), flush=True)
    R.close()


if __name__ == "__main__":
    main()
