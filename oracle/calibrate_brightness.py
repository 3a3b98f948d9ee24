"""Brightness calibration of the C2 and C3 workloads with the FP64 oracle.

TEST INFRASTRUCTURE ONLY (run once by hand; the result is written into
``paper_1309_1114_amd/configs.py`` as a constant).

The optical depth is linear in the brightness b, so rendering once with
b = 1 and taking b = 0.7 / median(L_G) makes the median green optical depth
of the plain render exactly 0.7.

    python oracle/calibrate_brightness.py c2     # 1e8 particles, 1920x1080
    python oracle/calibrate_brightness.py c3     # 1e7 particles, 2048x2048
    python oracle/calibrate_brightness.py c5     # 2e7 particles, 2048x2048
"""
from __future__ import annotations

import sys
import time
from dataclasses import replace
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))

from oracle import oracle  # noqa: E402
from paper_1309_1114_amd import configs, synth  # noqa: E402


def calibrate(which: str) -> float:
    t0 = time.time()
    if which == "c2":
        ps = synth.nbody_like(100_000_000, seed=1)
        cam = synth.Camera(eye=(0.5, 0.5, -1.5), target=(0.5, 0.5, 0.5), fov_deg=45.0,
                           width=1920, height=1080)
        prm = configs.c2_params(1920, brightness=1.0)
    elif which == "c3":
        ps = synth.pareto_cube(10_000_000, seed=2)
        cam = synth.Camera(eye=(0.5, 0.5, 0.5), target=(0.5, 0.5, 1.0), fov_deg=90.0,
                           width=2048, height=2048)
        prm = synth.Params(chi=3.0, brightness=(1.0,) * 4)
    elif which == "c5":
        # the upscaler's full-resolution frames: a 2e7-particle C2-style set
        # (validation seed 30000) through the C2 camera at 2048x2048
        ps = synth.nbody_like(20_000_000, seed=30000)
        cam = synth.Camera(eye=(0.5, 0.5, -1.5), target=(0.5, 0.5, 0.5), fov_deg=45.0,
                           width=2048, height=2048)
        prm = configs.c2_params(2048, brightness=1.0)
    else:
        raise SystemExit(f"unknown workload {which}")
    print(f"{which}: generated in {time.time() - t0:.1f} s", flush=True)
    t1 = time.time()
    out = oracle.render(ps, cam, synth.ramp_colormap(), replace(prm), want_image=False)
    med = float(np.median(out["L"][..., 1]))
    b = 0.7 / med
    print(f"{which}: oracle {time.time() - t1:.1f} s, samples {out['samples']}, "
          f"active {out['active']}, median L_G at b=1: {med!r}, brightness {b!r}", flush=True)
    return b


if __name__ == "__main__":
    for w in sys.argv[1:] or ["c2", "c3"]:
        calibrate(w)
