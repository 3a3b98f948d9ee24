"""Seeded test scenes whose disk rims stay clear of every pixel centre.

Particles sit at quarter-pixel offsets (k + 1/4 or k + 3/4) of a camera at
the origin looking down +z with a 90-degree field, so the perspective
projection X = W/2 - f x / z, Y = H/2 - f y / z (f = W/2) is exact in FP32
for depths with few mantissa bits.  Every pixel-centre offset is then
n +- 1/4 per axis, d^2 = 1/8 (mod 1/2), and radii with R^2 = 1/4 (mod 1/2)
(fixed sigmas of 1.5, 2.5 or 6 pixels at chi = 1) keep |d^2 - R^2| >= 1/8:
the in-disk decision cannot depend on rounding, so a sample on a rim, which
weighs e^-chi^2 of the peak, must agree exactly.
"""
import numpy as np

from paper_1309_1114_amd.synth import Camera, ParticleSet

DEPTHS = (1.0, 1.25, 1.5, 1.75, 2.0, 2.5, 3.0, 3.5, 4.0)


def lattice_camera(width, height):
    return Camera(eye=(0.0, 0.0, 0.0), target=(0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0),
                  fov_deg=90.0, width=width, height=height)


def lattice_scene(n, width, height, seed, n_species=3, margin=8):
    """n particles at quarter-pixel screen offsets over the image and a
    margin of `margin` pixels around it; returns (particles, X, Y) with the
    exact screen positions."""
    rng = np.random.default_rng(seed)
    X = rng.integers(-margin, width + margin, n) + rng.choice([0.25, 0.75], n)
    Y = rng.integers(-margin, height + margin, n) + rng.choice([0.25, 0.75], n)
    z = rng.choice(DEPTHS, n)
    f = width / 2.0
    x = ((width / 2.0 - X) * z / f).astype(np.float32)
    y = ((height / 2.0 - Y) * z / f).astype(np.float32)
    assert np.array_equal(x.astype(np.float64), (width / 2.0 - X) * z / f)
    assert np.array_equal(y.astype(np.float64), (height / 2.0 - Y) * z / f)
    f32 = lambda a: np.asarray(a, np.float32)
    ps = ParticleSet(x, y, f32(z), f32(np.full(n, 0.01)), f32(rng.uniform(0.2, 1.0, n)),
                     f32(rng.uniform(0.0, 1.0, n)),
                     rng.integers(0, n_species, n).astype(np.uint8))
    return ps, X, Y
