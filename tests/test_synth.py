"""Seeded generators: determinism and the shape of the distributions."""
import numpy as np

from paper_1309_1114_amd import synth


def test_uniform_cube_deterministic():
    a = synth.uniform_cube(5000, seed=0)
    b = synth.uniform_cube(5000, seed=0)
    for k, v in a.arrays().items():
        assert np.array_equal(v, b.arrays()[k]), k
    assert a.x.dtype == np.float32 and a.species.dtype == np.uint8
    assert 0 <= a.x.min() and a.x.max() < 1
    assert abs(np.median(a.h) - 0.005) < 2e-4
    assert abs(np.std(np.log(a.h)) - 0.5) < 0.02


def test_nbody_like_shape():
    ps = synth.nbody_like(200_000, seed=1)
    again = synth.nbody_like(200_000, seed=1)
    assert np.array_equal(ps.x, again.x) and np.array_equal(ps.h, again.h)
    assert ps.n == 200_000
    assert 0 <= ps.x.min() and ps.x.max() < 1
    assert 1e-4 <= ps.h.min() and ps.h.max() <= 0.05
    assert 0 <= ps.scalar.min() and ps.scalar.max() <= 1
    assert abs(ps.species.mean() - 0.5) < 0.01
    # clustering: the densest cells hold far more than the mean
    cell = np.minimum((np.stack([ps.x, ps.y, ps.z]) * 32).astype(int), 31)
    cnt = np.bincount((cell[0] * 32 + cell[1]) * 32 + cell[2], minlength=32 ** 3)
    assert cnt.max() > 20 * cnt.mean()


def test_pareto_cube_tail():
    ps = synth.pareto_cube(100_000, seed=2)
    assert ps.h.min() >= 0.001 and ps.h.max() <= 0.3
    # P(h > 0.01) = 10^-1.5 for a Pareto(1.5) tail starting at 0.001
    assert abs((ps.h > 0.01).mean() - 10 ** -1.5) < 0.004


def test_batch_shapes_and_cameras():
    shapes = synth.batch_shapes()
    assert len(shapes) == 16
    for s, n, side in shapes:
        assert 1e5 * 0.999 <= n <= 5e7 * 1.001 and side % 8 == 0 and 248 <= side <= 2056
    cams = synth.orbit_cameras(64)
    assert len(cams) == 64
    c = synth.random_camera(10000, 512, 512)
    d = np.linalg.norm(np.array(c.eye) - 0.5)
    assert 1.2 <= d <= 2.5 and 30 <= c.fov_deg <= 60


def test_colormap_ramp():
    cm = synth.ramp_colormap()
    assert cm.shape == (256, 3)
    np.testing.assert_allclose(cm[0], [0.1, 0.2, 1.0], rtol=1e-6)
    np.testing.assert_allclose(cm[255], [1.0, 0.6, 0.1], rtol=1e-6)
