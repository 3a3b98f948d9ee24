"""CPU checks of the lattice scenes used by the chi = 1 rim parity tests:
the oracle projects every particle exactly onto its quarter-pixel lattice
position, and no pixel centre lies within 1/8 px^2 of any disk rim, so the
in-disk decision of every (particle, pixel) pair is free of rounding."""
import numpy as np
import pytest

from oracle import oracle
from paper_1309_1114_amd.synth import Params
from scenes import lattice_camera, lattice_scene


@pytest.mark.parametrize("W,H,n,seed,fracs", [
    (256, 192, 100_001, 36, (2.5, 1.5, 6.0)),
    (64, 48, 60_001, 35, (1.5, 2.5)),
])
def test_lattice_positions_and_rim_margin(W, H, n, seed, fracs):
    ps, X, Y = lattice_scene(n, W, H, seed=seed, n_species=len(fracs))
    cam = lattice_camera(W, H)
    prm = Params(chi=1.0, fixed_sigma_frac=tuple(f / W for f in fracs) + (0.0,) * (4 - len(fracs)))
    pr = oracle.project(ps, cam, prm)
    assert np.abs(pr["X"] - X).max() < 1e-9 and np.abs(pr["Y"] - Y).max() < 1e-9
    assert np.array_equal(np.sort(np.unique(pr["sigma"])), np.sort(np.array(fracs)))
    # every pixel centre within R + 1 of every particle
    r = int(np.ceil(max(fracs))) + 1
    off = np.arange(-r, r + 1)
    cx = np.floor(X)[:, None, None] + off[None, :, None] + 0.5
    cy = np.floor(Y)[:, None, None] + off[None, None, :] + 0.5
    d2 = (cx - X[:, None, None]) ** 2 + (cy - Y[:, None, None]) ** 2
    R2 = (pr["sigma"] ** 2)[:, None, None]
    assert np.abs(d2 - R2).min() >= 0.125 - 1e-9
