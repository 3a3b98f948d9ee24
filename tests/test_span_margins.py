"""CPU checks of two conservative bounds the render kernels rely on.

The kernels decide every sample by the in-disk test d^2 <= R^2 in float32
(d^2 = fma(dx, dx, dy * dy), dx = i + 1/2 - X; Eq. 2's clip at chi sigma).
Two cheaper bounds run before that test and must never drop a pixel it
would pass:

* the pixel span of a footprint along one axis (the splat's and the large
  pass's loops, the ordered render's tile binning): ceil(X - R - 1/2 - m) ..
  floor(X + R - 1/2 + m) with R = sqrt(R^2) and a margin
  m = 1e-6 (|X| + R) + 1e-3;
* the ordered composite's quadrant cull: a record is walked by the wave of
  an 8 x 8 quadrant only if the nearest point of the quadrant's box of
  pixel centres lies within fma(R^2, 1.0001, 1e-4) of its centre.

Both are re-evaluated here in float32 with numpy (each operation rounded
once, as on the GPU) and checked by brute force against the per-pixel test
on random and adversarial footprints: centres on and next to pixel centres,
radii that put a pixel centre exactly on the rim, large coordinates.
"""
import numpy as np
import pytest

f32 = np.float32


def fmaf(a, b, c):
    # a*b is exact in float64 for float32 operands; one more rounding to
    # float32 after the float64 add (a double rounding can differ from a
    # fused result only on an exact float32 halfway point, which these
    # inputs do not hit by construction of the checks below: they test
    # inequalities with margins far above one ulp)
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(f32)


def in_disk_1d(X, R2, i):
    """The kernels' in-disk test for pixel column i on the centre's row."""
    dx = (i.astype(f32) + f32(0.5)) - X
    d2 = fmaf(dx, dx, f32(0.0) * f32(0.0))
    return d2 <= R2


def span(X, R2):
    R = np.sqrt(R2)                       # correctly rounded, as sqrtf
    m = fmaf(f32(1.0e-6), np.abs(X) + R, f32(1.0e-3))
    f0 = np.ceil(((X - R) - f32(0.5)) - m)
    f1 = np.floor(((X + R) - f32(0.5)) + m)
    return f0, f1


def footprints(rng, n):
    """Footprint centres X and squared radii R2 (float32), mixed so that
    pixel centres fall on, just inside and just outside the rim."""
    X = np.concatenate([
        rng.uniform(-50, 2100, n),                                   # ordinary
        rng.integers(-10, 4096, n) + 0.5,                            # on a pixel centre
        rng.integers(-10, 4096, n).astype(np.float64),               # on a pixel edge
        rng.uniform(-1e5, 1e5, n),                                   # far off-screen
    ]).astype(f32)
    X = np.concatenate([X, np.nextafter(X, f32(np.inf)), np.nextafter(X, f32(-np.inf))])
    k = X.size
    R = np.exp(rng.uniform(np.log(1e-3), np.log(600.0), k)).astype(f32)
    R2 = (R.astype(np.float64) ** 2).astype(f32)
    # a third of the radii put a pixel centre exactly on the rim: R2 = dx^2
    # (as the test computes it) for a pixel a few columns from the centre
    sel = rng.random(k) < 1 / 3
    j = np.floor(X[sel].astype(np.float64)) + rng.integers(-40, 41, sel.sum())
    dx = (j.astype(f32) + f32(0.5)) - X[sel]
    R2[sel] = fmaf(dx, dx, f32(0.0))
    # and some one ulp either side of that
    R2[sel] = np.where(rng.random(sel.sum()) < 0.5, R2[sel],
                       np.nextafter(R2[sel], np.where(rng.random(sel.sum()) < 0.5, np.inf, 0).astype(f32)))
    return X, R2


def test_pixel_span_holds_every_pixel_the_disk_test_passes():
    rng = np.random.default_rng(11)
    X, R2 = footprints(rng, 4000)
    f0, f1 = span(X, R2)
    R = np.sqrt(R2.astype(np.float64))
    missed, loose = 0, 0
    for x, r2, r, a, b in zip(X, R2, R, f0, f1):
        lo = int(np.floor(float(x) - r)) - 3
        hi = int(np.ceil(float(x) + r)) + 3
        cols = np.arange(lo, hi + 1)
        ok = cols[in_disk_1d(x, r2, cols)]
        if ok.size:
            missed += int(ok.min() < a) + int(ok.max() > b)
            # tight: at most one extra column either side
            loose += int(a < ok.min() - 1) + int(b > ok.max() + 1)
        else:
            loose += int(b - a > 1)
    assert missed == 0
    assert loose == 0


def test_pixel_span_of_a_particle_that_reaches_no_centre_is_at_most_a_column():
    # tiny disks between two pixel centres: no centre passes, and the span
    # holds at most the one column the margin lets in
    X = (np.arange(1000, dtype=np.float64) + 0.0).astype(f32)
    R2 = np.full(X.shape, f32(0.01))
    f0, f1 = span(X, R2)
    assert not in_disk_1d(X, R2, X.astype(np.int64)).any()
    assert np.all(f1 - f0 <= 0)


def quadrant_keep(X, Y, R2, bx0, by0, W, H, Q=8, Qy=None, clip=True):
    """The composite's cull for the Q x Qy box (a quadrant: 8 x 8, clipped
    to the image) whose first pixel is (bx0, by0)."""
    Qy = Q if Qy is None else Qy
    cx0 = f32(bx0) + f32(0.5)
    cy0 = f32(by0) + f32(0.5)
    cx1 = cx0 + f32(Q - 1)
    cy1 = cy0 + f32(Qy - 1)
    if clip:
        cx1 = min(cx1, f32(W) - f32(0.5))
        cy1 = min(cy1, f32(H) - f32(0.5))
    dx = max(max(cx0 - X, X - cx1), f32(0.0))
    dy = max(max(cy0 - Y, Y - cy1), f32(0.0))
    return bool(cx0 <= cx1 and cy0 <= cy1 and (dx * dx + dy * dy) <= fmaf(R2, f32(1.0001), f32(1e-4)))


@pytest.mark.parametrize("Q, Qy, clip, off", [(8, 8, True, 0), (8, 8, True, 4000)],
                         ids=["near", "far"])
def test_box_cull_keeps_every_record_that_reaches_a_centre(Q, Qy, clip, off):
    # off: the boxes sit at pixel off..off + W (coarser float32 spacing of
    # the coordinates there); the image is then off + W by off + H
    rng = np.random.default_rng(12)
    W, H = 70, 53                  # ragged: the last boxes are cut by the image
    n = 3000
    X = (off + rng.uniform(-6, W + 6, n)).astype(f32)
    Y = (off + rng.uniform(-6, H + 6, n)).astype(f32)
    # snap a third of the centres to pixel centres and edges
    s = rng.random(n) < 1 / 3
    X[s] = (np.round(X[s]) + rng.choice([0.0, 0.5], s.sum())).astype(f32)
    R2 = np.exp(rng.uniform(np.log(1e-3), np.log(400.0), n)).astype(f32)
    # a third exactly on the rim of some pixel centre
    s = rng.random(n) < 1 / 3
    px = (np.floor(X[s]) + rng.integers(-6, 7, s.sum())).astype(f32) + f32(0.5) - X[s]
    py = (np.floor(Y[s]) + rng.integers(-6, 7, s.sum())).astype(f32) + f32(0.5) - Y[s]
    R2[s] = fmaf(px, px, py * py)
    gx, gy = np.meshgrid(off + np.arange(W), off + np.arange(H))
    cx = gx.astype(f32) + f32(0.5)
    cy = gy.astype(f32) + f32(0.5)
    dropped = kept = 0
    for x, y, r2 in zip(X, Y, R2):
        dx = cx - x
        dy = cy - y
        hit = fmaf(dx, dx, dy * dy) <= r2
        for by0 in range(0, H, Qy):
            for bx0 in range(0, W, Q):
                reach = hit[by0:by0 + Qy, bx0:bx0 + Q].any()
                keep = quadrant_keep(x, y, r2, off + bx0, off + by0, off + W, off + H, Q, Qy, clip)
                dropped += int(reach and not keep)
                kept += int(keep)
    assert dropped == 0
    assert kept > 0


@pytest.mark.parametrize("scale", [1e3, 3e4])
def test_pixel_span_margin_at_large_coordinates(scale):
    # centres far from the origin (a footprint partly on screen from far
    # away): the relative part of the margin covers the coarser float32
    # spacing there
    rng = np.random.default_rng(13)
    X = (scale + rng.uniform(0, 64, 2000)).astype(f32)
    R = rng.uniform(0.3, 50, 2000)
    R2 = (R ** 2).astype(f32)
    f0, f1 = span(X, R2)
    for x, r2, a, b in zip(X, R2, f0, f1):
        r = float(np.sqrt(np.float64(r2)))
        cols = np.arange(int(np.floor(float(x) - r)) - 3, int(np.ceil(float(x) + r)) + 4)
        ok = cols[in_disk_1d(x, r2, cols)]
        if ok.size:
            assert a <= ok.min() and ok.max() <= b
