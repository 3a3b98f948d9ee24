"""Brute-force radiative transfer along pixel rays (NumPy, FP64).

TEST INFRASTRUCTURE ONLY.  This integrates Eq. 1 of the paper,
dI/dr = (E_p - A_p I) rho_p(x), summed over particles, along the ray from
the eye through each pixel centre, with rho_p the 3-D Gaussian of Eq. 2
clipped to zero beyond chi*h (Section "Splotch Overview").  Particles are
met in depth order simply because the integration walks the ray.  It shares
nothing with the splat oracle beyond the input generators: its own camera
rays, its own palette interpolation (``numpy.interp``), classical RK4.

It pins the splat oracle: for E = A and a narrow field of view, the
per-ray column of each clipped Gaussian equals the splat term
tau0 exp(-d^2/sigma^2) up to (i) the clip, at most tau0 exp(-chi^2), and
(ii) the small-angle difference between the distance of the particle to
the ray and its lateral offset in its depth plane, at most
tau0 exp(-1) sin^2(theta_max) (theta_max = widest ray angle off axis).
"""
from __future__ import annotations

import math

import numpy as np


def _basis(cam):
    e = np.asarray(cam.eye, np.float64)
    t = np.asarray(cam.target, np.float64)
    u = np.asarray(cam.up, np.float64)
    fwd = (t - e) / np.linalg.norm(t - e)
    right = np.cross(fwd, u)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    return e, right, up, fwd


def pixel_rays(cam):
    """Unit ray directions (H, W, 3) through pixel centres, and the largest
    angle between a ray and the optical axis."""
    e, right, up, fwd = _basis(cam)
    W, H = cam.width, cam.height
    f = 0.5 * W / math.tan(math.radians(cam.fov_deg) / 2)
    i = np.arange(W) + 0.5
    j = np.arange(H) + 0.5
    a = (i[None, :] - W / 2) / f                        # right component
    b = -(j[:, None] - H / 2) / f                       # up component
    d = (a[..., None] * right + b[..., None] * up + fwd)
    norm = np.linalg.norm(d, axis=-1, keepdims=True)
    d = d / norm
    theta_max = float(np.arccos(np.clip((d @ fwd).min(), -1, 1)))
    return e, d, theta_max


def coefficients(ps, cmap, prm, emission_scale=None):
    """Per-particle absorption A (n, 3) and emission E (n, 3).

    A = brightness[species] * palette(scalar); E = A unless an extra
    per-particle ``emission_scale`` (n,) is given for the E != A variant."""
    s = np.asarray(ps.scalar, np.float64)
    if prm.scalar_log10:
        s = np.log10(s)
    sn = np.clip((s - prm.scalar_min) / (prm.scalar_max - prm.scalar_min), 0.0, 1.0)
    sn = np.nan_to_num(sn, nan=0.0)
    cm = np.asarray(cmap, np.float64).reshape(-1, 3)
    knots = np.linspace(0.0, 1.0, cm.shape[0])
    col = np.stack([np.interp(sn, knots, cm[:, c]) for c in range(3)], axis=1)
    k = np.zeros(ps.n, np.int64) if ps.species is None else np.minimum(ps.species, 3)
    bright = np.asarray(prm.brightness, np.float64)[k]
    A = bright[:, None] * col
    E = A.copy() if emission_scale is None else A * np.asarray(emission_scale)[:, None]
    return A, E


def integrate(ps, cam, cmap, prm, steps_per_h: int = 50, reverse: bool = False,
              emission_scale=None):
    """Integrate Eq. 1 along every pixel ray; returns (I (H, W, 3), theta_max).

    Light reaches the eye from behind the particles, so the physical
    integration starts with I = 0 beyond the farthest particle and walks
    toward the eye.  ``reverse=True`` walks away from the eye instead (the
    order-swapped solution).  Central density rho0 = intensity / (sqrt(pi) h)
    (unit peak column) unless ``prm.col_norm`` is set (rho0 = intensity)."""
    eye, dirs, theta_max = pixel_rays(cam)
    H, W = cam.height, cam.width
    P = np.stack([ps.x, ps.y, ps.z], axis=1).astype(np.float64)
    h = np.asarray(ps.h, np.float64)
    inten = np.asarray(ps.intensity, np.float64)
    rho0 = inten if prm.col_norm else inten / (math.sqrt(math.pi) * h)
    A, E = coefficients(ps, cmap, prm, emission_scale)
    clip2 = (prm.chi * h) ** 2
    inv_h2 = 1.0 / h ** 2

    dist = np.linalg.norm(P - eye, axis=1)
    s_lo = max(float((dist - prm.chi * h).min()), 0.0)
    s_hi = float((dist + prm.chi * h).max())
    ds = float(h.min()) / steps_per_h
    nsteps = int(math.ceil((s_hi - s_lo) / ds))
    ds = (s_hi - s_lo) / nsteps

    D = dirs.reshape(-1, 3)
    # along-ray and squared perpendicular geometry of each particle per ray
    rel = P - eye                                   # (n, 3)
    t_p = D @ rel.T                                 # (npix, n) along-ray coordinate
    r2_p = (rel * rel).sum(1)[None, :] - t_p ** 2   # perpendicular distance^2

    def rho(s):
        d2 = r2_p + (s - t_p) ** 2
        val = rho0[None, :] * np.exp(-d2 * inv_h2[None, :])
        return np.where(d2 <= clip2[None, :], val, 0.0)   # (npix, n)

    def deriv(s, I):
        r = rho(s)
        return r @ E - I * (r @ A)

    I = np.zeros((D.shape[0], 3))
    if reverse:
        s, step = s_lo, ds
    else:
        s, step = s_hi, -ds
    # dI/dr with r the light-path coordinate: walking toward the eye means
    # dI/d(-s) = deriv; walking away means dI/ds = deriv.
    for _ in range(nsteps):
        k1 = deriv(s, I)
        k2 = deriv(s + step / 2, I + ds / 2 * k1)
        k3 = deriv(s + step / 2, I + ds / 2 * k2)
        k4 = deriv(s + step, I + ds * k3)
        I = I + ds / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        s += step
    return I.reshape(H, W, 3), theta_max


def splat_bound(ps, cmap, prm, theta_max):
    """Largest per-pixel |L_ode - L_splat| allowed by the two approximations
    named in the module docstring, summed over particles."""
    A, _ = coefficients(ps, cmap, prm)
    h = np.asarray(ps.h, np.float64)
    inten = np.asarray(ps.intensity, np.float64)
    col_fac = math.sqrt(math.pi) * h if prm.col_norm else 1.0
    tau0 = A * (inten * col_fac)[:, None]
    per = math.exp(-prm.chi ** 2) * math.exp(prm.chi ** 2 * math.sin(theta_max) ** 2) \
        + math.exp(-1.0) * math.sin(theta_max) ** 2
    return float((tau0.max(axis=1) * per).sum())
