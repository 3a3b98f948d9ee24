"""Seeded synthetic inputs for the Splotch rendering path.

This module only *draws* inputs: particle sets, colour tables and camera
presets.  It holds none of the rendering arithmetic (no projection, no
kernel evaluation, no accumulation), so both the HIP path and the FP64
reference renderer can take their inputs from here without sharing any of
the method.

The particle sets stand in for the paper's Gadget N-body/SPH snapshot
(Section "Results": about 2e8 dark-matter plus 2e8 gas particles), which is
not available.  They keep its shape: clustered matter, an even DM/gas split,
and smoothing lengths that follow the local density.

All arrays are float32 structure-of-arrays; ``species`` is uint8
(0 = gas with its own smoothing length, 1 = point-like dark matter).
Every draw uses ``numpy.random.Generator(PCG64(seed))`` in a fixed order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SPECIES_GAS = 0
SPECIES_DM = 1


@dataclass
class ParticleSet:
    """Host-side particle arrays (float32 SoA, uint8 species)."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    h: np.ndarray
    intensity: np.ndarray
    scalar: np.ndarray | None
    species: np.ndarray | None = None
    # vector colour input (e.g. velocity), used by the vector colour mode
    vx: np.ndarray | None = None
    vy: np.ndarray | None = None
    vz: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def subset(self, sl) -> "ParticleSet":
        def cut(a):
            return None if a is None else a[sl]
        return ParticleSet(
            self.x[sl], self.y[sl], self.z[sl], self.h[sl], self.intensity[sl],
            cut(self.scalar), cut(self.species), cut(self.vx), cut(self.vy), cut(self.vz),
        )

    def arrays(self):
        out = dict(x=self.x, y=self.y, z=self.z, h=self.h,
                   intensity=self.intensity, scalar=self.scalar,
                   species=self.species)
        if self.vx is not None:
            out.update(vx=self.vx, vy=self.vy, vz=self.vz)
        return out


@dataclass
class Camera:
    eye: tuple = (0.5, 0.5, -1.5)
    target: tuple = (0.5, 0.5, 0.5)
    up: tuple = (0.0, 1.0, 0.0)
    fov_deg: float = 45.0
    z_near: float = 1e-3
    width: int = 512
    height: int = 512


@dataclass
class Params:
    """Render parameters (mirrors the C struct ``splotch_params``)."""

    chi: float = 3.0
    brightness: tuple = (0.02, 0.02, 0.02, 0.02)
    fixed_sigma_frac: tuple = (0.0, 0.0, 0.0, 0.0)
    scalar_min: float = 0.0
    scalar_max: float = 1.0
    scalar_log10: int = 0
    col_norm: int = 0
    accum: int = 0           # 0 = FP32, 1 = int64 fixed point
    frac_bits: int = 40
    tile: int = 0            # 0 = tuned
    halo: int = -1           # <0 = tuned
    max_clip_tiles: int = 0  # 0 = tuned
    chunk: int = 0           # 0 = tuned
    colour_mode: int = 0     # 0 = palette of the scalar, 1 = vector (vx, vy, vz)
    transfer: int = 0        # 0 = emission equal to absorption, 1 = ordered (E != A)
    absorption: tuple = (0.0, 0.0, 0.0, 0.0)  # absorption scale per species (transfer 1)
    prefilter: float = 0.0   # screen-plane Gaussian prefilter sigma (px), 0 = none
    extra: dict = field(default_factory=dict)


def ramp_colormap(n: int = 256) -> np.ndarray:
    """The linear blue-to-orange palette used by every config: entry k is
    (1 - k/(n-1)) * (0.10, 0.20, 1.00) + (k/(n-1)) * (1.00, 0.60, 0.10)."""
    k = np.arange(n, dtype=np.float64)[:, None] / (n - 1)
    lo = np.array([0.10, 0.20, 1.00])
    hi = np.array([1.00, 0.60, 0.10])
    return ((1.0 - k) * lo + k * hi).astype(np.float32)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Config 1: uniform cube, log-normal smoothing lengths.
# ---------------------------------------------------------------------------
def uniform_cube(n: int = 131072, seed: int = 0, h_median: float = 0.005,
                 h_sigma_ln: float = 0.5) -> ParticleSet:
    """Positions uniform in [0,1)^3, h log-normal (median ``h_median``,
    sigma_ln ``h_sigma_ln``), intensity 1, scalar uniform in [0,1]."""
    g = _rng(seed)
    pos = g.random((3, n), dtype=np.float64)
    h = np.exp(math.log(h_median) + h_sigma_ln * g.standard_normal(n))
    scalar = g.random(n)
    return ParticleSet(
        x=pos[0].astype(np.float32), y=pos[1].astype(np.float32),
        z=pos[2].astype(np.float32), h=h.astype(np.float32),
        intensity=np.ones(n, np.float32), scalar=scalar.astype(np.float32),
        species=np.zeros(n, np.uint8),
    )


# ---------------------------------------------------------------------------
# Config 2 (and the sets of configs 4 and 5): N-body-like clustering.
# ---------------------------------------------------------------------------
def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    q = weights / weights.sum() * total
    base = np.floor(q).astype(np.int64)
    short = total - int(base.sum())
    if short > 0:
        order = np.argsort(-(q - base), kind="stable")
        base[order[:short]] += 1
    return base


def nbody_like(n: int, seed: int = 1, n_halos: int = 2000, halo_frac: float = 0.7,
               pareto_alpha: float = 1.9, rvir0: float = 0.02, grid: int = 256,
               h0: float = 0.002, h_min: float = 1e-4, h_max: float = 0.05,
               dm_frac: float = 0.5) -> ParticleSet:
    """Clustered particle set in the unit box.

    * ``halo_frac`` of the particles sit in ``n_halos`` halos whose masses are
      1 + Lomax(alpha) (a Pareto tail); particles are shared out in proportion
      to mass (largest remainder).  Halo centres are uniform; a halo's radius
      is ``rvir0 * M^(1/3)``; inside it the radius is uniform in [0, r_vir]
      (the 1/r^2 density profile) along an isotropic direction; positions wrap
      into the box.
    * The rest are uniform in the box.
    * Density: nearest-grid-point counts on a ``grid``^3 mesh divided by the
      cell volume, relative to the mean density N.  h = h0*(rho/rho_mean)^(-1/3)
      clipped to [h_min, h_max].
    * Species: dark matter with probability ``dm_frac`` (rendered with a fixed
      screen-space sigma), gas otherwise.
    * scalar = log10(rho) mapped to [0,1] between its 0.1 and 99.9 percentiles.
    * The particle order is random (halo membership is shuffled), so memory
      order carries no spatial locality.
    """
    g = _rng(seed)
    masses = 1.0 + g.pareto(pareto_alpha, n_halos)
    centres = g.random((n_halos, 3))
    rvir = rvir0 * np.cbrt(masses)
    n_halo_total = int(round(halo_frac * n))
    counts = _largest_remainder(masses, n_halo_total)
    labels = np.repeat(np.arange(n_halos, dtype=np.int16), counts)
    labels = np.concatenate([labels, np.full(n - n_halo_total, -1, np.int16)])
    labels = g.permutation(labels)
    in_halo = labels >= 0
    lab = np.where(in_halo, labels, 0).astype(np.int64)

    # isotropic directions and uniform radii for halo members
    d = g.standard_normal((3, n), dtype=np.float32)
    d /= np.sqrt((d * d).sum(axis=0, keepdims=True)) + np.float32(1e-30)
    r = (g.random(n, dtype=np.float32) * rvir[lab].astype(np.float32))
    bg = g.random((3, n), dtype=np.float32)
    pos = np.empty((3, n), np.float32)
    for a in range(3):
        hp = centres[lab, a].astype(np.float32) + r * d[a]
        hp = np.mod(hp, np.float32(1.0))
        pos[a] = np.where(in_halo, hp, bg[a])
    # guard against float32 mod landing exactly on 1.0
    np.minimum(pos, np.nextafter(np.float32(1.0), np.float32(0.0)), out=pos)
    del d, r, bg, lab, labels

    cell = np.minimum((pos * grid).astype(np.int64), grid - 1)
    flat = (cell[0] * grid + cell[1]) * grid + cell[2]
    del cell
    cnt = np.bincount(flat, minlength=grid ** 3)
    rho_rel = cnt[flat].astype(np.float64) * (grid ** 3) / n
    del flat, cnt
    h = np.clip(h0 * rho_rel ** (-1.0 / 3.0), h_min, h_max).astype(np.float32)
    logr = np.log10(rho_rel * n)
    lo, hi = np.percentile(logr, [0.1, 99.9])
    scalar = np.clip((logr - lo) / max(hi - lo, 1e-30), 0.0, 1.0).astype(np.float32)
    del logr, rho_rel
    species = (g.random(n, dtype=np.float32) < dm_frac).astype(np.uint8)
    return ParticleSet(x=pos[0].copy(), y=pos[1].copy(), z=pos[2].copy(), h=h,
                       intensity=np.ones(n, np.float32), scalar=scalar,
                       species=species)


def nbody_like_device(n: int, seed: int, device="cuda:0", n_halos: int = 2000,
                      halo_frac: float = 0.7, pareto_alpha: float = 1.9, rvir0: float = 0.02,
                      grid: int = 256, h0: float = 0.002, h_min: float = 1e-4,
                      h_max: float = 0.05, dm_frac: float = 0.5) -> dict:
    """The ``nbody_like`` recipe drawn on the device with torch's generator
    (the many sets of the upscaler's training and evaluation splits).  The
    halo catalogue (masses, centres, member counts) is the same as
    ``nbody_like`` draws for the seed; the per-particle draws come from a
    torch generator seeded with ``seed``, so the set has the same
    distribution but not the same particles.  Returns a dict of device
    tensors (x, y, z, h, intensity, scalar, species)."""
    import torch
    g = _rng(seed)
    masses = 1.0 + g.pareto(pareto_alpha, n_halos)
    centres = torch.from_numpy(g.random((n_halos, 3))).to(device=device, dtype=torch.float32)
    rvir = torch.from_numpy(rvir0 * np.cbrt(masses)).to(device=device, dtype=torch.float32)
    n_halo_total = int(round(halo_frac * n))
    counts = torch.from_numpy(_largest_remainder(masses, n_halo_total)).to(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    labels = torch.repeat_interleave(torch.arange(n_halos, device=device), counts)
    labels = torch.cat([labels, torch.full((n - n_halo_total,), -1, device=device,
                                           dtype=labels.dtype)])
    labels = labels[torch.randperm(n, generator=gen, device=device)]
    in_halo = labels >= 0
    lab = labels.clamp_min(0)
    del labels
    d = torch.randn((3, n), generator=gen, device=device)
    d /= torch.sqrt((d * d).sum(dim=0, keepdim=True)) + 1e-30
    r = torch.rand(n, generator=gen, device=device) * rvir[lab]
    pos = torch.rand((3, n), generator=gen, device=device)
    one_minus = float(np.nextafter(np.float32(1.0), np.float32(0.0)))
    for a in range(3):
        hp = torch.remainder(centres[lab, a] + r * d[a], 1.0)
        pos[a] = torch.where(in_halo, hp, pos[a]).clamp_(max=one_minus)
    del d, r, lab, in_halo
    cell = (pos * grid).long().clamp_(max=grid - 1)
    flat = (cell[0] * grid + cell[1]) * grid + cell[2]
    del cell
    cnt = torch.bincount(flat, minlength=grid ** 3)
    rho_rel = cnt[flat].double() * (grid ** 3) / n
    del flat, cnt
    h = torch.clamp(h0 * rho_rel ** (-1.0 / 3.0), h_min, h_max).float()
    logr = torch.log10(rho_rel * n)
    srt = torch.sort(logr).values
    lo = float(srt[int(round(0.001 * (n - 1)))])
    hi = float(srt[int(round(0.999 * (n - 1)))])
    del srt
    scalar = torch.clamp((logr - lo) / max(hi - lo, 1e-30), 0.0, 1.0).float()
    del logr, rho_rel
    species = (torch.rand(n, generator=gen, device=device) < dm_frac).to(torch.uint8)
    return dict(x=pos[0].contiguous(), y=pos[1].contiguous(), z=pos[2].contiguous(), h=h,
                intensity=torch.ones(n, device=device), scalar=scalar, species=species)


# ---------------------------------------------------------------------------
# Config 3: large-footprint stress.
# ---------------------------------------------------------------------------
def pareto_cube(n: int = 10_000_000, seed: int = 2, alpha: float = 1.5,
                x_min: float = 0.001, h_cap: float = 0.3) -> ParticleSet:
    """Uniform positions; h = min(x_min*(1 + Lomax(alpha)), h_cap)."""
    g = _rng(seed)
    pos = g.random((3, n), dtype=np.float32)
    h = np.minimum(x_min * (1.0 + g.pareto(alpha, n)), h_cap).astype(np.float32)
    scalar = g.random(n, dtype=np.float32)
    return ParticleSet(x=pos[0].copy(), y=pos[1].copy(), z=pos[2].copy(), h=h,
                       intensity=np.ones(n, np.float32), scalar=scalar,
                       species=np.zeros(n, np.uint8))


# ---------------------------------------------------------------------------
# Cameras.
# ---------------------------------------------------------------------------
def orbit_cameras(k: int = 64, radius: float = 1.8, width: int = 1024,
                  height: int = 1024, fov_deg: float = 45.0) -> list:
    """``k`` views on a horizontal circle of ``radius`` around the box centre."""
    cams = []
    for i in range(k):
        phi = 2.0 * math.pi * i / k
        eye = (0.5 + radius * math.sin(phi), 0.5, 0.5 - radius * math.cos(phi))
        cams.append(Camera(eye=eye, target=(0.5, 0.5, 0.5), fov_deg=fov_deg,
                           width=width, height=height))
    return cams


def random_camera(seed: int, width: int, height: int) -> Camera:
    """Random outside-in view of the unit box: eye = centre + D*v with v
    uniform on the sphere and D ~ U[1.2, 2.5]; target jittered by 0.1;
    fov ~ U[30, 60] degrees; up = +y unless the view is nearly vertical."""
    g = _rng(seed)
    v = g.standard_normal(3)
    v /= np.linalg.norm(v)
    dist = g.uniform(1.2, 2.5)
    target = 0.5 + 0.1 * g.uniform(-1.0, 1.0, 3)
    fov = g.uniform(30.0, 60.0)
    up = (0.0, 0.0, 1.0) if abs(v[1]) > 0.99 else (0.0, 1.0, 0.0)
    eye = 0.5 + dist * v
    return Camera(eye=tuple(float(a) for a in eye),
                  target=tuple(float(a) for a in target), up=up,
                  fov_deg=float(fov), width=width, height=height)


def batch_shapes(seeds=range(400, 416)) -> list:
    """Config 4b job shapes: (seed, n, side) with n log-uniform in
    [1e5, 5e7] and side*side log-uniform in [256^2, 2048^2], side a
    multiple of 8."""
    out = []
    for s in seeds:
        g = _rng(s)
        n = int(round(math.exp(g.uniform(math.log(1e5), math.log(5e7)))))
        area = math.exp(g.uniform(math.log(256.0 ** 2), math.log(2048.0 ** 2)))
        side = int(8 * round(math.sqrt(area) / 8))
        out.append((s, n, side))
    return out
