"""Learned x4 upscaler: weights, training step and the serving path with its
consistency check and plain-render fallback.

Network (all convolutions 3x3, zero padding, NHWC):
    input   [n, h, w, 4]   bf16: optical depth R, G, B and log1p(centre count)
    conv 4 -> 32, ReLU; four conv 32 -> 32, ReLU; conv 32 -> 48
    head    x4 pixel shuffle of the 48 = 3 x 16 channels, plus the x4
            bilinear upsample of the low-resolution optical depth, then the
            resolve I = 1 - exp(-L) (Eq. 1 with emission equal to absorption)

Every operation runs in the library's kernels (include/splotch_nn.h); this
module owns the buffers and the order of the calls.  Master weights, their
gradients and the Adam moments are FP32; the convolutions read bf16 copies.

Serving (``LearnedRenderer``): render at a quarter of the resolution per
side with the same camera and parameters (``low_params``: by default a
species drawn with a fixed screen-space sigma keeps its fraction of the
image width, and the weights may ask for an anti-aliasing prefilter), run
the network in one library call, compute the consistency of the prediction
with the low-resolution render per square region, and render the regions
whose metric exceeds the threshold theta (or is not finite) at full
resolution with the plain path, into the same frame.
"""
from __future__ import annotations

import math
from dataclasses import replace
from pathlib import Path

import numpy as np

from . import nn

LAYERS = ((4, 32, True), (32, 32, True), (32, 32, True), (32, 32, True), (32, 32, True),
          (32, 48, False))
SCALE = 4
PAD = 64          # every parameter segment starts on a 256-byte boundary


def _layout():
    segs, off = [], 0
    for ci, co, _ in LAYERS:
        wn, bn = co * 9 * ci, co
        segs.append((off, wn, off + wn + (-wn) % PAD, bn))
        off = segs[-1][2] + bn + (-bn) % PAD
    return segs, off


SEGMENTS, FLAT_SIZE = _layout()
N_PARAMS = sum(co * 9 * ci + co for ci, co, _ in LAYERS)


def he_init(seed=0, scale_last=0.1):
    """He-normal weights (the last layer scaled down so that an untrained
    network adds little to the bilinear residual) and zero biases."""
    g = np.random.default_rng(seed)
    out = []
    for k, (ci, co, _) in enumerate(LAYERS):
        std = math.sqrt(2.0 / (9 * ci)) * (scale_last if k == len(LAYERS) - 1 else 1.0)
        out.append((g.standard_normal((co, 3, 3, ci)) * std, np.zeros(co)))
    return out


class Upscaler:
    """Weights, optimiser state and scratch buffers on one device."""

    def __init__(self, params=None, device: int = 0, seed: int = 0, lr: float = 1e-3,
                 low_sigma: str = "fraction", prefilter: float = 0.0, low_chi: float = 0.0):
        import torch
        self.dev = torch.device(f"cuda:{device}")
        self.low_sigma = low_sigma
        self.prefilter = float(prefilter)
        self.low_chi = float(low_chi)      # 0: the frame's own chi
        self.meta = {}
        self.lr = lr
        self.step = 0
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.P = torch.zeros(FLAT_SIZE, **f32)
        self.G = torch.zeros(FLAT_SIZE, **f32)
        self.M = torch.zeros(FLAT_SIZE, **f32)
        self.V = torch.zeros(FLAT_SIZE, **f32)
        self.Pb = torch.zeros(FLAT_SIZE, dtype=torch.bfloat16, device=self.dev)
        self.set_params(params if params is not None else he_init(seed))
        self._bufs = {}
        self.loss_sum = torch.zeros(1, **f32)

    # -- parameter views ---------------------------------------------------
    def _w(self, t, k):
        ci, co, _ = LAYERS[k]
        o, n, _, _ = SEGMENTS[k]
        return t[o:o + n].reshape(co, 3, 3, ci)

    def _b(self, t, k):
        _, _, o, n = SEGMENTS[k]
        return t[o:o + n]

    def set_params(self, params):
        import torch
        host = np.zeros(FLAT_SIZE, np.float32)
        for k, (w, b) in enumerate(params):
            o, n, ob, nb = SEGMENTS[k]
            host[o:o + n] = np.asarray(w, np.float32).reshape(-1)
            host[ob:ob + nb] = np.asarray(b, np.float32)
        self.P.copy_(torch.from_numpy(host))
        self.sync_weights()

    def params(self):
        P = self.P.cpu().numpy()
        return [(self._w(P, k).copy(), self._b(P, k).copy()) for k in range(len(LAYERS))]

    def gradients(self):
        G = self.G.cpu().numpy()
        return [(self._w(G, k).copy(), self._b(G, k).copy()) for k in range(len(LAYERS))]

    def sync_weights(self):
        """bf16 copies of the master weights and the flipped copies the data
        gradient uses."""
        nn.to_bf16(self.P, out=self.Pb)
        self.Wt = [None] + [nn.flip_weights(self._w(self.Pb, k)) for k in range(1, len(LAYERS))]
        ws = nn.NNWeights()
        for k in range(len(LAYERS)):
            ws.w[k] = self._w(self.Pb, k).data_ptr()
            ws.b[k] = self._b(self.P, k).data_ptr()
        self.weights_struct = ws

    # -- buffers -------------------------------------------------------------
    def _buf(self, name, shape, dtype):
        import torch
        key = (name, tuple(shape), dtype)
        t = self._bufs.get(key)
        if t is None:
            t = torch.empty(shape, dtype=dtype, device=self.dev)
            self._bufs[key] = t
        return t

    # -- network -------------------------------------------------------------
    def forward(self, x, L_low, rgb=None, L_full=None, target=None, dconv6=None):
        """x: bf16 [n, h, w, 4]; L_low: float [n, h, w, 3].  Returns rgb
        [n, 4h, 4w, 3] and keeps the activations for ``backward``."""
        import torch
        n, h, w, _ = x.shape
        acts = [x]
        a = x
        for k, (ci, co, relu) in enumerate(LAYERS):
            last = k == len(LAYERS) - 1
            out = self._buf(f"a{k}", (n, h, w, co), torch.float32 if last else torch.bfloat16)
            a = nn.conv3x3_fwd(a, self._w(self.Pb, k), self._b(self.P, k), relu=relu,
                               out_f32=last, out=out)
            acts.append(a)
        self.acts = acts
        if rgb is None:
            rgb = self._buf("rgb", (n, SCALE * h, SCALE * w, 3), torch.float32)
        return nn.head(acts[-1], L_low, rgb=rgb, L_full=L_full, target=target,
                       loss_sum=self.loss_sum if target is not None else None, dconv6=dconv6)

    def train_step(self, x, L_low, target, apply=True, lr=None):
        """One step on a batch: forward, MSE against ``target``, backward
        into self.G and (if apply) an Adam update.  Returns the batch MSE
        (this reads one scalar back)."""
        import torch
        n, h, w, _ = x.shape
        self.loss_sum.zero_()
        d6 = self._buf("d6", (n, h, w, 48), torch.bfloat16)
        self.forward(x, L_low, target=target, dconv6=d6)
        self.G.zero_()
        g = d6
        for k in range(len(LAYERS) - 1, -1, -1):
            ci, co, relu = LAYERS[k]
            mask = self.acts[k + 1] if relu else None
            nn.conv3x3_bwd_weight(self.acts[k], g, self._w(self.G, k), self._b(self.G, k),
                                  mask=mask)
            if k > 0:
                g = nn.conv3x3_fwd(g, self.Wt[k], mask=mask, relu=False,
                                   out=self._buf(f"g{k}", (n, h, w, ci), torch.bfloat16))
        if apply:
            self.step += 1
            nn.adam(self.P, self.G, self.M, self.V, self.step, lr=self.lr if lr is None else lr)
            self.sync_weights()
        return float(self.loss_sum.item()) / (3.0 * target[..., 0].numel())

    # -- persistence -----------------------------------------------------------
    def save(self, path, **meta):
        arrays = {"P": self.P.cpu().numpy(), "M": self.M.cpu().numpy(),
                  "V": self.V.cpu().numpy(), "step": np.array(self.step),
                  "low_sigma": np.array(self.low_sigma),
                  "prefilter": np.array(self.prefilter), "low_chi": np.array(self.low_chi)}
        for k, v in meta.items():
            arrays[f"meta_{k}"] = np.asarray(v)
        np.savez(path, **arrays)

    @classmethod
    def load(cls, path, device: int = 0):
        import torch
        z = np.load(path, allow_pickle=False)
        up = cls(params=he_init(0), device=device)
        up.P.copy_(torch.from_numpy(z["P"]))
        up.M.copy_(torch.from_numpy(z["M"]))
        up.V.copy_(torch.from_numpy(z["V"]))
        up.step = int(z["step"])
        up.low_sigma = str(z["low_sigma"]) if "low_sigma" in z.files else "fraction"
        up.prefilter = float(z["prefilter"]) if "prefilter" in z.files else 0.0
        up.low_chi = float(z["low_chi"]) if "low_chi" in z.files else 0.0
        up.meta = {k[5:]: z[k] for k in z.files if k.startswith("meta_")}
        up.sync_weights()
        return up


def low_params(prm, low_sigma="fraction", prefilter=0.0, chi=0.0):
    """Parameters of the quarter-resolution render.  low_sigma "pixel": a
    species with a fixed screen-space sigma keeps that sigma in pixels of
    the rendered frame (its fraction of the image width grows by the scale
    factor); "fraction": it keeps its fraction of the image width (the
    same scene, sampled more coarsely).  prefilter > 0: the render samples
    the optical depth convolved with a Gaussian of that sigma (pixels of
    the rendered frame), an anti-aliased coarse image.  chi > 0: the clip
    radius of the coarse render in sigmas (the network's input need not
    carry the far tails).  Everything else is unchanged."""
    if low_sigma == "pixel":
        prm = replace(prm, fixed_sigma_frac=tuple(min(1.0, SCALE * f)
                                                  for f in prm.fixed_sigma_frac))
    elif low_sigma != "fraction":
        raise ValueError(f"unknown low_sigma {low_sigma!r}")
    if prefilter:
        prm = replace(prm, prefilter=float(prefilter))
    return replace(prm, chi=float(chi)) if chi else prm


class LearnedRenderer:
    """Serve frames through the upscaler, falling back to the plain
    full-resolution render region by region: each square region of
    ``region`` full-resolution pixels whose consistency metric exceeds
    theta (or is not finite) is rendered by the plain path into the frame,
    in one render restricted to those regions."""

    def __init__(self, renderer, upscaler: Upscaler, theta: float, region: int = 64):
        self.R = renderer
        self.up = upscaler
        self.theta = float(theta)
        self.region = int(region)
        self.metric = None             # whole-frame consistency RMS
        self.fallback = False          # some region was rendered by the plain path
        self.fallback_fraction = 0.0   # share of the regions rendered by the plain path

    def low_camera(self, cam):
        if cam.width % SCALE or cam.height % SCALE:
            raise ValueError("image sides must be multiples of 4")
        return replace(cam, width=cam.width // SCALE, height=cam.height // SCALE)

    def n_regions(self, cam):
        return (-(-cam.width // self.region)) * (-(-cam.height // self.region))

    def render(self, parts, cam, cmap, prm, rgb=None):
        """Returns the [H, W, 3] image; sets self.metric, self.fallback and
        self.fallback_fraction.  Two scalars are read back (the marked
        region count and the frame metric)."""
        import torch
        lc = self.low_camera(cam)
        h, w = lc.height, lc.width
        up = self.up
        la = up._buf("low_L", (1, h, w, 3), torch.float32)
        cc = up._buf("low_cc", (1, h, w), torch.int32)
        low_rgb = up._buf("low_rgb", (h, w, 3), torch.float32)
        self.R.render(parts, lc, cmap, low_params(prm, up.low_sigma, up.prefilter, up.low_chi),
                      rgb=low_rgb,
                      log_accum=la[0], center_count=cc[0])
        if rgb is None:
            rgb = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device=up.dev)
        Lf = up._buf("L_full", (1, cam.height, cam.width, 3), torch.float32)
        s = up._buf("check", (1,), torch.float32)
        ws = up._buf("upscale_ws", (nn.upscale_workspace_size(1, h, w),), torch.uint8)
        nn.upscale(up.weights_struct, la, cc, rgb.view(1, cam.height, cam.width, 3), L_full=Lf,
                   check=s, workspace=ws)
        nreg = self.n_regions(cam)
        mask = up._buf("region_mask", (nreg,), torch.uint8)
        rmet = up._buf("region_metric", (nreg,), torch.float32)
        nm = up._buf("n_marked", (1,), torch.int32)
        nm.zero_()
        nn.region_check(Lf, la, self.region, self.theta, mask, nm, metric=rmet)
        n_marked = int(nm.item())
        self.metric = math.sqrt(float(s.item()) / (3.0 * h * w))
        self.fallback_fraction = n_marked / nreg
        self.fallback = n_marked > 0
        if n_marked:
            self.R.render(parts, cam, cmap, prm, rgb=rgb, region_mask=mask,
                          region_size=self.region)
        return rgb


def default_weights_path() -> Path:
    return Path(__file__).resolve().parent / "weights" / "upscaler_c5.npz"
