"""FP64 NumPy reference of the learned x4 upscaler.

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's checks are the
only callers; the product path never imports this module.

The paper has no learned component; the network is the one the workload
description fixes: six 3x3 convolutions (4 -> 32, four 32 -> 32, 32 -> 48;
ReLU after all but the last), a x4 pixel shuffle of the 48 = 3*16 output
channels, the bilinearly upsampled low-resolution optical depth added as a
residual, clamped at zero (an optical depth is never negative), and the
resolve I = 1 - exp(-L) of Eq. 1 with E = A.  The input features are
log1p of the three low-resolution optical depths and of the centre count.  Parity of
this part is not pinned by the paper; its pins are mathematical (finite
differences, identities) and library cross-checks (see the tests).

Layouts (NHWC throughout):
  x      [N, H, W, Cin]          activations
  w      [Cout, 3, 3, Cin]       3x3 weights, cross-correlation, zero pad 1
  b      [Cout]                  bias
  conv6  [N, h, w, 48]           last layer output (low resolution)
  L_low  [N, h, w, 3]            low-resolution optical depth
  out    [N, 4h, 4w, 3]          image
"""
from __future__ import annotations

import math

import numpy as np

LAYERS = [(4, 32, True), (32, 32, True), (32, 32, True), (32, 32, True), (32, 32, True),
          (32, 48, False)]
SCALE = 4


def conv3x3(x, w, b=None):
    """y[n,i,j,o] = b[o] + sum_{dy,dx,c} w[o,dy,dx,c] x[n,i+dy-1,j+dx-1,c]."""
    N, H, W, C = x.shape
    O = w.shape[0]
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((N, H, W, O))
    for dy in range(3):
        for dx in range(3):
            y += xp[:, dy:dy + H, dx:dx + W, :] @ w[:, dy, dx, :].T
    if b is not None:
        y += b
    return y


def conv3x3_bwd_data(dy, w):
    """Gradient with respect to the input of conv3x3."""
    N, H, W, O = dy.shape
    C = w.shape[3]
    dxp = np.zeros((N, H + 2, W + 2, C))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + H, kx:kx + W, :] += dy @ w[:, ky, kx, :]
    return dxp[:, 1:-1, 1:-1]


def conv3x3_bwd_weight(x, dy):
    """Gradients with respect to w and b of conv3x3."""
    N, H, W, C = x.shape
    O = dy.shape[3]
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1] = x
    dw = np.zeros((O, 3, 3, C))
    d2 = dy.reshape(-1, O)
    for ky in range(3):
        for kx in range(3):
            dw[:, ky, kx, :] = d2.T @ xp[:, ky:ky + H, kx:kx + W, :].reshape(-1, C)
    return dw, d2.sum(axis=0)


def pixel_shuffle(a, r=SCALE):
    """out[n, r*i+p, r*j+q, c] = a[n, i, j, c*r*r + p*r + q]."""
    N, h, w, C = a.shape
    c = C // (r * r)
    t = a.reshape(N, h, w, c, r, r)            # [..., c, p, q]
    t = t.transpose(0, 1, 4, 2, 5, 3)           # N, h, p, w, q, c
    return t.reshape(N, h * r, w * r, c)


def pixel_unshuffle(o, r=SCALE):
    """Inverse of pixel_shuffle."""
    N, H, W, c = o.shape
    t = o.reshape(N, H // r, r, W // r, r, c)   # N, h, p, w, q, c
    t = t.transpose(0, 1, 3, 5, 2, 4)           # N, h, w, c, p, q
    return t.reshape(N, H // r, W // r, c * r * r)


def _bilinear_axis(n_in, r):
    """Source index pairs and weights of a x r bilinear upsample along one
    axis with half-pixel centres (output x <- input (x + 1/2)/r - 1/2,
    clamped to the edges)."""
    n_out = n_in * r
    src = (np.arange(n_out) + 0.5) / r - 0.5
    src = np.maximum(src, 0.0)
    i0 = np.floor(src).astype(np.int64)
    f = src - i0
    i0 = np.minimum(i0, n_in - 1)
    i1 = np.minimum(i0 + 1, n_in - 1)
    return i0, i1, f


def bilinear_up(a, r=SCALE):
    """x r bilinear upsampling of [N, h, w, C]."""
    N, h, w, C = a.shape
    y0, y1, fy = _bilinear_axis(h, r)
    x0, x1, fx = _bilinear_axis(w, r)
    top = a[:, y0] * (1 - fy)[None, :, None, None] + a[:, y1] * fy[None, :, None, None]
    return top[:, :, x0] * (1 - fx)[None, None, :, None] + top[:, :, x1] * fx[None, None, :, None]


def head(conv6, L_low):
    """Full-resolution optical depth (clamped at zero) and image from the
    last layer."""
    L = np.maximum(pixel_shuffle(conv6) + bilinear_up(L_low), 0.0)
    return L, -np.expm1(-L)


def mse(I, target):
    return float(np.mean((I - target) ** 2))


def head_backward(L, I, target):
    """d(MSE)/d(conv6) through resolve, clamp and shuffle (the clamp passes
    the gradient where L > 0)."""
    dL = 2.0 * (I - target) * np.exp(-L) * (L > 0) / I.size
    return pixel_unshuffle(dL)


def forward(params, x, L_low):
    """params: list of (w, b).  Returns (activations, L, I); activations[k]
    is the input of layer k, activations[-1] the last layer's output."""
    acts = [x]
    a = x
    for (w, b), (_, _, relu) in zip(params, LAYERS):
        a = conv3x3(a, w, b)
        if relu:
            a = np.maximum(a, 0.0)
        acts.append(a)
    L, I = head(acts[-1], L_low)
    return acts, L, I


def backward(params, acts, L, I, target):
    """Gradients (dw, db) of the MSE for every layer."""
    grads = [None] * len(params)
    d = head_backward(L, I, target)
    for k in range(len(params) - 1, -1, -1):
        w, _ = params[k]
        if LAYERS[k][2]:
            d = d * (acts[k + 1] > 0)
        dw, db = conv3x3_bwd_weight(acts[k], d)
        grads[k] = (dw, db)
        if k > 0:
            d = conv3x3_bwd_data(d, w)
    return grads


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (in place on p, m, v) with bias correction."""
    m *= b1
    m += (1 - b1) * g
    v *= b2
    v += (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p -= lr * mh / (np.sqrt(vh) + eps)


def consistency(L_full, L_low):
    """RMS over low-resolution pixels and channels of the image difference
    between the low-resolution optical depth and the predicted optical depth
    averaged over the 2x2 central full-resolution pixels of each 4x4 block."""
    c = (L_full[:, 1::4, 1::4] + L_full[:, 1::4, 2::4] + L_full[:, 2::4, 1::4]
         + L_full[:, 2::4, 2::4]) / 4.0
    d = np.expm1(-L_low) - np.expm1(-c)
    return float(math.sqrt(np.mean(d * d)))


def region_consistency(L_full, L_low, region):
    """Per square region of `region` full-resolution pixels (region/4
    low-resolution pixels per side), row-major: the RMS over the region's
    low-resolution pixels (inside the image) and channels of the image
    difference of ``consistency``.  L_full [4h, 4w, 3], L_low [h, w, 3]."""
    h, w = L_low.shape[:2]
    q = region // 4
    out = []
    for y0 in range(0, h, q):
        for x0 in range(0, w, q):
            lo = L_low[y0:y0 + q, x0:x0 + q]
            qy, qx = lo.shape[:2]
            blk = L_full[4 * y0:4 * (y0 + qy), 4 * x0:4 * (x0 + qx)]
            c = (blk[1::4, 1::4] + blk[1::4, 2::4] + blk[2::4, 1::4] + blk[2::4, 2::4]) / 4.0
            d = np.expm1(-lo) - np.expm1(-c)
            out.append(math.sqrt(float(np.mean(d * d))))
    return np.array(out)


def pack_input(log_accum, center_count):
    """Network input [N, h, w, 4]: log1p of the three optical depths and of
    the centre count."""
    return np.concatenate([np.log1p(log_accum),
                           np.log1p(center_count.astype(np.float64))[..., None]], axis=-1)


def psnr(I, ref):
    m = np.mean((np.asarray(I, np.float64) - np.asarray(ref, np.float64)) ** 2)
    return float("inf") if m == 0 else float(10.0 * math.log10(1.0 / m))


def init_params(seed=0, scale_last=0.1):
    """He-initialised weights (the last layer scaled down so that the
    untrained network adds little to the bilinear residual)."""
    g = np.random.default_rng(seed)
    params = []
    for k, (ci, co, _) in enumerate(LAYERS):
        std = math.sqrt(2.0 / (9 * ci))
        if k == len(LAYERS) - 1:
            std *= scale_last
        params.append((g.standard_normal((co, 3, 3, ci)) * std, np.zeros(co)))
    return params
