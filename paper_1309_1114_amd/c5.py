"""The upscaler workload: training pairs, training loop, threshold choice and
the learned-versus-plain evaluation.

Pairs are rendered on the GPU by the plain path from seeded C2-style
particle sets (``synth.nbody_like_device``) seen through random cameras:
the low-resolution render (512^2: optical depth and centre counts, packed
into the network input) and the full-resolution image (2048^2) it should
reproduce.  The low-resolution frame is the same scene at a quarter of the
resolution per side (point-like dark matter stays one pixel wide, as the
serving path renders it).

    python -m paper_1309_1114_amd.c5 train --out weights.npz [--sets 200 ...]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import configs, nn, splotch, synth
from .upscaler import SCALE, LearnedRenderer, Upscaler, low_params


def log(msg):
    print(f"[c5] {msg}", flush=True)


def psnr(a, b) -> float:
    """PSNR in dB of two images in [0, 1] (device tensors)."""
    m = float(((a.double() - b.double()) ** 2).mean())
    return math.inf if m == 0 else 10.0 * math.log10(1.0 / m)


class Pairs:
    """Training pairs held in HBM: x (bf16 [P, h, w, 4]), L_low (float
    [P, h, w, 3]) and the target image (float16 [P, H, W, 3])."""

    def __init__(self, R, cmap, set_seeds, cams_per_set, n=configs.C5_N,
                 full=configs.C5_FULL, device="cuda:0", low_sigma="pixel", prefilter=0.0,
                 low_chi=0.0):
        import torch
        low = full // SCALE
        P = len(set_seeds) * cams_per_set
        self.x = torch.empty((P, low, low, 4), dtype=torch.bfloat16, device=device)
        self.L = torch.empty((P, low, low, 3), dtype=torch.float32, device=device)
        self.t = torch.empty((P, full, full, 3), dtype=torch.float16, device=device)
        prm = configs.c5_params(full)
        lprm = low_params(prm, low_sigma, prefilter, low_chi)
        rgb = torch.empty((full, full, 3), device=device)
        lrgb = torch.empty((low, low, 3), device=device)
        cc = torch.empty((low, low), dtype=torch.int32, device=device)
        t0 = time.time()
        i = 0
        for s in set_seeds:
            parts = synth.nbody_like_device(n, s, device=device)
            for k in range(cams_per_set):
                cam = configs.c5_camera(s, k, full)
                R.render(parts, cam, cmap, prm, rgb=rgb)
                self.t[i].copy_(rgb)
                lc = configs.c5_camera(s, k, low)
                R.render(parts, lc, cmap, lprm, rgb=lrgb, log_accum=self.L[i], center_count=cc)
                nn.pack_input(self.L[i:i + 1], cc[None], out=self.x[i:i + 1])
                i += 1
            del parts
            if (s - set_seeds[0]) % 20 == 0:
                torch.cuda.synchronize()
                log(f"pairs: set {s} done, {i}/{P} pairs, {time.time() - t0:.1f} s")
        torch.cuda.synchronize()
        self.P = P
        log(f"pairs: {P} rendered in {time.time() - t0:.1f} s")


def train(up: Upscaler, pairs: Pairs, steps: int, batch: int, crop: int, lr: float,
          seed: int = 0, log_every: int = 200, rng_state=None, ckpt=None, ckpt_every: int = 0,
          until=None):
    """Adam on random crops (crop x crop low-resolution pixels) with a
    cosine learning-rate decay to lr / 20 over `steps` steps.  Training runs
    from step up.step (0 for a new network) to `until` (default: steps), so
    a network loaded from a checkpoint continues where it stopped; rng_state,
    the crop sampler's state saved with that checkpoint, makes it draw the
    same crops as an uninterrupted run.  With ckpt and ckpt_every, every
    ckpt_every steps the weights, Adam moments, step and sampler state are
    saved to ckpt."""
    import torch
    g = np.random.default_rng(seed)
    if rng_state is not None:
        g.bit_generator.state = rng_state
    low = pairs.x.shape[1]
    xb = torch.empty((batch, crop, crop, 4), dtype=torch.bfloat16, device=up.dev)
    Lb = torch.empty((batch, crop, crop, 3), dtype=torch.float32, device=up.dev)
    tb = torch.empty((batch, SCALE * crop, SCALE * crop, 3), dtype=torch.float32, device=up.dev)
    t0 = time.time()
    hist = []
    for it in range(up.step, steps if until is None else min(until, steps)):
        for b in range(batch):
            i = int(g.integers(pairs.P))
            y, x = (int(v) for v in g.integers(0, low - crop + 1, 2))
            xb[b].copy_(pairs.x[i, y:y + crop, x:x + crop])
            Lb[b].copy_(pairs.L[i, y:y + crop, x:x + crop])
            tb[b].copy_(pairs.t[i, SCALE * y:SCALE * (y + crop), SCALE * x:SCALE * (x + crop)])
        cur = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * it / max(steps, 1))))
        mse = up.train_step(xb, Lb, tb, lr=cur)
        hist.append(mse)
        if (it + 1) % log_every == 0 or it == 0:
            m = float(np.mean(hist[-log_every:]))
            log(f"step {it + 1}/{steps} lr {cur:.2e} mse {m:.3e} "
                f"(psnr {10 * math.log10(1 / max(m, 1e-30)):.2f} dB) {time.time() - t0:.1f} s")
        if ckpt and ckpt_every > 0 and (it + 1) % ckpt_every == 0:
            save_checkpoint(up, ckpt, g, steps=steps, batch=batch, crop=crop, lr=lr, seed=seed)
    return hist


def save_checkpoint(up: Upscaler, path, g, **meta):
    """The network and optimiser (Upscaler.save) plus the crop sampler's
    state, as JSON text in the same .npz."""
    up.save(path, rng_state=json.dumps(g.bit_generator.state), **meta)


def checkpoint_rng_state(up: Upscaler):
    """The sampler state saved by save_checkpoint, or None."""
    s = up.meta.get("rng_state")
    return None if s is None else json.loads(str(s))


def evaluate(R, up: Upscaler, cmap, seeds, theta=math.inf, n=configs.C5_N,
             full=configs.C5_FULL, reps=1, device="cuda:0", tune=True, region=64):
    """Per frame: the plain full-resolution render (reference and timing),
    the learned path (low-resolution render, network, per-region check,
    plain render of the regions whose metric exceeds theta) and the bilinear
    baseline (the same head with the network's residual set to zero).  With
    tune, the schedule knobs of both renders' size buckets are tuned on the
    first frame (the context keeps them).  Each row also holds, per region,
    the consistency metric and the squared error of the network's own
    prediction (for the choice of theta).  Returns a list of dicts."""
    import torch
    prm = configs.c5_params(full)
    LR = LearnedRenderer(R, up, theta, region)
    ref = torch.empty((full, full, 3), device=device)
    out = torch.empty_like(ref)
    low = full // SCALE
    zero6 = torch.zeros((1, low, low, 48), device=device)
    base = torch.empty((1, full, full, 3), device=device)
    nrx = -(-full // region)
    rows = []
    for s in seeds:
        parts = synth.nbody_like_device(n, s, device=device)
        cam = configs.c5_camera(s, 0, full)
        if tune:
            R.autotune(parts, cam, cmap, prm, ref)
            lc = LR.low_camera(cam)
            R.autotune(parts, lc, cmap, low_params(prm, up.low_sigma, up.prefilter, up.low_chi),
                       torch.empty((lc.height, lc.width, 3), device=device))
            tune = False
        # warm both paths once (workspace, first-launch costs)
        R.render(parts, cam, cmap, prm, rgb=ref)
        LR.render(parts, cam, cmap, prm, rgb=out)
        torch.cuda.synchronize()
        tp, tl = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            R.render(parts, cam, cmap, prm, rgb=ref)
            torch.cuda.synchronize()
            tp.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            LR.render(parts, cam, cmap, prm, rgb=out)
            torch.cuda.synchronize()
            tl.append(time.perf_counter() - t0)
        # the network's own prediction (before any fallback) for the PSNR
        metric, frac = LR.metric, LR.fallback_fraction
        pred = up._buf("pred", (1, full, full, 3), torch.float32)
        la = up._bufs[("low_L", (1, low, low, 3), torch.float32)]
        cc = up._bufs[("low_cc", (1, low, low), torch.int32)]
        nn.upscale(up.weights_struct, la, cc, pred,
                   workspace=up._bufs[("upscale_ws", (nn.upscale_workspace_size(1, low, low),),
                                       torch.uint8)])
        nn.head(zero6, la, rgb=base)
        rmet = up._bufs[("region_metric", (LR.n_regions(cam),), torch.float32)]
        err = ((pred[0].double() - ref.double()) ** 2).sum(-1)
        rerr = err.reshape(nrx, region, nrx, region).sum((1, 3)).flatten()
        rows.append(dict(seed=s, t_plain=float(np.median(tp)), t_learned=float(np.median(tl)),
                         metric=metric, fallback=LR.fallback, fallback_fraction=frac,
                         psnr_net=psnr(pred[0], ref), psnr_served=psnr(out, ref),
                         psnr_bilinear=psnr(base[0], ref),
                         region_metric=rmet.cpu().numpy().astype(np.float64),
                         region_err=rerr.cpu().numpy()))
        del parts
    return rows


def served_psnr(row, theta):
    """PSNR of a frame whose regions with metric > theta (or not finite) are
    replaced by the plain render (their error taken as zero)."""
    m, e = row["region_metric"], row["region_err"]
    keep = m <= theta
    mse = float(e[keep].sum()) / (3.0 * configs.C5_FULL * configs.C5_FULL)
    return math.inf if mse == 0 else 10.0 * math.log10(1.0 / mse)


def choose_theta(rows, target_db=40.0, margin_db=0.5):
    """Largest region threshold under which every validation frame, with
    its marked regions rendered by the plain path, reaches target_db +
    margin_db (-inf: every region falls back)."""
    cand = np.unique(np.concatenate([r["region_metric"] for r in rows]))
    cand = cand[np.isfinite(cand)]
    if cand.size == 0:
        return -math.inf
    cand = np.unique(np.quantile(cand, np.linspace(0.0, 1.0, 2001)))
    best = -math.inf
    for th in cand:                       # ascending: the last that passes wins
        if all(served_psnr(r, th) >= target_db + margin_db for r in rows):
            best = float(th)
        else:
            break
    return best


def summary(rows):
    """Mean frames/s of both paths, the share of regions the plain path
    rendered, the PSNR of the served frames and, over all frames, of the
    network's prediction and of the bilinear baseline."""
    tp = np.array([r["t_plain"] for r in rows])
    tl = np.array([r["t_learned"] for r in rows])
    served = np.array([r["psnr_served"] for r in rows])
    pn = np.array([r["psnr_net"] for r in rows])
    pb = np.array([r["psnr_bilinear"] for r in rows])
    fr = np.array([r["fallback_fraction"] for r in rows])
    return dict(frames=len(rows), fps_plain=float(np.mean(1.0 / tp)),
                fps_learned=float(np.mean(1.0 / tl)),
                region_fallback_mean=float(fr.mean()), region_fallback_max=float(fr.max()),
                frames_without_fallback=int(sum(not r["fallback"] for r in rows)),
                psnr_served_mean=float(np.mean(served)), psnr_served_min=float(np.min(served)),
                psnr_net_mean=float(np.mean(pn)), psnr_net_min=float(np.min(pn)),
                psnr_net_max=float(np.max(pn)),
                psnr_bilinear_mean=float(np.mean(pb)), psnr_bilinear_min=float(np.min(pb)))


def _dump(path, rows):
    if path:
        import json
        with open(path, "w") as f:
            json.dump([{k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in r.items()}
                       for r in rows], f, indent=0, default=float)


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--weights", default=None)
    ap.add_argument("--sets", type=int, default=len(configs.C5_TRAIN_SEEDS))
    ap.add_argument("--cams", type=int, default=configs.C5_CAMS_PER_SET)
    ap.add_argument("--steps", type=int, default=30000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--crop", type=int, default=96)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--valid", type=int, default=len(configs.C5_VALID_SEEDS))
    ap.add_argument("--heldout", type=int, default=len(configs.C5_HELDOUT_SEEDS))
    ap.add_argument("--n", type=int, default=configs.C5_N)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--rows-out", default=None, help="write the per-frame rows as JSON")
    ap.add_argument("--low-sigma", default="fraction", choices=["pixel", "fraction"])
    ap.add_argument("--prefilter", type=float, default=0.75,
                    help="Gaussian prefilter sigma of the low-resolution render (its pixels)")
    ap.add_argument("--low-chi", type=float, default=0.0,
                    help="clip radius (sigmas) of the low-resolution render; 0: the frame's")
    ap.add_argument("--resume", default=None,
                    help="continue training from this checkpoint (weights, moments, step, sampler)")
    ap.add_argument("--checkpoint", default=None, help="checkpoint file written while training")
    ap.add_argument("--checkpoint-every", type=int, default=1000)
    a = ap.parse_args(argv)
    R = splotch.Renderer(0)
    cmap = torch.from_numpy(synth.ramp_colormap()).cuda()
    if a.cmd == "train":
        rng_state = None
        if a.resume:
            up = Upscaler.load(a.resume)
            up.lr = a.lr
            rng_state = checkpoint_rng_state(up)
            log(f"resuming {a.resume} at step {up.step}")
        else:
            up = Upscaler(seed=a.seed, lr=a.lr, low_sigma=a.low_sigma, prefilter=a.prefilter,
                          low_chi=a.low_chi)
        pairs = Pairs(R, cmap, list(configs.C5_TRAIN_SEEDS)[:a.sets], a.cams, n=a.n,
                      low_sigma=up.low_sigma, prefilter=up.prefilter, low_chi=up.low_chi)
        train(up, pairs, a.steps, a.batch, a.crop, a.lr, seed=a.seed, rng_state=rng_state,
              ckpt=a.checkpoint, ckpt_every=a.checkpoint_every)
        del pairs
        torch.cuda.empty_cache()
        vrows = evaluate(R, up, cmap, list(configs.C5_VALID_SEEDS)[:a.valid], n=a.n)
        theta = choose_theta(vrows)
        log(f"validation (no fallback): {summary(vrows)}; region theta {theta}")
        _dump(a.rows_out, vrows)
        if a.out:
            up.save(a.out, theta_region=theta, region=64, train_sets=a.sets, cams=a.cams,
                    steps=a.steps,
                    batch=a.batch, crop=a.crop, lr=a.lr, n=a.n)
            log(f"saved {a.out}")
    else:
        up = Upscaler.load(a.weights)
        theta = float(up.meta.get("theta_region", -math.inf))
        rows = evaluate(R, up, cmap, list(configs.C5_HELDOUT_SEEDS)[:a.heldout], theta=theta,
                        n=a.n)
        log(f"held-out: {summary(rows)}; theta {theta}")
        _dump(a.rows_out, rows)
    R.close()


if __name__ == "__main__":
    sys.exit(main())
