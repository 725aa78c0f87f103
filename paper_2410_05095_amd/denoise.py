"""Training data, training loop and evaluation of the soft-shadow denoiser.

The data are rendered by the library itself: for random views of training scenes, the 1-sample
area-light visibility (with its G-buffer features) and the 256-sample visibility of the same pixels
from an independent random stream.  Host code here only picks views and crops and schedules the
learning rate; rendering, feature packing, the network's forward/backward and Adam run in the
library's HIP kernels.
"""
from __future__ import annotations

import math
import time
from typing import List, Optional

import numpy as np

from . import _native as N
from . import scenegen as sg

STREAM_1SPP, STREAM_PLAIN, STREAM_REF = 0, 1, 2
NO_HIT = 0xFFFFFFFF


def scene_diagonal(scene: sg.Scene) -> float:
    lo = scene.positions.min(axis=0).astype(np.float64)
    hi = scene.positions.max(axis=0).astype(np.float64)
    return float(np.linalg.norm(hi - lo))


def orbit_views(rng: np.random.Generator, n: int, width: int, height: int, seed0: int = 0,
                center=(0.0, 8.0, 0.0)) -> List[sg.Camera]:
    """Cameras 24-34 m from the scene centre, 8-35 degrees above the horizon, within 120 degrees of -z."""
    cams = []
    for i in range(n):
        r = rng.uniform(24.0, 34.0)
        el = math.radians(rng.uniform(8.0, 35.0))
        az = math.radians(rng.uniform(-120.0, 120.0))
        eye = (center[0] + r * math.cos(el) * math.sin(az), center[1] + r * math.sin(el),
               center[2] - r * math.cos(el) * math.cos(az))
        tgt = (center[0] + rng.uniform(-3, 3), center[1] + rng.uniform(-3, 3), center[2] + rng.uniform(-3, 3))
        cams.append(sg.Camera(eye=eye, target=tgt, up=(0.0, 1.0, 0.0), vfov_deg=float(rng.uniform(40, 55)),
                              width=width, height=height, ssaa=1, seed=seed0 + i))
    return cams


def render_visibility(ctx: N.Context, gs: N.Scene, cam, rect, spp: int, stream: int, out: Optional[dict] = None,
                      shade: bool = True):
    """Camera rays and rect-light visibility (and, with `shade`, the shaded image) of one view."""
    return ctx.render(gs, cam, (), rect=rect, area_samples=spp, area_stream=stream, out=out, shade=shade)


class TrainingSet:
    """Crops of (features, 256-sample visibility target, primary-hit mask) resident on the GPU."""

    def __init__(self, feats, targets, masks):
        self.feats, self.targets, self.masks = feats, targets, masks

    def __len__(self):
        return int(self.feats.shape[0])


def make_training_set(ctx: N.Context, scenes, n_views: int, crops_per_view: int, crop: int,
                      width: int = 1920, height: int = 1080, ref_spp: int = 256, seed: int = 0,
                      log=None) -> TrainingSet:
    """scenes: list of (sg.Scene, N.Scene handle).  Views are spread over the scenes in turn."""
    torch = ctx.torch
    rng = np.random.default_rng(seed)
    cams = orbit_views(rng, n_views, width, height, seed0=1000 * (seed + 1))
    F, T, M = [], [], []
    t0 = time.perf_counter()
    for i, cam in enumerate(cams):
        sc, gs = scenes[i % len(scenes)]
        o1 = render_visibility(ctx, gs, cam, sc.rect_light, 1, STREAM_1SPP)
        feat = N.pack_features(ctx, gs, cam, o1, scene_diagonal(sc))
        ref = render_visibility(ctx, gs, cam, sc.rect_light, ref_spp, STREAM_REF)["visibility"].clone()
        mask = (o1["hit"][:, 0] != -1).reshape(height, width).float()
        for _ in range(crops_per_view):
            y0 = int(rng.integers(0, height - crop + 1)) & ~3
            x0 = int(rng.integers(0, width - crop + 1)) & ~3
            F.append(feat[y0:y0 + crop, x0:x0 + crop].contiguous())
            T.append(ref[y0:y0 + crop, x0:x0 + crop].contiguous())
            M.append(mask[y0:y0 + crop, x0:x0 + crop].contiguous())
        if log and (i + 1) % max(1, n_views // 4) == 0:
            log(f"[denoise] rendered {i + 1}/{n_views} training views ({time.perf_counter() - t0:.1f} s)")
    return TrainingSet(torch.stack(F), torch.stack(T), torch.stack(M))


def train(den: N.Denoiser, data: TrainingSet, steps: int, batch: int = 8, lr: float = 1e-3, seed: int = 0,
          log=None, log_every: int = 50, warmup: int = 0) -> List[float]:
    """Adam with a cosine learning-rate schedule from lr to lr / 20, after a linear ramp from lr / warmup over
    the first `warmup` steps; returns the loss of every step."""
    rng = np.random.default_rng(seed)
    losses = []
    n = len(data)
    torch = den.ctx.torch
    for s in range(steps):
        idx = torch.from_numpy(rng.choice(n, size=min(batch, n), replace=False)).to(data.feats.device)
        f = data.feats.index_select(0, idx).contiguous()
        t = data.targets.index_select(0, idx).contiguous()
        m = data.masks.index_select(0, idx).contiguous()
        cur = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * s / max(steps, 1))))
        if s < warmup:
            cur *= (s + 1) / warmup
        want = log is not None and (s % log_every == 0 or s == steps - 1)
        losses.append(den.train_step(f, t, m, cur, want_loss=want))
        if want:
            log(f"[denoise] step {s}/{steps} lr {cur:.2e} loss {losses[-1]:.5f}")
    return losses


def plain_frame(ctx: N.Context, gs: N.Scene, scene: sg.Scene, cam, spp: int, ref, mask, reps: int = 5) -> dict:
    """The plain path at `spp` light samples per pixel: shadow MSE against `ref` and the device frame time
    (camera rays, shadow rays, shading; median of reps)."""
    torch = ctx.torch
    out = {}
    render_visibility(ctx, gs, cam, scene.rect_light, spp, STREAM_PLAIN, out=out)
    mse = masked_mse(out["visibility"], ref, mask)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record()
        render_visibility(ctx, gs, cam, scene.rect_light, spp, STREAM_PLAIN, out=out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return {"spp": spp, "mse": mse, "frame_ms": float(np.median(ts))}


def masked_mse(a, b, mask) -> float:
    m = mask.double()
    return float(((a.double() - b.double()) ** 2 * m).sum() / m.sum().clamp(min=1.0))


def evaluate_views(ctx: N.Context, den: N.Denoiser, gs: N.Scene, scene: sg.Scene, cams, plain_spp: int = 64,
                   ref_spp: int = 256) -> dict:
    """Shadow MSE against the ref_spp reference on each of `cams` (held-out views of an evaluation scene):
    denoised 1 spp (BF16 network and its FP32 copy), raw 1 spp and plain plain_spp; per-view values and means."""
    torch = ctx.torch
    rect = scene.rect_light
    diag = scene_diagonal(scene)
    rows = []
    for cam in cams:
        H, W = cam.height, cam.width
        ref = render_visibility(ctx, gs, cam, rect, ref_spp, STREAM_REF)["visibility"].clone()
        o1 = render_visibility(ctx, gs, cam, rect, 1, STREAM_1SPP)
        mask = (o1["hit"][:, 0] != -1).reshape(H, W)
        feat = N.pack_features(ctx, gs, cam, o1, diag).unsqueeze(0)
        vden = den.infer(feat)[0]
        v32 = den.infer(feat, fp32=True)[0]
        vp = render_visibility(ctx, gs, cam, rect, plain_spp, STREAM_PLAIN)["visibility"]
        rows.append({"den": masked_mse(vden, ref, mask), "den_fp32": masked_mse(v32, ref, mask),
                     "raw": masked_mse(o1["visibility"], ref, mask), "plain": masked_mse(vp, ref, mask)})
    torch.cuda.synchronize()
    mean = {k: float(np.mean([r[k] for r in rows])) for k in rows[0]}
    return {"views": len(cams), "mse_denoised_1spp": mean["den"], "mse_denoised_1spp_fp32": mean["den_fp32"],
            "mse_raw_1spp": mean["raw"], f"mse_plain_{plain_spp}spp": mean["plain"],
            "per_view_denoised": [round(r["den"], 7) for r in rows],
            f"per_view_plain_{plain_spp}spp": [round(r["plain"], 7) for r in rows]}


def evaluate(ctx: N.Context, den: N.Denoiser, gs: N.Scene, scene: sg.Scene, cam, plain_spp: int = 64,
             ref_spp: int = 256, reps: int = 5) -> dict:
    """Shadow MSE against the 256-sample reference for: denoised 1 spp, raw 1 spp, plain plain_spp;
    and device frame times of the learned and the plain path (median of reps)."""
    torch = ctx.torch
    H, W = cam.height, cam.width
    rect = scene.rect_light
    diag = scene_diagonal(scene)
    ref = render_visibility(ctx, gs, cam, rect, ref_spp, STREAM_REF)["visibility"].clone()
    o1 = render_visibility(ctx, gs, cam, rect, 1, STREAM_1SPP)
    mask = (o1["hit"][:, 0] != -1).reshape(H, W)
    v1 = o1["visibility"].clone()
    feat = N.pack_features(ctx, gs, cam, o1, diag)
    vden = den.infer(feat.unsqueeze(0))[0]
    op = render_visibility(ctx, gs, cam, rect, plain_spp, STREAM_PLAIN)
    vplain = op["visibility"].clone()
    torch.cuda.synchronize()
    res = {"mse_denoised_1spp": masked_mse(vden, ref, mask), "mse_raw_1spp": masked_mse(v1, ref, mask),
           f"mse_plain_{plain_spp}spp": masked_mse(vplain, ref, mask), "pixels": int(mask.sum().item()),
           "mean_ref_visibility": float(ref[mask].mean().item())}
    # frame times on the stream the library runs on
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    learned, plain, den_ms = [], [], []
    o_l, o_p, vd = {}, {}, torch.empty((1, H, W), dtype=torch.float32, device=ref.device)
    for _ in range(reps + 1):
        ev[0].record()
        render_visibility(ctx, gs, cam, rect, 1, STREAM_1SPP, out=o_l, shade=False)   # shaded below, once
        ev[1].record()
        f = N.pack_features(ctx, gs, cam, o_l, diag, feat=feat)
        den.infer(f.unsqueeze(0), out=vd)
        ev[2].record()
        ctx.shade(gs, cam, o_l, rect=rect, visibility=vd)
        ev[3].record()
        render_visibility(ctx, gs, cam, rect, plain_spp, STREAM_PLAIN, out=o_p)
        ev[4].record()
        torch.cuda.synchronize()
        learned.append(ev[0].elapsed_time(ev[3]))
        den_ms.append(ev[1].elapsed_time(ev[2]))
        plain.append(ev[3].elapsed_time(ev[4]))
    res["frame_ms_learned"] = float(np.median(learned[1:]))
    res["denoiser_ms"] = float(np.median(den_ms[1:]))
    res[f"frame_ms_plain_{plain_spp}spp"] = float(np.median(plain[1:]))
    # the plain path at the sample count whose binomial MSE (MSE_1 / N) matches the denoised MSE
    n_eq = int(math.ceil(res["mse_raw_1spp"] / max(res["mse_denoised_1spp"], 1e-12)))
    res["plain_spp_equivalent"] = res["mse_raw_1spp"] / max(res["mse_denoised_1spp"], 1e-12)
    res["plain_at_equal_mse"] = plain_frame(ctx, gs, scene, cam, max(1, min(n_eq, 4096)), ref, mask, reps)
    return res
