"""Animated frames: rigid bodies moved every frame, the BVH refit (not rebuilt), many views per frame
rendered by the learned 1-spp path, the BF16 denoiser compared with its FP32 copy, and per-frame shadow
MSE against the 256-sample visibility.

Host code here only schedules: the motion, refit, rendering, feature packing, both network evaluations
and shading run in the library's HIP kernels.
"""
from __future__ import annotations

from dataclasses import replace
from typing import Callable, List, Optional

import numpy as np

from . import _native as N
from . import denoise as D
from . import scenegen as sg


def run(ctx: N.Context, scene: sg.Scene, gs: N.Scene, den: N.Denoiser, anim: sg.RigidAnimation,
        views: List[sg.Camera], n_frames: int, ref_views: Callable[[int], List[int]],
        log: Optional[Callable] = None, lanes: int = 3) -> dict:
    """Render n_frames frames.  Frame f >= 1 first applies anim.transforms(f) and refits the BVH; then every
    view renders its 1-spp visibility and features (Philox frame index f), is denoised in BF16 and shaded.
    That part is timed with device events.  Untimed, for the views in ref_views(f): the FP32 copy of the
    network on the same features and the 256-sample reference, giving the shadow MSE of BF16, FP32 and
    raw 1-spp visibility over pixels with a primary hit.

    The views are dealt over `lanes` streams, each with a context and a copy of the network of its own (the
    work buffers of a context or a network serve one launch sequence at a time), so that the traversal of one
    view, bound by dependent node loads, runs beside the denoiser of another.  Every view's result is the one
    it has with one stream.  16 views of 1080p on 7.3M triangles: 36.3 ms per frame on one stream, 30.5 ms on
    two, 29.0 ms on three."""
    torch = ctx.torch
    rect = scene.rect_light
    diag = D.scene_diagonal(scene)
    dev = torch.device("cuda", ctx.device)
    lanes = max(1, min(int(lanes), len(views)))
    main = torch.cuda.current_stream(dev)
    streams = [main] + [torch.cuda.Stream(dev) for _ in range(lanes - 1)]
    ctxs, dens = [ctx], [den]
    for i in range(1, lanes):
        with torch.cuda.stream(streams[i]):
            ctxs.append(N.Context(ctx.device))
            dens.append(N.Denoiser(ctxs[i], seed=0))
            dens[i].set_params(den.params())
    outs = [dict() for _ in views]
    feats: List = [None] * len(views)
    y16 = [torch.empty((1, c.height, c.width), dtype=torch.float32, device=dev) for c in views]
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    ready = torch.cuda.Event()
    done = [torch.cuda.Event() for _ in streams]
    ids = torch.from_numpy(anim.body_ids.astype(np.int32)).to(dev)
    records = []
    for f in range(n_frames):
        cams = [replace(c, frame=f) for c in views]
        xf = torch.from_numpy(anim.transforms(f)).to(dev) if f > 0 else None
        torch.cuda.synchronize()
        e0.record()
        if xf is not None:
            gs.set_transforms(xf, ids)
            gs.refit()
        e1.record()
        ready.record(main)
        for i in range(lanes):
            with torch.cuda.stream(streams[i]):
                streams[i].wait_event(ready)
                c, d = ctxs[i], dens[i]
                for v in range(i, len(cams), lanes):
                    cam = cams[v]
                    D.render_visibility(c, gs, cam, rect, 1, D.STREAM_1SPP, out=outs[v], shade=False)
                    feats[v] = N.pack_features(c, gs, cam, outs[v], diag, feat=feats[v])
                    d.infer(feats[v].unsqueeze(0), out=y16[v])
                    c.shade(gs, cam, outs[v], rect=rect, visibility=y16[v][0])
                done[i].record(streams[i])
        for i in range(1, lanes):
            main.wait_event(done[i])
        e2.record()
        torch.cuda.synchronize()
        rec = {"frame": f, "refit_ms": e0.elapsed_time(e1), "views_ms": e1.elapsed_time(e2), "views": []}
        for v in ref_views(f):
            cam = cams[v]
            y32 = den.infer(feats[v].unsqueeze(0), fp32=True)[0]
            ref = D.render_visibility(ctx, gs, cam, rect, 256, D.STREAM_REF)["visibility"]
            mask = (outs[v]["hit"][:, 0] != -1).reshape(cam.height, cam.width)
            rec["views"].append({
                "view": v,
                "mse_bf16": D.masked_mse(y16[v][0], ref, mask),
                "mse_fp32": D.masked_mse(y32, ref, mask),
                "mse_raw_1spp": D.masked_mse(outs[v]["visibility"], ref, mask),
                "max_abs_bf16_fp32": float((y16[v][0] - y32).abs().max().item()),
            })
        records.append(rec)
        if log:
            m = rec["views"]
            log(f"[anim] frame {f}: refit {rec['refit_ms']:.3f} ms, {len(views)} views {rec['views_ms']:.2f} ms"
                + (f", MSE bf16 {np.mean([x['mse_bf16'] for x in m]):.6f} fp32 "
                   f"{np.mean([x['mse_fp32'] for x in m]):.6f}" if m else ""))
    torch.cuda.synchronize()
    for c in ctxs:
        assert c.last_error() == 0
    for i in range(1, lanes):
        dens[i].close()
        ctxs[i].close()
    allv = [x for r in records for x in r["views"]]
    moved = [r for r in records if r["frame"] > 0]
    return {
        "frames": n_frames, "views": len(views), "bodies": int(len(anim.body_ids)), "streams": lanes,
        "width": int(views[0].width), "height": int(views[0].height),
        "refit_ms_median": float(np.median([r["refit_ms"] for r in moved])) if moved else 0.0,
        "views_ms_median": float(np.median([r["views_ms"] for r in records])),
        "frame_ms_median": float(np.median([r["refit_ms"] + r["views_ms"] for r in records])),
        "mse_bf16_mean": float(np.mean([x["mse_bf16"] for x in allv])) if allv else None,
        "mse_fp32_mean": float(np.mean([x["mse_fp32"] for x in allv])) if allv else None,
        "mse_raw_1spp_mean": float(np.mean([x["mse_raw_1spp"] for x in allv])) if allv else None,
        "max_abs_bf16_fp32": float(max(x["max_abs_bf16_fp32"] for x in allv)) if allv else None,
        "reference_views": len(allv),
        "per_frame_mse_bf16": [round(float(np.mean([x["mse_bf16"] for x in r["views"]])), 6) for r in records],
        "per_frame_mse_fp32": [round(float(np.mean([x["mse_fp32"] for x in r["views"]])), 6) for r in records],
        "per_frame_refit_ms": [round(r["refit_ms"], 4) for r in records],
        "per_frame": [{"frame": r["frame"], "refit_ms": round(r["refit_ms"], 4), "views_ms": round(r["views_ms"], 3),
                       "mse_bf16": [round(x["mse_bf16"], 6) for x in r["views"]],
                       "mse_fp32": [round(x["mse_fp32"], 6) for x in r["views"]]} for r in records],
    }
