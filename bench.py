"""Benchmark of the ray-cast rendering path on one MI355X.

One step = one frame of the whole path on a synthetic scene resident in HBM: camera rays
into the G-buffer, shadow rays, shading and resolve.  Default workload: ~7.3M triangles
(1500 seeded procedural instances) at 1920x1080, one primary ray per pixel and 64 shadow
rays per pixel towards a 1x1 m rectangular light (the plain soft-shadow path).
Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload big_7M|city_1M] [--spp 64]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s + 1080p frame ms at 7.3M tris; denoised 1spp vs 64spp at equal shadow MSE"
HBM_PEAK_GBS = 8000.0
NODE_BYTES, TRI_BYTES = 128, 48
# FP32 lane-operations of the traversal as written (selects not counted; an FMA is one operation, as it
# issues as one): per 4-wide node visit 4 x (6 FMA for the plane distances, 3 max with 0, 3 min with the
# bound, 1 compare) + 5 sorting compares = 57; per Moller-Trumbore test 2 cross products (6 mul, 6 FMA),
# 4 dot products (4 mul, 8 FMA), 3 sub, 1 reciprocal, 3 mul by it, 1 add and 5 compares for the hit
# conditions = 37.
NODE_OPS, TRI_OPS = 57, 37
# Issue peak of non-packed FP32 vector ops: 256 CUs x 64 lanes per clock x 2.4 GHz (the 157.3 TFLOP/s
# datasheet figure counts packed FMAs, i.e. 4 FLOP per lane and clock).
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# Bytes per launch of the dominant kernel measured with rocprofv3 FETCH_SIZE + WRITE_SIZE (scaled by
# the copy-kernel calibration), keyed by (workload, spp, hash of the traversal kernel sources); the
# value only applies while those sources are unchanged (summaries under profiles/).
MEASURED_TRAFFIC = {
    ("big_7M", 64, "ff787ee5bc0f2761:5ce1cb11be5fdbcb:70040863f1edf569"): 446_670_000,
}


def kernel_hash():
    import hashlib
    h = []
    for f in ("k_trace.hip", "rc_device.h", "rc_trav.h"):
        with open(os.path.join(ROOT, "paper_2410_05095_amd", "csrc", f), "rb") as fh:
            h.append(hashlib.sha256(fh.read()).hexdigest()[:16])
    return ":".join(h)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(scene, cam, args, budget_s=12.0):
    """The FP64 oracle as it stands, on a bounded random sample of the same frame's pixels."""
    import numpy as np

    from oracle import oracle as O
    t0 = time.perf_counter()
    osc = O.OracleScene.from_scene(scene)
    build_s = time.perf_counter() - t0
    rng = np.random.default_rng(123)
    npix = cam.width * cam.height
    threads = O.n_threads()

    def run(n):
        pix = np.sort(rng.choice(npix, n, replace=False))
        t = time.perf_counter()
        if args.workload == "big_7M":
            r = osc.render_rect(cam, scene.rect_light, args.spp, 0, pix, threads=threads)
            rays = n + int(r["cast_count"].sum())
        else:
            spp = cam.ssaa ** 2
            smp = (pix[:, None] * spp + np.arange(spp)[None, :]).ravel()
            r = osc.render_point(cam, scene.point_lights, smp, threads=threads)
            rays = len(smp) + int(sum(bin(int(m)).count("1") for m in r["mask"]))  # lit shadow rays only: a lower bound
        return rays, time.perf_counter() - t

    rays, dt = run(500)
    n = int(min(npix, max(500, 500 * budget_s / max(dt, 1e-3))))
    rays, dt = run(n)
    return {"value": rays / dt / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} random pixels of the same frame ({rays} rays, {dt:.1f} s); oracle BVH build "
                      f"{build_s:.1f} s not included"}


def learned_path(ctx, gs, scene, cam, args):
    """Train the denoiser on the method's own 1/256-sample renders of other scene seeds, then compare
    on this frame: shadow MSE against 256 samples and device frame time, learned 1 spp vs plain."""
    import torch

    from paper_2410_05095_amd import _native as N
    from paper_2410_05095_amd import denoise as D
    from paper_2410_05095_amd import scenegen as sg
    t0 = time.perf_counter()
    train_scenes = []
    for seed in range(args.seed + 1, args.seed + 1 + args.denoiser_scenes):
        sc = sg.big_scene(seed)
        train_scenes.append((sc, ctx.scene_from(sc).build()))
    log(f"[bench] training scenes ready ({time.perf_counter() - t0:.1f} s)")
    data = D.make_training_set(ctx, train_scenes, n_views=args.denoiser_views, crops_per_view=12, crop=256,
                               seed=args.seed, log=log)
    n_crops = len(data)
    for _, h in train_scenes:
        h.close()
    den = N.Denoiser(ctx, seed=args.seed)
    t1 = time.perf_counter()
    losses = D.train(den, data, steps=args.denoiser_steps, batch=8, lr=2e-3, seed=args.seed, log=log, log_every=300)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    del data
    ev = D.evaluate(ctx, den, gs, scene, cam, plain_spp=args.spp, ref_spp=256, reps=5)
    if args.anim_frames > 0:
        ev["animated"] = animated(ctx, gs, scene, den, args)
    ev.update({"train_steps": args.denoiser_steps, "train_s": round(train_s, 1), "train_crops": n_crops,
               "crop": 256, "final_loss": [x for x in losses if x == x][-1],
               "weights": "bf16 (FP32 master)", "parity": "unpinned (statistical)"})
    rnd = lambda v: round(v, 6) if isinstance(v, float) else v
    return {k: ({a: rnd(b) for a, b in v.items()} if isinstance(v, dict) else rnd(v)) for k, v in ev.items()}


def post_pass(ctx, out, args):
    """The display post pass (tone map + sRGB8, FXAA) on the benchmark frame: device time per frame, and the
    bytes each kernel moves at minimum (tone map: 16 B in + 4 B out per pixel; FXAA: 4 B in + 4 B out)."""
    import numpy as np
    import torch
    rgba = out["rgba"]
    H, W = int(rgba.shape[0]), int(rgba.shape[1])
    img = torch.empty((H, W, 4), dtype=torch.uint8, device=rgba.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for aa in (False, True):
        for _ in range(args.warmup):
            ctx.postprocess(rgba, fxaa=aa, out=img)
        ts = []
        for _ in range(max(args.steps, 5)):
            e0.record()
            ctx.postprocess(rgba, fxaa=aa, out=img)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        res["tonemap_fxaa_ms" if aa else "tonemap_ms"] = round(float(np.median(ts)), 4)
    n = H * W
    res["min_bytes"] = {"tonemap": 20 * n, "fxaa": 8 * n}
    res["achieved_GBps_tonemap"] = round(20 * n / (res["tonemap_ms"] * 1e-3) / 1e9, 1)
    return res


def hard_shadows(ctx, gs, scene, cam, args):
    """The configuration the paper times (Sec. V): one camera ray and one hard-shadow ray per pixel, one point
    light (placed at the rect light's centre, intensity 400), 1920x1080, the 7.3M-triangle scene.  Device
    time of the whole frame (camera rays, shadow rays, shading), median of args.steps frames."""
    import numpy as np
    import torch
    c = scene.rect_light.center
    light = np.array([[c[0], c[1], c[2], 400.0, 400.0, 400.0]], np.float32)
    out = {}
    for _ in range(args.warmup):
        ctx.render(gs, cam, light, out=out, timing=True)
    frames = []
    for _ in range(args.steps):
        ctx.render(gs, cam, light, out=out, timing=True)
        frames.append(ctx.stage_times())
    torch.cuda.synchronize()
    assert ctx.last_error() == 0
    med = lambda k: round(float(np.median([f[k] for f in frames])), 4)
    rays = frames[-1]["primary_rays"] + frames[-1]["shadow_rays"]
    return {"frame_ms": med("total_ms"), "primary_ms": med("primary_ms"), "shadow_ms": med("shadow_ms"),
            "rays_per_frame": int(rays), "mrays_per_s": round(rays / med("total_ms") / 1e3, 1),
            "paper_context": "paper: >7M triangles within 2 ms of GPU time per frame on an RTX 4090 "
                             "(raster + hardware ray queries; resolution not stated)"}


def device_build(ctx, scene, cam, kw, args):
    """The GPU LBVH build of the same scene (positions already in HBM): build time (median of 3, from the
    first kernel to the finished tree, allocation included), tree size and SAH cost, and the frame's
    device time rendered through that tree (median of args.steps frames)."""
    import numpy as np
    gs = ctx.scene_from(scene)
    ms = []
    for _ in range(3):
        gs.build(device=True)
        ms.append(gs.stats()["build_ms"])
    st = gs.stats()
    out = {}
    for _ in range(args.warmup):
        ctx.render(gs, cam, out=out, timing=True, **kw)
    frames = []
    for _ in range(args.steps):
        ctx.render(gs, cam, out=out, timing=True, **kw)
        frames.append(ctx.stage_times())
    assert ctx.last_error() == 0
    gs.close()
    med = lambda k: round(float(np.median([f[k] for f in frames])), 4)
    return {"build_ms": round(float(np.median(ms)), 2), "nodes": int(st["n_nodes"]), "depth": int(st["depth"]),
            "sah": round(st["sah_cost"], 2), "frame_device_ms": med("total_ms"), "shadow_ms": med("shadow_ms"),
            "primary_ms": med("primary_ms")}


def watertight_frames(ctx, scene, cam, kw, args):
    """The same frames with every ray/triangle test watertight (RC_BUILD_WATERTIGHT, host binned-SAH tree of
    the same scene): device time of the 64-sample frame and of the hard-shadow frame, medians of args.steps."""
    import numpy as np
    gs = ctx.scene_from(scene).build(watertight=True)
    c = scene.rect_light.center
    hard = dict(lights=np.array([[c[0], c[1], c[2], 400.0, 400.0, 400.0]], np.float32))
    res = {}
    for name, k in (("soft", kw), ("hard", hard)):
        out = {}
        for _ in range(args.warmup):
            ctx.render(gs, cam, out=out, timing=True, **k)
        frames = []
        for _ in range(args.steps):
            ctx.render(gs, cam, out=out, timing=True, **k)
            frames.append(ctx.stage_times())
        med = lambda key: round(float(np.median([f[key] for f in frames])), 4)
        res[name] = {"frame_device_ms": med("total_ms"), "shadow_ms": med("shadow_ms"), "primary_ms": med("primary_ms")}
    assert ctx.last_error() == 0
    gs.close()
    return res


def dynamic_structures(ctx, gs_flat, scene, cam, args):
    """Moving bodies with the paper's structure choice (Sec. IV-B, "Ray-traced shadows"): a top level over
    per-body trees rebuilt every frame on an asynchronous queue, against updating (refitting) one flat BVH.
    300 of the 1501 bodies move (<= 5 cm, <= 2 degrees per frame, the same motion as the animated frames).
    Per frame: move the bodies, update the structure, render the paper's timed configuration (one camera ray
    and one hard-shadow ray per pixel, 1080p) or the 64-sample soft-shadow frame.  Device time per frame,
    mean over the frames after a warm-up frame; node visits and triangle tests per ray of the last frame.
    Paths: flat BVH + refit; two-level + top-level rebuild in line; two-level with the rebuild of frame f+1
    on a second stream beside the render of frame f (two scene copies, alternating)."""
    import numpy as np
    import torch

    from paper_2410_05095_amd import scenegen as sg
    c = scene.rect_light.center
    hard = dict(lights=np.array([[c[0], c[1], c[2], 400.0, 400.0, 400.0]], np.float32))
    soft = dict(lights=(), rect=scene.rect_light, area_samples=args.spp, area_stream=0)
    anim = sg.RigidAnimation(scene, n_bodies=300, seed=args.seed)
    F = args.dyn_frames
    xfs = [torch.from_numpy(anim.transforms(f)).cuda() for f in range(1, F + 2)]
    ids = torch.from_numpy(anim.body_ids.astype(np.int32)).cuda()
    rest = torch.eye(3, 4, dtype=torch.float32).repeat(len(anim.body_ids), 1, 1).reshape(-1, 12).cuda()
    main = torch.cuda.current_stream()
    res = {}

    def per_ray(st):
        return {"primary_nodes": round(st["primary_nodes"] / max(st["primary_rays"], 1), 2),
                "shadow_nodes": round(st["shadow_nodes"] / max(st["shadow_rays"], 1), 2),
                "shadow_tris": round(st["shadow_tris"] / max(st["shadow_rays"], 1), 2)}

    def inline(g, kw, update):
        g.set_transforms(rest, ids)
        update(g)
        out = {}
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        upd, tot = [], []
        for f in range(F):
            ev[0].record(main)
            g.set_transforms(xfs[f], ids)
            update(g)
            ev[1].record(main)
            ctx.render(g, cam, out=out, **kw)
            ev[2].record(main)
            torch.cuda.synchronize()
            if f > 0:
                upd.append(ev[0].elapsed_time(ev[1]))
                tot.append(ev[0].elapsed_time(ev[2]))
        ctx.render(g, cam, out=out, timing=True, **kw)
        st = ctx.stage_times()
        assert ctx.last_error() == 0
        return {"update_ms": round(float(np.mean(upd)), 4), "frame_ms": round(float(np.mean(tot)), 4), **per_ray(st)}

    def overlapped(pair, kw):
        side = torch.cuda.Stream()
        for g in pair:
            g.set_transforms(rest, ids)
            g.tlas_rebuild()
        pair[0].set_transforms(xfs[0], ids)
        pair[0].tlas_rebuild()
        torch.cuda.synchronize()
        out = {}
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for f in range(F):
            if f == 1:
                e0.record(main)
            cur, nxt = pair[f % 2], pair[(f + 1) % 2]
            side.wait_stream(main)              # nxt's previous render is done before it moves
            with torch.cuda.stream(side):
                nxt.set_transforms(xfs[f + 1], ids)
                nxt.tlas_rebuild(stream=side)
            ctx.render(cur, cam, out=out, **kw)
            main.wait_stream(side)              # the next frame renders nxt
        e1.record(main)
        torch.cuda.synchronize()
        assert ctx.last_error() == 0
        return {"frame_ms": round(e0.elapsed_time(e1) / (F - 1), 4)}

    refit = lambda g: g.refit()
    rebuild = lambda g: g.tlas_rebuild()
    two = ctx.scene_from(scene).build(two_level=True)
    two_b = ctx.scene_from(scene).build(two_level=True)
    tst = two.stats()
    for name, kw in (("hard_1080p", hard), ("soft_64spp", soft)):
        r = {"flat_refit": inline(gs_flat, kw, refit), "two_level_rebuild": inline(two, kw, rebuild),
             "two_level_rebuild_async": overlapped((two, two_b), kw)}
        res[name] = r
        log(f"[bench] dynamic structures {name}: {r}")
    gs_flat.set_transforms(rest, ids)
    gs_flat.refit()
    torch.cuda.synchronize()
    two.close()
    two_b.close()
    res["two_level_build_ms"] = round(tst["build_ms"], 2)
    res["tlas_levels"] = int(tst["tlas_levels"])
    res["bodies"] = int(tst["n_instances"])
    res["moving_bodies"] = int(len(anim.body_ids))
    res["frames"] = F
    return res


def animated(ctx, gs, scene, den, args):
    """The same scene with 300 rigid bodies moving (<= 5 cm, <= 2 degrees per frame), BVH refit every frame,
    args.anim_views 1080p views per frame on the learned 1-spp path; per-frame shadow MSE of the BF16
    denoiser and of its FP32 copy against 256 samples, for view f mod V of frame f and for every view of the
    first and last frame."""
    import numpy as np

    from paper_2410_05095_amd import animate as A
    from paper_2410_05095_amd import denoise as D
    from paper_2410_05095_amd import scenegen as sg
    anim = sg.RigidAnimation(scene, n_bodies=300, seed=args.seed)
    views = D.orbit_views(np.random.default_rng(args.seed + 77), args.anim_views, 1920, 1080, seed0=5000)
    F, V = args.anim_frames, args.anim_views
    plan = lambda f: list(range(V)) if f in (0, F - 1) else [f % V]
    res = A.run(ctx, scene, gs, den, anim, views, F, plan, log=log)
    rnd = lambda v: round(v, 6) if isinstance(v, float) else v
    return {k: rnd(v) for k, v in res.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="big_7M", choices=["big_7M", "city_1M"])
    ap.add_argument("--spp", type=int, default=64, help="rect-light samples per pixel (big_7M)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--denoiser-steps", type=int, default=12000,
                    help="training steps of the learned 1-spp path (0 = skip the learned-path comparison)")
    ap.add_argument("--denoiser-scenes", type=int, default=4,
                    help="training scenes (seeds after the evaluation seed) of the denoiser's training set")
    ap.add_argument("--denoiser-views", type=int, default=400,
                    help="1080p views of the training scenes rendered for the denoiser's training set (12 crops each)")
    ap.add_argument("--anim-frames", type=int, default=12,
                    help="animated frames (moving bodies, refit) rendered after the learned-path comparison")
    ap.add_argument("--anim-views", type=int, default=16, help="1080p views per animated frame")
    ap.add_argument("--dyn-frames", type=int, default=24,
                    help="frames of the moving-body comparison of flat refit and two-level rebuild (0 = skip)")
    ap.add_argument("--profile-denoiser", type=int, default=0,
                    help="instead of rendering, run this many BF16 denoiser inferences of one 1080p view (twice: "
                         "warm-up, timed) and one FP32-copy inference")
    ap.add_argument("--build-only", type=int, default=0,
                    help="instead of rendering, build the scene's BVH on the GPU this many times (for profilers)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="instead of rendering, copy a buffer of this many MiB 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (views or tiles would be split "
              "across GPUs with a final image gather; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_mib:
        a = torch.ones(args.copy_mib * (1 << 18), dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": a.numel() * 4, "copy_bytes_written_per_launch": b.numel() * 4,
                          "launches": 5}), flush=True)
        return

    from paper_2410_05095_amd import _native as N
    from paper_2410_05095_amd import scenegen as sg

    if args.profile_denoiser:
        # the denoiser alone (for profilers): BF16 inference of a 1920x1080 view, then the FP32 copy
        ctx = N.Context(0)
        den = N.Denoiser(ctx, seed=args.seed)
        g = torch.Generator(device="cuda").manual_seed(args.seed)
        feat = torch.rand((1, 1080, 1920, 8), device="cuda", generator=g).to(torch.bfloat16).contiguous()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        for _ in range(args.profile_denoiser):
            den.infer(feat)
        ev[0].record()
        for _ in range(args.profile_denoiser):
            den.infer(feat)
        ev[1].record()
        den.infer(feat, fp32=True)
        ev[2].record()
        torch.cuda.synchronize()
        print(json.dumps({"denoiser_bf16_ms": ev[0].elapsed_time(ev[1]) / args.profile_denoiser,
                          "denoiser_fp32_ms": ev[1].elapsed_time(ev[2]), "width": 1920, "height": 1080}), flush=True)
        return

    t0 = time.perf_counter()
    scene = sg.big_scene(args.seed) if args.workload == "big_7M" else sg.city_scene(args.seed)
    cam = scene.cameras[0]
    log(f"[bench] scene {scene.name}: {scene.n_tris} tris, generated in {time.perf_counter() - t0:.1f} s")
    ctx = N.Context(0)
    if args.build_only:
        gs = ctx.scene_from(scene)
        ms = []
        for _ in range(args.build_only):
            gs.build(device=True)
            ms.append(gs.stats()["build_ms"])
        print(json.dumps({"device_build_ms": ms, "tris": scene.n_tris, **gs.stats()}), flush=True)
        return
    gs = ctx.scene_from(scene).build()
    bst = gs.stats()
    log(f"[bench] BVH: {bst}")

    if args.workload == "big_7M":
        kw = dict(lights=(), rect=scene.rect_light, area_samples=args.spp, area_stream=0)
    else:
        kw = dict(lights=scene.point_lights)
    out = {}
    for i in range(args.warmup):
        ctx.render(gs, cam, out=out, timing=True, **kw)
    torch.cuda.synchronize()
    assert ctx.last_error() == 0
    log(f"[bench] warmup done")

    stages = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ctx.render(gs, cam, out=out, timing=True, **kw)
        stages.append(ctx.stage_times())   # synchronises the stream after each frame
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert ctx.last_error() == 0
    ms_step = wall * 1000.0 / args.steps
    st = {k: float(np.mean([s[k] for s in stages])) for k in stages[0]}
    rays = st["primary_rays"] + st["shadow_rays"]
    value = rays / (ms_step / 1000.0) / 1e6
    # roofline of the dominant kernel (shadow traversal).  Its lanes mostly fetch the same nodes (the
    # light samples of one pixel share a wave), so the caches serve nearly all node and triangle bytes and
    # the measured fabric traffic is far below HBM bandwidth: the bound is instruction issue, reported as
    # FP32 arithmetic per launch (counted node visits and triangle tests) against the FP32 issue peak.
    npix = cam.width * cam.height * cam.ssaa ** 2
    dom_ms = st["shadow_ms"]
    dom_ops = st["shadow_nodes"] * NODE_OPS + st["shadow_tris"] * TRI_OPS
    achieved = dom_ops / (dom_ms / 1000.0) / 1e12
    logical_bytes = st["shadow_nodes"] * NODE_BYTES + st["shadow_tris"] * TRI_BYTES + npix * 20
    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"{scene.name}: {scene.n_tris} FP32 triangles, {cam.width}x{cam.height}, "
                                + (f"1 primary ray/pixel, rect light {args.spp} shadow rays/pixel"
                                   if args.workload == "big_7M" else
                                   f"{cam.ssaa ** 2} samples/pixel, {len(scene.point_lights)} point lights")),
                   "tris": scene.n_tris, "width": cam.width, "height": cam.height},
        "frame_ms": round(ms_step, 4),
        "stages_ms": {"primary": round(st["primary_ms"], 4), "shadow": round(st["shadow_ms"], 4),
                      "shade_resolve": round(st["shade_ms"], 4), "render_device": round(st["total_ms"], 4)},
        "rays_per_frame": {"primary": int(st["primary_rays"]), "shadow": int(st["shadow_rays"])},
        "mrays_per_s_kernel": {"primary": round(st["primary_rays"] / st["primary_ms"] / 1e3, 1),
                               "shadow": round(st["shadow_rays"] / st["shadow_ms"] / 1e3, 1)},
        "per_ray": {"primary_nodes": round(st["primary_nodes"] / max(st["primary_rays"], 1), 2),
                    "primary_tris": round(st["primary_tris"] / max(st["primary_rays"], 1), 2),
                    "shadow_nodes": round(st["shadow_nodes"] / max(st["shadow_rays"], 1), 2),
                    "shadow_tris": round(st["shadow_tris"] / max(st["shadow_rays"], 1), 2)},
        "bvh": {"build_ms": round(bst["build_ms"], 1), "nodes": int(bst["n_nodes"]), "depth": int(bst["depth"]),
                "sah": round(bst["sah_cost"], 2)},
        "roofline": ({"kernel": "k_rect_wave", "bound": "alu", "achieved": round(achieved, 3),
                      "peak": round(ALU_PEAK_TOPS, 2), "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TOPS, 4),
                      "traffic": MEASURED_TRAFFIC.get((args.workload, args.spp, kernel_hash())),
                      "logical_node_tri_GBps": round(logical_bytes / (dom_ms / 1000.0) / 1e9, 1)}
                     if args.workload == "big_7M" else
                     {"kernel": "k_trace<point>", "bound": "alu", "achieved": round(achieved, 3),
                      "peak": round(ALU_PEAK_TOPS, 2), "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TOPS, 4),
                      "traffic": None,
                      "logical_node_tri_GBps": round(logical_bytes / (dom_ms / 1000.0) / 1e9, 1)}),
    }
    res["post"] = post_pass(ctx, out, args)
    res["device_bvh"] = device_build(ctx, scene, cam, kw, args)
    if args.workload == "big_7M":
        res["watertight"] = watertight_frames(ctx, scene, cam, kw, args)
    if args.workload == "big_7M" and args.dyn_frames > 1:
        res["dynamic_structures"] = dynamic_structures(ctx, gs, scene, cam, args)
    if args.workload == "big_7M":
        res["hard_shadows"] = hard_shadows(ctx, gs, scene, cam, args)
    if args.workload == "big_7M" and args.denoiser_steps > 0:
        res["denoiser"] = learned_path(ctx, gs, scene, cam, args)
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        res["cpu_baseline"] = cpu_baseline(scene, cam, args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
