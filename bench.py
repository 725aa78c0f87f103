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
# Per-lane (vector) part of a node visit: the 5 sorting compares run on wave-uniform keys in scalar
# instructions in the wave kernel, so the algorithmic vector work of a node visit is 4 x 13 = 52.
NODE_VOPS = 52
# Issue peak of non-packed FP32 vector ops: 256 CUs x 64 lanes per clock x 2.4 GHz (the 157.3 TFLOP/s
# datasheet figure counts packed FMAs, i.e. 4 FLOP per lane and clock).
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# Bytes per launch of the dominant kernel measured with rocprofv3 FETCH_SIZE + WRITE_SIZE (scaled by
# the copy-kernel calibration), keyed by (workload, spp, hash of the traversal kernel sources); the
# value only applies while those sources are unchanged (summaries under profiles/).
MEASURED_TRAFFIC = {
    ("big_7M", 64, "7d238b039053ec4a:5ce1cb11be5fdbcb:619146c7bd55091c"): 442_900_000,
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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(scene, cam, args):
    """The FP64 oracle as it stands, on the host cores (one thread per core), median of 3 runs per workload:
    bounded random pixel samples of the benchmark frame at 1, args.spp and 256 rect-light samples per pixel,
    the 12+1280-triangle box frame whole, a sample of the 1.1M-triangle 4-light 2x2-supersampled frame, and a
    sample of the 64 batched views.  Rays counted: camera rays plus the shadow rays the oracle casts (point
    lights: those it casts, i.e. with the light above the surface).  Scene generation and the oracle's BVH
    builds are timed separately."""
    import numpy as np

    from oracle import oracle as O
    from paper_2410_05095_amd import scenegen as sg
    threads = O.n_threads()
    rng = np.random.default_rng(123)

    def rect_run(osc, sc, c, spp, n):
        pix = np.sort(rng.choice(c.width * c.height, n, replace=False))
        t = time.perf_counter()
        r = osc.render_rect(c, sc.rect_light, spp, 0, pix, threads=threads)
        return n + int(r["cast_count"].sum()), time.perf_counter() - t

    def point_run(osc, sc, c, n):
        npix = c.width * c.height
        pix = np.sort(rng.choice(npix, min(n, npix), replace=False))
        spp = c.ssaa ** 2
        smp = (pix[:, None] * spp + np.arange(spp)[None, :]).ravel()
        t = time.perf_counter()
        r = osc.render_point(c, sc.point_lights, smp, threads=threads)
        dt = time.perf_counter() - t
        cast = int(np.unpackbits(r["cast"].view(np.uint8)).sum())
        return len(smp) + cast, dt

    def median3(fn, calib, target_s):
        rays, dt = fn(calib)
        n = int(max(calib, calib * target_s / max(dt, 1e-3)))
        runs = [fn(n) for _ in range(3)]
        rates = sorted(r / t / 1e6 for r, t in runs)
        return {"mrays_per_s": round(rates[1], 3), "runs_mrays_per_s": [round(x, 3) for x in rates],
                "pixels_per_run": n, "rays_per_run": int(np.median([r for r, _ in runs])),
                "s_per_run": round(float(np.median([t for _, t in runs])), 2)}

    res = {}
    t0 = time.perf_counter()
    osc = O.OracleScene.from_scene(scene)
    build7 = time.perf_counter() - t0
    head = median3(lambda n: rect_run(osc, scene, cam, args.spp, n), 400, 4.0)
    res[f"big_7M_{args.spp}spp"] = head
    res["big_7M_1spp"] = median3(lambda n: rect_run(osc, scene, cam, 1, n), 4000, 1.0)
    res["big_7M_256spp"] = median3(lambda n: rect_run(osc, scene, cam, 256, n), 100, 3.0)
    del osc
    tiny = sg.tiny_box_scene(0)
    tosc = O.OracleScene.from_scene(tiny)
    tc = tiny.cameras[0]
    res["tiny_box_full_frame"] = median3(lambda n: point_run(tosc, tiny, tc, n), tc.width * tc.height, 0.0)
    t1 = time.perf_counter()
    city = sg.city_scene(args.seed)
    cosc = O.OracleScene.from_scene(city)
    city_build = time.perf_counter() - t1
    res["city_1M_4spp_4lights"] = median3(lambda n: point_run(cosc, city, city.cameras[0], n), 2000, 2.0)
    del cosc, city
    t2 = time.perf_counter()
    bscenes, bcams = sg.batch_scenes(args.seed)
    boscs = [O.OracleScene.from_scene(b) for b in bscenes]
    batch_build = time.perf_counter() - t2

    def batch_run(n):
        # n pixels spread evenly over the 64 views; the views run concurrently, one host thread each
        from concurrent.futures import ThreadPoolExecutor
        per = max(1, n // len(bcams))
        jobs = []
        for i, c in enumerate(bcams):
            pix = np.sort(rng.choice(c.width * c.height, min(per, c.width * c.height), replace=False))
            jobs.append((boscs[i % 4], bscenes[i % 4], c, pix))

        def one(j):
            osc_, sc_, c_, pix = j
            r = osc_.render_point(c_, sc_.point_lights, pix, threads=1)
            return len(pix) + int(np.unpackbits(r["cast"].view(np.uint8)).sum())

        t = time.perf_counter()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            rays = sum(ex.map(one, jobs))
        return rays, time.perf_counter() - t

    res["batch_64_views"] = median3(batch_run, 64 * 500, 2.0)
    return {"value": head["mrays_per_s"], "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "model": cpu_model(), "runs": 3, "statistic": "median of 3 runs",
            "sample": (f"{head['pixels_per_run']} random pixels of the benchmark frame per run "
                       f"({head['rays_per_run']} rays, {head['s_per_run']} s); oracle BVH builds not included "
                       f"(7.3M: {build7:.1f} s, city: {city_build:.1f} s with scene generation, batch scenes: "
                       f"{batch_build:.1f} s with generation)"),
            "configs": res}


def learned_path(ctx, gs, scene, cam, args):
    """Train the denoiser on the method's own 1/256-sample renders of other scene seeds (2000 crops of 512x512
    from 200 1080p views by default: 50 views of each of 4 seeds, 10 crops each), then compare on the
    evaluation scene: shadow MSE against 256 samples on the benchmark view and on 8 held-out views, and
    device frame times of the learned 1-spp path and of the plain path (64 spp, and the sample count of
    equal MSE).  `target_met`: denoised 1 spp at or below the plain 64-spp MSE on the held-out views with a
    faster frame."""
    import numpy as np
    import torch

    from paper_2410_05095_amd import _native as N
    from paper_2410_05095_amd import denoise as D
    from paper_2410_05095_amd import scenegen as sg
    t0 = time.perf_counter()
    train_scenes = []
    for seed in range(args.seed + 1, args.seed + 1 + args.denoiser_scenes):
        sc = sg.big_scene(seed)
        train_scenes.append((sc, ctx.scene_from(sc).build(device_sah=True)))
    log(f"[bench] training scenes ready ({time.perf_counter() - t0:.1f} s)")
    data = D.make_training_set(ctx, train_scenes, n_views=args.denoiser_views, crops_per_view=args.denoiser_cpv,
                               crop=args.denoiser_crop, seed=args.seed, log=log)
    n_crops = len(data)
    for _, h in train_scenes:
        h.close()
    den = N.Denoiser(ctx, seed=args.seed)
    t1 = time.perf_counter()
    losses = D.train(den, data, steps=args.denoiser_steps, batch=8, lr=args.denoiser_lr, seed=args.seed, log=log,
                     log_every=500, warmup=args.denoiser_warmup)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    del data
    torch.cuda.empty_cache()
    ev = D.evaluate(ctx, den, gs, scene, cam, plain_spp=args.spp, ref_spp=256, reps=5)
    held = D.orbit_views(np.random.default_rng(args.seed + 4242), 8, cam.width, cam.height, seed0=90000)
    ev["held_out"] = D.evaluate_views(ctx, den, gs, scene, held, plain_spp=args.spp)
    ho = ev["held_out"]
    ev["target_met"] = bool(ho["mse_denoised_1spp"] <= ho[f"mse_plain_{args.spp}spp"]
                            and ev["frame_ms_learned"] < ev[f"frame_ms_plain_{args.spp}spp"])
    ev["frame_faster_than_plain"] = bool(ev["frame_ms_learned"] < ev[f"frame_ms_plain_{args.spp}spp"])
    ev["held_out_plain_spp_equivalent"] = ho["mse_raw_1spp"] / max(ho["mse_denoised_1spp"], 1e-12)
    if args.anim_frames > 0:
        ev["animated"] = animated(ctx, gs, scene, den, args)
    ev.update({"train_steps": args.denoiser_steps, "train_s": round(train_s, 1), "train_crops": n_crops,
               "lr": args.denoiser_lr, "warmup_steps": args.denoiser_warmup,
               "crop": args.denoiser_crop, "train_views": args.denoiser_views,
               "train_scene_seeds": list(range(args.seed + 1, args.seed + 1 + args.denoiser_scenes)),
               "final_loss": [x for x in losses if x == x][-1],
               "weights": "bf16 (FP32 master)", "parity": "unpinned (statistical)"})
    den.close()
    rnd = lambda v: round(v, 7) if isinstance(v, float) else v
    return {k: ({a: rnd(b) for a, b in v.items()} if isinstance(v, dict) else rnd(v)) for k, v in ev.items()}


def timed_frames(ctx, gs, cam, kw, steps, warmup, out=None):
    """`steps` frames back to back after `warmup` untimed ones, a HIP event pair around each frame on the
    stream the library enqueues on (torch's current stream), the host synchronised only before and after.
    Returns (outputs, wall ms per frame, median event ms, event ms of each frame)."""
    import numpy as np
    import torch
    out = {} if out is None else out
    for _ in range(warmup):
        ctx.render(gs, cam, out=out, **kw)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        ctx.render(gs, cam, out=out, **kw)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    return out, wall * 1000.0 / steps, float(np.median(ms)), ms


def frame_and_stages(ctx, gs, cam, kw, steps, warmup):
    """Device time of a frame (HIP events around plain renders, median of `steps`), its stage split (renders
    timed by stage, medians of `steps`) and the ray, node and triangle counts (one counting render)."""
    import numpy as np
    out, _, frame_ms, _ = timed_frames(ctx, gs, cam, kw, steps, warmup)
    frames = []
    for _ in range(steps):
        ctx.render(gs, cam, out=out, timing=True, **kw)
        frames.append(ctx.stage_times())
    st = {k: float(np.median([f[k] for f in frames])) for k in ("primary_ms", "shadow_ms", "shade_ms", "total_ms")}
    ctx.render(gs, cam, out=out, count=True, **kw)
    c = ctx.stage_times()
    assert ctx.last_error() == 0
    st.update({k: c[k] for k in c if not k.endswith("_ms")})
    return out, frame_ms, st


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
    time of the whole frame (camera rays, shadow rays, shading), median of args.steps frames, and its stage
    split."""
    import numpy as np
    import torch
    c = scene.rect_light.center
    light = np.array([[c[0], c[1], c[2], 400.0, 400.0, 400.0]], np.float32)
    _, frame_ms, st = frame_and_stages(ctx, gs, cam, dict(lights=light), args.steps, args.warmup)
    torch.cuda.synchronize()
    rays = st["primary_rays"] + st["shadow_rays"]
    return {"frame_ms": round(frame_ms, 4), "primary_ms": round(st["primary_ms"], 4),
            "shadow_ms": round(st["shadow_ms"], 4), "rays_per_frame": int(rays),
            "mrays_per_s": round(rays / frame_ms / 1e3, 1),
            "paper_context": "paper: >7M triangles within 2 ms of GPU time per frame on an RTX 4090 "
                             "(raster + hardware ray queries; resolution not stated)"}


def device_build(ctx, scene, cam, kw, args):
    """The GPU builds of the same scene (positions already in HBM): the binned SAH (the host build's algorithm,
    giving its tree) and the linear BVH.  Build time (median of 3, from the first kernel to the finished tree,
    allocation included), tree size and SAH cost, and the frame's device time rendered through each tree
    (median of args.steps frames)."""
    import numpy as np
    res = {}
    for name, opt in (("binned_sah", dict(device_sah=True)), ("lbvh", dict(device=True))):
        gs = ctx.scene_from(scene)
        ms = []
        for _ in range(3):
            gs.build(**opt)
            ms.append(gs.stats()["build_ms"])
        st = gs.stats()
        _, frame_ms, sg_ = frame_and_stages(ctx, gs, cam, kw, args.steps, args.warmup)
        gs.close()
        res[name] = {"build_ms": round(float(np.median(ms)), 2), "nodes": int(st["n_nodes"]), "depth": int(st["depth"]),
                     "sah": round(st["sah_cost"], 4), "frame_device_ms": round(frame_ms, 4),
                     "shadow_ms": round(sg_["shadow_ms"], 4), "primary_ms": round(sg_["primary_ms"], 4)}
        log(f"[bench] device build {name}: {res[name]}")
    return res


def watertight_frames(ctx, scene, cam, kw, args):
    """The same frames with every ray/triangle test watertight (RC_BUILD_WATERTIGHT, binned-SAH tree of
    the same scene): device time of the 64-sample frame and of the hard-shadow frame, medians of args.steps."""
    import numpy as np
    gs = ctx.scene_from(scene).build(watertight=True, device_sah=True)
    c = scene.rect_light.center
    hard = dict(lights=np.array([[c[0], c[1], c[2], 400.0, 400.0, 400.0]], np.float32))
    res = {}
    for name, k in (("soft", kw), ("hard", hard)):
        _, frame_ms, st = frame_and_stages(ctx, gs, cam, k, args.steps, args.warmup)
        res[name] = {"frame_device_ms": round(frame_ms, 4), "shadow_ms": round(st["shadow_ms"], 4),
                     "primary_ms": round(st["primary_ms"], 4)}
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
        ctx.render(g, cam, out=out, count=True, **kw)
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


def batch_views(ctx, args):
    """Batched views: 64 cameras (square, 256..1024 pixels a side) over four scenes of 0.1M, 0.5M, 1M and 2M
    triangles with 1-4 point lights each, all rendered by one persistent launch fed by the device work queue.
    The autotuner times every candidate of its built-in grid (tile, queue depth, rays per wave, waves per
    SIMD) on this batch and picks the fastest; the batch is then captured as a hipGraph and replayed:
    device time per replay (HIP events, median), rays per batch, and Mrays/s."""
    import numpy as np
    import torch

    from paper_2410_05095_amd import scenegen as sg
    t0 = time.perf_counter()
    scenes, _ = sg.batch_scenes(args.seed)
    handles, views, lights = [], [], []
    for si, sc in enumerate(scenes):
        handles.append(ctx.scene_from(sc).build(device_sah=True))
        lf = len(lights)
        lights.extend(sc.point_lights.tolist())
        for cam in sc.cameras:
            views.append((si, cam, lf, len(sc.point_lights)))
    lights = np.asarray(lights, np.float32).reshape(-1, 6)
    log(f"[bench] batch: {len(views)} views over {[s.n_tris for s in scenes]} triangles "
        f"({time.perf_counter() - t0:.1f} s)")
    t1 = time.perf_counter()
    best, tune_ms = ctx.autotune(handles, views, lights, reps=3)
    tune_s = time.perf_counter() - t1
    outs = ctx.render_batch(handles, views, lights, tune=best, timing=True, count=True)
    st = ctx.stage_times()
    for _ in range(3):
        outs = ctx.render_batch(handles, views, lights, tune=best, graph=True, outs=outs)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        ctx.render_batch(handles, views, lights, tune=best, graph=True, outs=outs)
        b.record()
    torch.cuda.synchronize()
    assert ctx.last_error() == 0
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    default_outs = ctx.render_batch(handles, views, lights, timing=True)
    default_ms = ctx.stage_times()["total_ms"]
    for h in handles:
        h.close()
    del outs, default_outs
    rays = int(st["primary_rays"]) + int(st["shadow_rays"])   # the three-kernel form counts them apart
    pixels = int(sum(c.width * c.height for _, c, _, _ in views))
    log(f"[bench] batch: tuning {best} ({tune_s:.1f} s), replay {ms:.3f} ms")
    return {"views": len(views), "scenes_tris": [int(s.n_tris) for s in scenes], "pixels": pixels,
            "rays_per_batch": rays, "camera_rays": pixels, "shadow_rays": rays - pixels,
            "graph_replay_ms": round(ms, 4), "mrays_per_s": round(rays / ms / 1e3, 1),
            "default_tuning_ms": round(default_ms, 4), "tuning": best,
            "autotune": {"grid": "built-in (one kernel / three kernels, tile 8x8/16x8/16x16, queue 64/256/1024, "
                                 "min rays 16/32/48, 2 occupancies)", "best_candidate_ms": round(tune_ms, 4), "search_s": round(tune_s, 1)}}


def animated(ctx, gs, scene, den, args):
    """The same scene with 300 rigid bodies moving (<= 5 cm, <= 2 degrees per frame), BVH refit every frame,
    args.anim_views 1080p views per frame on the learned 1-spp path; per-frame shadow MSE of the BF16
    denoiser and of its FP32 copy against 256 samples, for every view of frames 0, 30, 60, 90 and the last,
    and for view f mod V of every other frame f."""
    import numpy as np

    from paper_2410_05095_amd import animate as A
    from paper_2410_05095_amd import denoise as D
    from paper_2410_05095_amd import scenegen as sg
    anim = sg.RigidAnimation(scene, n_bodies=300, seed=args.seed)
    views = D.orbit_views(np.random.default_rng(args.seed + 77), args.anim_views, 1920, 1080, seed0=5000)
    F, V = args.anim_frames, args.anim_views
    full = {0, F - 1} | {f for f in (30, 60, 90) if f < F}
    plan = lambda f: list(range(V)) if f in full else [f % V]
    res = A.run(ctx, scene, gs, den, anim, views, F, plan, log=log)
    res.pop("per_frame")
    res["reference_plan"] = (f"256-sample references for all {V} views of frames {sorted(full)} and for view "
                             f"f mod {V} of every other frame f")
    rnd = lambda v: round(v, 6) if isinstance(v, float) else v
    return {k: rnd(v) for k, v in res.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="big_7M", choices=["big_7M", "city_1M"])
    ap.add_argument("--spp", type=int, default=64, help="rect-light samples per pixel (big_7M)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--denoiser-steps", type=int, default=6000,
                    help="training steps (batches of 8 crops) of the learned 1-spp path (0 = skip the learned path)")
    ap.add_argument("--denoiser-scenes", type=int, default=4,
                    help="training scenes (seeds after the evaluation seed) of the denoiser's training set")
    ap.add_argument("--denoiser-views", type=int, default=200,
                    help="1080p views of the training scenes rendered for the denoiser's training set")
    ap.add_argument("--denoiser-cpv", type=int, default=10, help="training crops cut from each view")
    ap.add_argument("--denoiser-crop", type=int, default=512, help="training crop side in pixels")
    ap.add_argument("--denoiser-lr", type=float, default=1e-3, help="peak Adam learning rate (cosine decay)")
    ap.add_argument("--denoiser-warmup", type=int, default=300, help="steps of linear learning-rate ramp")
    ap.add_argument("--anim-frames", type=int, default=120,
                    help="animated frames (moving bodies, refit) rendered after the learned-path comparison")
    ap.add_argument("--anim-views", type=int, default=16, help="1080p views per animated frame")
    ap.add_argument("--dyn-frames", type=int, default=24,
                    help="frames of the moving-body comparison of flat refit and two-level rebuild (0 = skip)")
    ap.add_argument("--batch", type=int, default=1, help="run the 64-view / 4-scene batched leg (autotuned, graph replay)")
    ap.add_argument("--profile-denoiser-train", type=int, default=0,
                    help="time N training steps of the denoiser alone (batch 8 x crop^2) and exit")
    ap.add_argument("--profile-denoiser", type=int, default=0,
                    help="instead of rendering, run this many BF16 denoiser inferences of one 1080p view (twice: "
                         "warm-up, timed) and one FP32-copy inference")
    ap.add_argument("--build-only", type=int, default=0,
                    help="instead of rendering, build the scene's BVH on the GPU this many times (for profilers)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="instead of rendering, copy a buffer of this many MiB 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (views or tiles would be split "
              "across GPUs with a final image gather).", file=sys.stderr)
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

    if args.profile_denoiser_train:
        # the denoiser's training step alone (for profilers): batch 8 of crops of --denoiser-crop pixels, random
        # features, targets and an all-ones mask
        ctx = N.Context(0)
        den = N.Denoiser(ctx, seed=args.seed)
        g = torch.Generator(device="cuda").manual_seed(args.seed)
        S = args.denoiser_crop
        feat = torch.rand((8, S, S, 8), device="cuda", generator=g).to(torch.bfloat16).contiguous()
        tgt = torch.rand((8, S, S), device="cuda", generator=g).contiguous()
        msk = torch.ones((8, S, S), device="cuda")
        for _ in range(2):
            den.train_step(feat, tgt, msk, 1e-4, want_loss=False)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(args.profile_denoiser_train):
            den.train_step(feat, tgt, msk, 1e-4, want_loss=False)
        ev[1].record()
        torch.cuda.synchronize()
        print(json.dumps({"denoiser_train_step_ms": ev[0].elapsed_time(ev[1]) / args.profile_denoiser_train,
                          "batch": 8, "crop": S}), flush=True)
        return

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
    gs = ctx.scene_from(scene).build(device_sah=True)   # the binned-SAH tree of the host builder, built on the GPU
    bst = gs.stats()
    log(f"[bench] BVH: {bst}")

    if args.workload == "big_7M":
        kw = dict(lights=(), rect=scene.rect_light, area_samples=args.spp, area_stream=0)
    else:
        kw = dict(lights=scene.point_lights)
    out = {}
    for i in range(args.warmup):
        ctx.render(gs, cam, out=out, **kw)
    torch.cuda.synchronize()
    assert ctx.last_error() == 0
    log(f"[bench] warmup done")

    # timed region: K frames back to back on the library's stream, HIP events around each frame, one host
    # synchronisation at each end
    out, ms_step, frame_med, _ = timed_frames(ctx, gs, cam, kw, args.steps, 0, out)
    assert ctx.last_error() == 0
    # per-stage device times (RC_FLAG_TIMING adds events between the stages): median of 10 frames
    stages = []
    for _ in range(10):
        ctx.render(gs, cam, out=out, timing=True, **kw)
        stages.append(ctx.stage_times())
    st = {k: float(np.median([s[k] for s in stages])) for k in stages[0]}
    # rays cast and the wave kernels' node visits and triangle tests: one counting render (RC_FLAG_COUNT)
    ctx.render(gs, cam, out=out, count=True, **kw)
    cnt = ctx.stage_times()
    st.update({k: float(cnt[k]) for k in cnt if not k.endswith("_ms")})
    # own-path work: the same frame through the per-lane kernels, whose counters count each ray's own node
    # visits and triangle tests (near-first order, any hit), as the oracle's instrumented traversal does
    ctx.render(gs, cam, out={}, per_lane=True, count=True, **kw)
    own = ctx.stage_times()
    torch.cuda.synchronize()
    assert ctx.last_error() == 0
    rays = st["primary_rays"] + st["shadow_rays"]
    value = rays / (ms_step / 1000.0) / 1e6
    # roofline of the dominant kernel (shadow traversal).  Its lanes mostly fetch the same nodes (the
    # light samples of one pixel share a wave), so the caches serve nearly all node and triangle bytes and
    # the measured fabric traffic is far below HBM bandwidth: the bound is vector instruction issue.
    # achieved = the algorithmic vector work of the launch (each ray's own node visits x 52 + own triangle
    # tests x 37 FP32 lane-operations) / the kernel's device time.
    npix = cam.width * cam.height * cam.ssaa ** 2
    dom_ms = st["shadow_ms"]
    sh_rays = max(st["shadow_rays"], 1)
    own_nodes, own_tris = own["shadow_nodes"] / max(own["shadow_rays"], 1), own["shadow_tris"] / max(own["shadow_rays"], 1)
    dom_ops = st["shadow_rays"] * (own_nodes * NODE_VOPS + own_tris * TRI_OPS)
    exec_ops = st["shadow_nodes"] * NODE_VOPS + st["shadow_tris"] * TRI_OPS
    achieved = dom_ops / (dom_ms / 1000.0) / 1e12
    logical_bytes = st["shadow_rays"] * (own_nodes * NODE_BYTES + own_tris * TRI_BYTES) + npix * 20
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
        "frame_ms_median_events": round(frame_med, 4),
        "stages_ms": {"primary": round(st["primary_ms"], 4), "shadow": round(st["shadow_ms"], 4),
                      "shade_resolve": round(st["shade_ms"], 4), "render_device": round(st["total_ms"], 4)},
        "rays_per_frame": {"primary": int(st["primary_rays"]), "shadow": int(st["shadow_rays"])},
        "mrays_per_s_kernel": {"primary": round(st["primary_rays"] / st["primary_ms"] / 1e3, 1),
                               "shadow": round(st["shadow_rays"] / st["shadow_ms"] / 1e3, 1)},
        "mrays_per_s_frame": {"primary": round(st["primary_rays"] / ms_step / 1e3, 1),
                              "shadow": round(st["shadow_rays"] / ms_step / 1e3, 1)},
        "per_ray": {"primary_nodes": round(own["primary_nodes"] / max(own["primary_rays"], 1), 2),
                    "primary_tris": round(own["primary_tris"] / max(own["primary_rays"], 1), 2),
                    "shadow_nodes": round(own_nodes, 2), "shadow_tris": round(own_tris, 2),
                    "counted_by": "own path (per-lane traversal counters)",
                    "wave_union_primary_nodes": round(st["primary_nodes"] / max(st["primary_rays"], 1), 2),
                    "wave_union_primary_tris": round(st["primary_tris"] / max(st["primary_rays"], 1), 2),
                    "wave_union_shadow_nodes": round(st["shadow_nodes"] / sh_rays, 2),
                    "wave_union_shadow_tris": round(st["shadow_tris"] / sh_rays, 2)},
        "bvh": {"method": "binned SAH (32 bins, leaves <= 4, node cost 4) built on the GPU",
                "build_ms": round(bst["build_ms"], 1), "nodes": int(bst["n_nodes"]), "depth": int(bst["depth"]),
                "sah": round(bst["sah_cost"], 4)},
        "roofline": {"kernel": "k_rect_wave" if args.workload == "big_7M" else "k_point_wave", "bound": "alu",
                     "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2), "unit": "T lane-ops/s",
                     "frac": round(achieved / ALU_PEAK_TOPS, 4),
                     "traffic": (MEASURED_TRAFFIC.get((args.workload, args.spp, kernel_hash()))
                                 if args.workload == "big_7M" else None),
                     "work": f"own path: {own_nodes:.2f} node visits x {NODE_VOPS} + {own_tris:.2f} triangle tests "
                             f"x {TRI_OPS} FP32 lane-ops per ray",
                     "executed_union_over_own": round(exec_ops / max(dom_ops, 1.0), 3),
                     "logical_node_tri_GBps": round(logical_bytes / (dom_ms / 1000.0) / 1e9, 1)},
    }
    res["post"] = post_pass(ctx, out, args)
    res["device_bvh"] = device_build(ctx, scene, cam, kw, args)
    if args.workload == "big_7M":
        res["watertight"] = watertight_frames(ctx, scene, cam, kw, args)
    if args.workload == "big_7M" and args.dyn_frames > 1:
        res["dynamic_structures"] = dynamic_structures(ctx, gs, scene, cam, args)
    if args.workload == "big_7M":
        res["hard_shadows"] = hard_shadows(ctx, gs, scene, cam, args)
    if args.batch:
        res["batch"] = batch_views(ctx, args)
    if args.workload == "big_7M" and args.denoiser_steps > 0:
        res["denoiser"] = learned_path(ctx, gs, scene, cam, args)
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        res["cpu_baseline"] = cpu_baseline(scene, cam, args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
