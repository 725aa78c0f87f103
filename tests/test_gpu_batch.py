"""Batched persistent rendering: every view bit-identical to its single-view render for any tuning,
graph replays identical to eager launches, autotuner + cache, and the 64-view / 4-scene workload."""
import os
import sys
import tempfile

import numpy as np
import pytest

from paper_2410_05095_amd import scenegen as sg
from tests.parity import assert_clean, compare_point, to_np

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_05095_amd import _native as N
    c = N.Context(0)
    yield c
    c.close()


def build_batch(ctx, scenes, cams_per_scene):
    """-> (scene handles, views [(scene idx, cam, light_first, n_lights)], lights array)"""
    handles, views, lights = [], [], []
    for si, sc in enumerate(scenes):
        handles.append(ctx.scene_from(sc).build())
        lf = len(lights)
        lights.extend(sc.point_lights.tolist())
        for cam in cams_per_scene[si]:
            views.append((si, cam, lf, len(sc.point_lights)))
    return handles, views, np.asarray(lights, np.float32).reshape(-1, 6)


def single_renders(ctx, scenes, handles, views):
    import torch
    out = []
    for si, cam, lf, nl in views:
        o = ctx.render(handles[si], cam, scenes[si].point_lights, per_lane=True)
        out.append({k: v.clone() for k, v in o.items() if v is not None})
    torch.cuda.synchronize()
    return out


def same(a, b):
    import torch
    for k in ("rgba", "hit", "shadow"):
        if k in a and a[k] is not None:
            if not torch.equal(a[k], b[k]):
                return k
    return None


def small_batch():
    scenes = [sg.small_random_scene(10 + i, n_instances=10 + 5 * i, width=8, height=8, n_lights=i) for i in range(3)]
    cams = [[], [], []]
    rng = np.random.default_rng(0)
    sizes = [(37, 29, 1), (64, 64, 2), (23, 41, 2), (80, 45, 1), (16, 16, 1), (51, 33, 2), (40, 40, 1)]
    for n, (w, h, ss) in enumerate(sizes):
        eye = tuple(float(x) for x in rng.uniform([-20, 5, -30], [20, 25, -20]))
        cams[n % 3].append(sg.Camera(eye=eye, target=(0.0, 6.0, 0.0), up=(0, 1, 0), vfov_deg=45.0 + n, width=w,
                                     height=h, ssaa=ss, seed=n, frame=n % 2))
    return scenes, cams


TUNES = [None,
         dict(tile_w=4, tile_h=4, queue_depth=64, min_rays=1, waves_per_simd=1, passes=1),
         dict(tile_w=32, tile_h=32, queue_depth=4096, min_rays=64, waves_per_simd=0, passes=1),
         dict(tile_w=16, tile_h=4, queue_depth=128, min_rays=24, waves_per_simd=2, passes=1),
         dict(tile_w=4, tile_h=4, queue_depth=64, min_rays=1, waves_per_simd=1, passes=3),
         dict(tile_w=32, tile_h=32, queue_depth=4096, min_rays=64, waves_per_simd=0, passes=3),
         dict(tile_w=16, tile_h=4, queue_depth=128, min_rays=24, waves_per_simd=2, passes=3)]


def test_batch_bit_identical_to_single_views(ctx):
    import torch
    scenes, cams = small_batch()
    handles, views, lights = build_batch(ctx, scenes, cams)
    ref = single_renders(ctx, scenes, handles, views)
    for tune in TUNES:
        outs = ctx.render_batch(handles, views, lights, tune=tune)
        torch.cuda.synchronize()
        assert ctx.last_error() == 0
        for i in range(len(views)):
            assert same(outs[i], ref[i]) is None, (tune, i, same(outs[i], ref[i]))
        say(f"[batch] tune {tune}: {len(views)} views identical")


@pytest.mark.parametrize("passes", [3, 1])
def test_batch_graph_replays(ctx, passes):
    import torch
    scenes, cams = small_batch()
    handles, views, lights = build_batch(ctx, scenes, cams)
    ref = single_renders(ctx, scenes, handles, views)
    tune = dict(tile_w=8, tile_h=8, queue_depth=256, min_rays=40, waves_per_simd=0, passes=passes)
    outs = None
    for rep in range(4):
        outs = ctx.render_batch(handles, views, lights, tune=tune, graph=True, outs=outs)
        torch.cuda.synchronize()
        # eager work between replays
        x = torch.randn(1 << 16, device="cuda").sum().item()
        for i in range(len(views)):
            assert same(outs[i], ref[i]) is None, (rep, i)
        for o in outs:
            for k in o:
                if o[k] is not None:
                    o[k].zero_()
    # same shape, moved cameras: the replay uses the new table
    moved = [(si, sg.Camera(**{**cam.__dict__, "eye": (cam.eye[0] + 1.0, cam.eye[1], cam.eye[2])}), lf, nl)
             for si, cam, lf, nl in views]
    ref2 = single_renders(ctx, scenes, handles, moved)
    outs = ctx.render_batch(handles, moved, lights, tune=tune, graph=True, outs=outs)
    torch.cuda.synchronize()
    for i in range(len(views)):
        assert same(outs[i], ref2[i]) is None
    assert ctx.last_error() == 0


@pytest.mark.parametrize("passes", [3, 1])
def test_batch_more_views_than_the_lds_table(ctx, passes):
    """300 small views (the kernels keep the views' first items in LDS only up to 256 views and search the
    device table beyond): every view bit-identical to its single-view render."""
    import torch
    scenes = [sg.small_random_scene(30 + i, n_instances=8, width=8, height=8, n_lights=1 + i) for i in range(2)]
    rng = np.random.default_rng(5)
    cams = [[], []]
    for n in range(300):
        eye = tuple(float(x) for x in rng.uniform([-20, 5, -30], [20, 25, -20]))
        cams[n % 2].append(sg.Camera(eye=eye, target=(0.0, 6.0, 0.0), up=(0, 1, 0), vfov_deg=40.0 + n % 30,
                                     width=12 + n % 9, height=8 + n % 7, ssaa=1 + n % 2, seed=n, frame=n % 3))
    handles, views, lights = build_batch(ctx, scenes, cams)
    assert len(views) > 256
    ref = single_renders(ctx, scenes, handles, views)
    tune = dict(tile_w=8, tile_h=8, queue_depth=256, min_rays=40, waves_per_simd=0, passes=passes)
    outs = ctx.render_batch(handles, views, lights, tune=tune)
    torch.cuda.synchronize()
    assert ctx.last_error() == 0
    bad = [i for i in range(len(views)) if same(outs[i], ref[i]) is not None]
    say(f"[batch300] passes {passes}: {len(views)} views, {len(bad)} differ")
    assert not bad
    for h in handles:
        h.close()


def test_batch_graph_after_buffer_growth():
    """A single-view render that grows the context's overflow stack area between two launches of a captured
    batch graph: the context captures again instead of replaying into the freed area."""
    import torch
    from paper_2410_05095_amd import _native as N
    from tests.test_gpu_render import deep_scene
    c2 = N.Context(0)
    scenes, cams = small_batch()
    handles, views, lights = build_batch(c2, scenes, cams)
    ref = single_renders(c2, scenes, handles, views)
    outs = c2.render_batch(handles, views, lights, graph=True)
    torch.cuda.synchronize()
    deep = deep_scene()
    gd = c2.scene_from(deep).build()
    c2.render(gd, deep.cameras[0], (), rect=deep.rect_light, area_samples=4, area_stream=0, per_lane=True)
    torch.cuda.synchronize()
    for o in outs:
        for k in o:
            if o[k] is not None:
                o[k].zero_()
    outs = c2.render_batch(handles, views, lights, graph=True, outs=outs)
    torch.cuda.synchronize()
    for i in range(len(views)):
        assert same(outs[i], ref[i]) is None, i
    assert c2.last_error() == 0
    gd.close()
    for h in handles:
        h.close()
    c2.close()


def test_autotune_and_cache(ctx):
    scenes, cams = small_batch()
    handles, views, lights = build_batch(ctx, scenes, cams)
    cands = [dict(tile_w=8, tile_h=8, queue_depth=256, min_rays=40, waves_per_simd=0, passes=3),
             dict(tile_w=16, tile_h=16, queue_depth=64, min_rays=16, waves_per_simd=1, passes=1)]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.jsonl")
        best, ms = ctx.autotune(handles, views, lights, candidates=cands, reps=2, cache_path=path)
        say("[autotune]", best, ms)
        assert ms > 0
        assert (best["tile_w"], best["tile_h"]) in ((8, 8), (16, 16))
        text = open(path).read()
        assert '"key":"gfx' in text and text.count("\n") == 1
        best2, ms2 = ctx.autotune(handles, views, lights, candidates=cands, reps=2, cache_path=path)
        assert best2 == best and open(path).read() == text     # served from the cache


def test_batch_64_views_4_scenes(ctx, oracle_mod):
    """64 views (256..1024 square) over scenes of 0.1M/0.5M/1M/2M triangles in one launch with the tuning the
    autotuner picks from its built-in grid (as the benchmark runs it), replayed from a hipGraph; 8 views
    compared bit for bit with single-view renders, 2 views sampled against the oracle."""
    import torch
    O = oracle_mod
    scenes, cams = sg.batch_scenes(0)
    handles, views, lights = build_batch(ctx, scenes, [s.cameras for s in scenes])
    say(f"[batch64] {len(views)} views, {sum(c.width * c.height for _, c, _, _ in views)} pixels, "
        f"tris {[s.n_tris for s in scenes]}")
    best, best_ms = ctx.autotune(handles, views, lights, reps=1)
    say(f"[batch64] autotuned: {best} ({best_ms:.2f} ms)")
    outs = ctx.render_batch(handles, views, lights, tune=best, timing=True, count=True)
    st = ctx.stage_times()
    say(f"[batch64] {st['total_ms']:.2f} ms, {st['primary_rays'] + st['shadow_rays']} rays")
    for o in outs:
        for k in o:
            if o[k] is not None:
                o[k].zero_()
    outs = ctx.render_batch(handles, views, lights, tune=best, graph=True, outs=outs)
    torch.cuda.synchronize()
    assert ctx.last_error() == 0
    rng = np.random.default_rng(0)
    pick = rng.choice(len(views), 8, replace=False)
    ref = single_renders(ctx, scenes, handles, [views[i] for i in pick])
    for n, i in enumerate(pick):
        assert same(outs[i], ref[n]) is None, i
    for i in pick[:2]:
        si, cam, lf, nl = views[i]
        smp = np.sort(rng.choice(cam.n_samples, 3000, replace=False))
        orc = O.OracleScene.from_scene(scenes[si]).render_point(cam, scenes[si].point_lights, smp)
        o = ctx.render(handles[si], cam, scenes[si].point_lights, sample_rgba=True, per_lane=True)
        torch.cuda.synchronize()
        stt = compare_point(to_np(outs[i]["hit"])[smp], to_np(outs[i]["shadow"])[smp],
                            to_np(o["sample_rgba"])[smp], orc, nl)
        say(f"[batch64 parity view {i}]", stt)
        assert_clean(stt)
