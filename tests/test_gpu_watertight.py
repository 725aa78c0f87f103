"""The watertight ray/triangle test (RC_BUILD_WATERTIGHT) through the C ABI.

Renders match the oracle with the watertight band model exactly outside its band (camera rays with one and
four samples, point-light and rect-light shadows with both rect kernels; flat host and GPU builds and the
two-level structure).  On a mesh whose vertices lie on the camera's pixel rays (every interior ray passes
through a vertex shared by six triangles, within FP32 rounding) no ray escapes between triangles."""
import sys

import numpy as np
import pytest

from paper_2410_05095_amd import scenegen as sg
from tests.test_gpu_render import compare_rect, render_and_compare

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


@pytest.mark.parametrize("seed,ssaa,w,h,how", [(0, 1, 37, 29, "host"), (2, 2, 48, 36, "host"),
                                               (5, 1, 40, 30, "device"), (3, 2, 33, 27, "two_level")])
def test_watertight_point_parity(ctx, oracle_mod, seed, ssaa, w, h, how):
    O = oracle_mod
    scene = sg.small_random_scene(seed, n_instances=30, width=w, height=h, ssaa=ssaa, n_lights=3)
    gs = ctx.scene_from(scene).build(watertight=True, device=how == "device", two_level=how == "two_level")
    if how == "two_level":
        nb = len(scene.body_tri_range)
        o2w = np.zeros((nb, 12), np.float32)
        o2w[:, 0] = o2w[:, 5] = o2w[:, 10] = 1.0
        osc = O.OracleScene.two_level(scene.positions, scene.positions, scene.indices, scene.tri_material,
                                      scene.materials, scene.body_tri_range, o2w, watertight=True)
    else:
        osc = O.OracleScene.from_scene(scene, watertight=True)
    render_and_compare(ctx, O, scene, scene.cameras[0], gs=gs, osc=osc)
    gs.close()


@pytest.mark.parametrize("seed,N,stream", [(0, 16, 0), (6, 64, 4)])
def test_watertight_rect_parity(ctx, oracle_mod, seed, N, stream):
    O = oracle_mod
    scene = sg.small_random_scene(seed, n_instances=40, width=40, height=32, ssaa=1)
    gs = ctx.scene_from(scene).build(watertight=True)
    compare_rect(ctx, O, scene, scene.cameras[0], N, stream, gs=gs, osc=O.OracleScene.from_scene(scene, watertight=True))
    gs.close()


def vertex_grid_scene(cam, seed=0):
    """A bumpy sheet whose vertex (i, j) is the point at distance 6 + 0.8 sin(..) along pixel (i, j)'s camera
    ray (FP64, rounded to FP32), triangulated over neighbouring pixels; every interior pixel's ray passes
    through a vertex shared by six triangles."""
    from oracle import oracle as O
    W, H = cam.width, cam.height
    o, d = O.gen_rays(cam, np.arange(W * H))
    i, j = np.meshgrid(np.arange(W), np.arange(H))
    t = 6.0 + 0.8 * np.sin(0.37 * i.ravel() + 0.21 * j.ravel() + seed)
    pos = (o.astype(np.float64) + d.astype(np.float64) * t[:, None]).astype(np.float32)
    tris = []
    for y in range(H - 1):
        for x in range(W - 1):
            a, b, c, e = y * W + x, y * W + x + 1, (y + 1) * W + x, (y + 1) * W + x + 1
            if (x + y) % 2 == 0:
                tris += [(a, b, e), (a, e, c)]
            else:
                tris += [(a, b, c), (b, e, c)]
    idx = np.asarray(tris, np.uint32)
    mats = np.array([[0.6, 0.6, 0.6, 0.5, 0.0]], np.float32)
    return pos, idx, np.zeros(len(idx), np.uint32), mats


@pytest.mark.parametrize("seed", [0, 1])
def test_no_camera_ray_escapes_through_shared_vertices(ctx, seed):
    import torch
    cam = sg.Camera(eye=(0.3, 1.1, -2.0), target=(0.0, 0.4, 3.0), up=(0.0, 1.0, 0.0), vfov_deg=55.0,
                    width=96, height=72, ssaa=1)
    pos, idx, tm, mats = vertex_grid_scene(cam, seed)
    interior = np.zeros((cam.height, cam.width), bool)
    interior[1:-1, 1:-1] = True
    interior = interior.ravel()
    misses = {}
    for wt in (True, False):
        gs = ctx.scene(pos, idx, tm, mats).build(watertight=wt)
        out = ctx.render(gs, cam, ())
        torch.cuda.synchronize()
        hit = out["hit"].cpu().numpy().view(np.uint32)[:, 0]
        misses[wt] = int((hit[interior] == 0xFFFFFFFF).sum())
        gs.close()
    say(f"[watertight] interior camera rays through shared vertices that miss: watertight {misses[True]}, "
        f"Moller-Trumbore {misses[False]} (of {int(interior.sum())})")
    assert misses[True] == 0
