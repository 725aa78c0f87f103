"""Rigid-body transforms and BVH refit on the GPU: positions bit-exact against the oracle's FP32
mirror, every refit box equal to the exact bounds of its contents, renders of the moved scene at
parity with the oracle."""
import sys

import numpy as np
import pytest

from paper_2410_05095_amd import scenegen as sg
from tests.parity import assert_clean, bvh_bound_errors, compare_point, to_np

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


def move(ctx, gs, anim, frame):
    import torch
    xf = torch.from_numpy(anim.transforms(frame)).cuda()
    ids = torch.from_numpy(anim.body_ids.astype(np.int32)).cuda()
    gs.set_transforms(xf, ids)
    gs.refit()
    torch.cuda.synchronize()
    return xf.cpu().numpy()


def test_refit_small_scene_parity(ctx, oracle_mod):
    O = oracle_mod
    scene = sg.small_random_scene(3, n_instances=30, width=64, height=48, ssaa=2, n_lights=2)
    gs = ctx.scene_from(scene).build()
    sah0 = gs.stats()["sah_cost"]
    nodes, order = gs.export()
    assert bvh_bound_errors(nodes, order, scene.positions, scene.indices)[0] == 0   # checker on a fresh build
    anim = sg.RigidAnimation(scene, n_bodies=12, seed=1, max_disp=0.5, max_rot_deg=20.0)
    for frame in (1, 2, 5):
        xf = move(ctx, gs, anim, frame)
        want = O.transform_f32(scene.positions, scene.body_vertex_range, anim.body_ids, xf)
        got = gs.positions()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), frame
        nodes, order = gs.export()
        bad, _ = bvh_bound_errors(nodes, order, want, scene.indices)
        assert bad == 0
        moved = sg.Scene(**{**scene.__dict__, "positions": want})
        cam = scene.cameras[0]
        out = ctx.render(gs, cam, scene.point_lights, sample_rgba=True)
        orc = O.OracleScene.from_scene(moved).render_point(cam, scene.point_lights, np.arange(cam.n_samples))
        st = compare_point(to_np(out["hit"]), to_np(out["shadow"]), to_np(out["sample_rgba"]), orc,
                           len(scene.point_lights))
        say(f"[refit frame {frame}]", st)
        assert_clean(st)
    sah1 = gs.stats()["sah_cost"]
    fresh = ctx.scene(want, scene.indices, scene.tri_material, scene.materials).build().stats()["sah_cost"]
    say(f"[sah] built {sah0:.3f} refit {sah1:.3f} rebuilt {fresh:.3f}")
    assert sah1 >= 0.99 * fresh


def test_refit_big_scene_300_bodies(ctx, oracle_mod):
    """The 7.3M-triangle scene with 300 rigid bodies moving (<= 5 cm, <= 2 degrees per frame)."""
    O = oracle_mod
    import torch
    scene = sg.big_scene(0)
    gs = ctx.scene_from(scene).build()
    sah0 = gs.stats()["sah_cost"]
    anim = sg.RigidAnimation(scene, n_bodies=300, seed=0)
    for frame in (1, 2, 3):
        xf = move(ctx, gs, anim, frame)
    want = O.transform_f32(scene.positions, scene.body_vertex_range, anim.body_ids, xf)
    got = gs.positions()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    nodes, order = gs.export()
    bad, hist = bvh_bound_errors(nodes, order, want, scene.indices)
    assert bad == 0
    # moved scene renders at parity on sampled pixels (rect light, 16 samples)
    cam = scene.cameras[0]
    out = ctx.render(gs, cam, (), rect=scene.rect_light, area_samples=16, area_stream=2)
    torch.cuda.synchronize()
    moved = sg.Scene(**{**scene.__dict__, "positions": want})
    rng = np.random.default_rng(3)
    pix = np.sort(rng.choice(cam.width * cam.height, 3000, replace=False))
    orc = O.OracleScene.from_scene(moved).render_rect(cam, scene.rect_light, 16, 2, pix)
    hit = to_np(out["hit"]).view(np.uint32)[pix, 0]
    cnt = np.rint(to_np(out["visibility"]).reshape(-1)[pix] * 16).astype(np.int64)
    ok = orc["band_primary"] == 0
    assert (hit[ok] != orc["hit_id"][ok]).sum() == 0
    assert (np.abs(cnt - orc["vis_count"])[ok] <= orc["band_count"][ok]).all()
    say(f"[big refit] sah built {sah0:.3f} after 3 frames {gs.stats()['sah_cost']:.3f}; leaf sizes {hist.tolist()}")


@pytest.mark.parametrize("build", ["device", "watertight"])
def test_refit_after_several_moves(ctx, oracle_mod, build):
    """The refit recomputes only the nodes that hold moved triangles (and their ancestors): two transform calls
    on different bodies before one refit, on a GPU-built tree and on a watertight (raw-vertex) tree, leave
    every box exact and the renders at parity."""
    import torch
    O = oracle_mod
    scene = sg.small_random_scene(8, n_instances=40, width=48, height=40, ssaa=1, n_lights=2)
    gs = ctx.scene_from(scene)
    gs.build(device=(build == "device"), watertight=(build == "watertight"))
    anim = sg.RigidAnimation(scene, n_bodies=20, seed=4, max_disp=0.4, max_rot_deg=15.0)
    xf = anim.transforms(3)
    ids = anim.body_ids.astype(np.int32)
    half = len(ids) // 2
    for sel in (slice(0, half), slice(half, None)):
        gs.set_transforms(torch.from_numpy(xf[sel].copy()).cuda(), torch.from_numpy(ids[sel].copy()).cuda())
    gs.refit()
    torch.cuda.synchronize()
    assert ctx.last_error() == 0
    want = O.transform_f32(scene.positions, scene.body_vertex_range, anim.body_ids, xf)
    assert np.array_equal(gs.positions().view(np.uint32), want.view(np.uint32))
    nodes, order = gs.export()
    assert bvh_bound_errors(nodes, order, want, scene.indices)[0] == 0
    # a second refit without motion changes nothing
    gs.refit()
    nodes2, _ = gs.export()
    assert np.array_equal(nodes, nodes2)
    moved = sg.Scene(**{**scene.__dict__, "positions": want})
    cam = scene.cameras[0]
    out = ctx.render(gs, cam, scene.point_lights, sample_rgba=True)
    orc = O.OracleScene.from_scene(moved, watertight=(build == "watertight")).render_point(
        cam, scene.point_lights, np.arange(cam.n_samples))
    st = compare_point(to_np(out["hit"]), to_np(out["shadow"]), to_np(out["sample_rgba"]), orc,
                       len(scene.point_lights))
    say(f"[refit {build}]", st)
    assert_clean(st)


def test_transform_rejects_unknown_body(ctx):
    """A body id beyond the scene's bodies moves nothing and sets the sticky RC_ERR_INVALID_VALUE."""
    import torch
    scene = sg.small_random_scene(9, n_instances=6, width=16, height=16)
    gs = ctx.scene_from(scene).build()
    before = gs.positions()
    xf = torch.from_numpy(np.tile(np.array([1, 0, 0, 5, 0, 1, 0, 0, 0, 0, 1, 0], np.float32), (1, 1))).cuda()
    gs.set_transforms(xf, torch.tensor([scene.body_vertex_range.shape[0] + 3], dtype=torch.int32).cuda())
    gs.refit()
    torch.cuda.synchronize()
    assert ctx.last_error() == -2
    assert np.array_equal(gs.positions(), before)
