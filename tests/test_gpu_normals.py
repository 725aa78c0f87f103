"""Smooth shading with vertex normals through the C ABI against the oracle: at rest (camera rays with one and
four samples, point and rect lights) and with moved bodies, whose normals rotate with them (flat refit and
the two-level structure)."""
import numpy as np
import pytest

from paper_2410_05095_amd import scenegen as sg
from tests.test_gpu_render import compare_rect, render_and_compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_05095_amd import _native as N
    c = N.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("seed,ssaa,w,h", [(0, 1, 37, 29), (2, 2, 48, 36)])
def test_smooth_point_parity(ctx, oracle_mod, seed, ssaa, w, h):
    scene = sg.with_vertex_normals(sg.small_random_scene(seed, n_instances=30, width=w, height=h, ssaa=ssaa,
                                                         n_lights=3))
    render_and_compare(ctx, oracle_mod, scene, scene.cameras[0])


def test_smooth_rect_parity(ctx, oracle_mod):
    scene = sg.with_vertex_normals(sg.small_random_scene(6, n_instances=40, width=40, height=32, ssaa=1))
    compare_rect(ctx, oracle_mod, scene, scene.cameras[0], 64, 4)


@pytest.mark.parametrize("two_level", [False, True])
def test_smooth_moved_bodies(ctx, oracle_mod, two_level):
    import torch
    O = oracle_mod
    scene = sg.with_vertex_normals(sg.small_random_scene(4, n_instances=30, width=48, height=36, ssaa=1, n_lights=2))
    gs = ctx.scene_from(scene).build(two_level=two_level)
    anim = sg.RigidAnimation(scene, n_bodies=15, seed=3, max_disp=0.5, max_rot_deg=25.0)
    xf = anim.transforms(4)
    gs.set_transforms(torch.from_numpy(xf).cuda(), torch.from_numpy(anim.body_ids.astype(np.int32)).cuda())
    gs.refit()
    torch.cuda.synchronize()
    world = O.transform_f32(scene.positions, scene.body_vertex_range, anim.body_ids, xf)
    wn = O.rotate_f32(scene.normals, scene.body_vertex_range, anim.body_ids, xf)
    moved = sg.Scene(**{**scene.__dict__, "positions": world, "normals": wn})
    if two_level:
        nb = len(scene.body_tri_range)
        o2w = np.zeros((nb, 12), np.float32)
        o2w[:, 0] = o2w[:, 5] = o2w[:, 10] = 1.0
        o2w[anim.body_ids] = xf
        osc = O.OracleScene.two_level(world, scene.positions, scene.indices, scene.tri_material, scene.materials,
                                      scene.body_tri_range, o2w, world_normals=wn)
    else:
        osc = O.OracleScene.from_scene(moved)
    render_and_compare(ctx, O, moved, scene.cameras[0], gs=gs, osc=osc)
    gs.close()
