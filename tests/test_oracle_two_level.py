"""Pins of the oracle's two-level (instanced) hit queries.

Rigid motion does not change which triangle a ray meets: ray casting through instances (each body in
its rest frame, the ray mapped by the inverse of the body's rigid map) must give the hits of the flat
scene whose vertices are the mapped rest vertices, wherever neither side's FP32 band holds the ray.
The world-to-object map is pinned by its closed form, and the per-instance BVHs by brute force.  A
map with the rotation transposed (a plausible mistake) must fail the flat comparison."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_05095_amd import scenegen as sg


def two_level(scene, o2w, world=None, use_bvh=True):
    if world is None:
        world = scene.positions
    return O.OracleScene.two_level(world, scene.positions, scene.indices, scene.tri_material, scene.materials,
                                   scene.body_tri_range, o2w, use_bvh=use_bvh)


def identity_o2w(n):
    x = np.zeros((n, 12), np.float32)
    x[:, 0] = x[:, 5] = x[:, 10] = 1.0
    return x


def moved(scene, frame, seed=1):
    anim = sg.RigidAnimation(scene, n_bodies=len(scene.body_tri_range) // 2, seed=seed, max_disp=0.6,
                             max_rot_deg=25.0)
    xf = anim.transforms(frame)
    o2w = identity_o2w(len(scene.body_tri_range))
    o2w[anim.body_ids] = xf
    world = O.transform_f32(scene.positions, scene.body_vertex_range, anim.body_ids, xf)
    return o2w, world


def test_w2o_closed_form():
    rng = np.random.default_rng(0)
    n = 200
    o2w = np.zeros((n, 12), np.float32)
    for i in range(n):
        R = sg.random_rotation(rng).astype(np.float32)
        t = rng.uniform(-30, 30, 3).astype(np.float32)
        o2w[i] = np.concatenate([R, t[:, None]], 1).ravel()
    w = O.w2o_f32(o2w).reshape(n, 3, 4)
    X = o2w.reshape(n, 3, 4)
    assert np.array_equal(w[:, :, :3], np.transpose(X[:, :, :3], (0, 2, 1)))
    # m = -(R^T t) with the fixed FP32 order ((R0k t0 + R1k t1) + R2k t2)
    R, t = X[:, :, :3], X[:, :, 3]
    a = R[:, 0, :] * t[:, 0:1]
    b = R[:, 1, :] * t[:, 1:2]
    c = R[:, 2, :] * t[:, 2:3]
    assert np.array_equal(w[:, :, 3], -((a + b) + c))
    # the map inverts x = R x' + t up to FP32 rounding
    xo = rng.uniform(-2, 2, (n, 3))
    xw = np.einsum("nij,nj->ni", R.astype(np.float64), xo) + t
    back = np.einsum("nij,nj->ni", w[:, :, :3].astype(np.float64), xw) + w[:, :, 3]
    assert np.abs(back - xo).max() < 1e-4


def compare_point(a, b, n_lights):
    """Hit ids and shadow masks of two oracle runs, compared where neither run's band holds the sample."""
    ok = (a["band_primary"] == 0) & (b["band_primary"] == 0)
    assert (a["hit_id"][ok] != b["hit_id"][ok]).sum() == 0
    sh = ok & (a["band_shadow"] == 0) & (b["band_shadow"] == 0) & (a["hit_id"] != 0xFFFFFFFF)
    assert (a["mask"][sh] != b["mask"][sh]).sum() == 0
    return int((~ok).sum()), int(ok.sum())


@pytest.mark.parametrize("seed", [0, 3])
def test_identity_instances_match_flat(seed):
    scene = sg.small_random_scene(seed, n_instances=12, width=40, height=30, ssaa=2, n_lights=2)
    cam = scene.cameras[0]
    smp = np.arange(cam.n_samples)
    flat = O.OracleScene.from_scene(scene).render_point(cam, scene.point_lights, smp)
    inst = two_level(scene, identity_o2w(len(scene.body_tri_range))).render_point(cam, scene.point_lights, smp)
    band, n = compare_point(flat, inst, len(scene.point_lights))
    assert band < 0.01 * len(smp) and (flat["hit_id"] != 0xFFFFFFFF).sum() > 0.3 * len(smp)
    ok = (flat["band_primary"] == 0) & (inst["band_primary"] == 0)
    assert np.allclose(flat["rgb"][ok], inst["rgb"][ok], rtol=1e-9, atol=0)


@pytest.mark.parametrize("seed,frame", [(1, 2), (4, 5)])
def test_moved_instances_match_flat_on_moved_vertices(seed, frame):
    scene = sg.small_random_scene(seed, n_instances=14, width=96, height=72, ssaa=1, n_lights=2)
    o2w, world = moved(scene, frame)
    cam = scene.cameras[0]
    smp = np.arange(cam.n_samples)
    flat = O.OracleScene(world, scene.indices, scene.tri_material, scene.materials).render_point(
        cam, scene.point_lights, smp)
    inst = two_level(scene, o2w, world).render_point(cam, scene.point_lights, smp)
    band, n = compare_point(flat, inst, len(scene.point_lights))
    assert band < 0.02 * len(smp)
    # the motion matters: the rest-pose scene sees other triangles in many samples
    rest = O.OracleScene.from_scene(scene).render_point(cam, scene.point_lights, smp)
    assert (rest["hit_id"] != flat["hit_id"]).sum() > 50
    # area light: visible counts agree wherever no sample of the pixel is in either band
    pix = np.arange(0, cam.width * cam.height, 3)
    fr = O.OracleScene(world, scene.indices, scene.tri_material, scene.materials).render_rect(
        cam, scene.rect_light, 16, 1, pix)
    ir = two_level(scene, o2w, world).render_rect(cam, scene.rect_light, 16, 1, pix)
    ok = (fr["band_primary"] == 0) & (ir["band_primary"] == 0) & (fr["band_count"] == 0) & (ir["band_count"] == 0)
    assert ok.sum() > 0.9 * len(pix)
    assert np.array_equal(fr["hit_id"][ok], ir["hit_id"][ok])
    assert np.array_equal(fr["vis_count"][ok], ir["vis_count"][ok])


def test_instance_bvh_matches_brute_force():
    scene = sg.small_random_scene(6, n_instances=8, tris_lo=20, tris_hi=120, width=24, height=18, n_lights=2)
    o2w, world = moved(scene, 3, seed=2)
    cam = scene.cameras[0]
    smp = np.arange(cam.n_samples)
    a = two_level(scene, o2w, world).render_point(cam, scene.point_lights, smp)
    b = two_level(scene, o2w, world, use_bvh=False).render_point(cam, scene.point_lights, smp)
    for k in ("hit_id", "band_primary", "mask", "band_shadow"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["tuv"], b["tuv"]) and np.array_equal(a["rgb"], b["rgb"])


def test_transposed_rotation_is_caught():
    """Planted mistake: the instances get R^T in place of R; the flat comparison must fail."""
    scene = sg.small_random_scene(1, n_instances=14, width=40, height=30, ssaa=1, n_lights=1)
    o2w, world = moved(scene, 2)
    bad = o2w.reshape(-1, 3, 4).copy()
    bad[:, :, :3] = np.transpose(bad[:, :, :3], (0, 2, 1))
    cam = scene.cameras[0]
    smp = np.arange(cam.n_samples)
    flat = O.OracleScene(world, scene.indices, scene.tri_material, scene.materials).render_point(
        cam, scene.point_lights, smp)
    inst = two_level(scene, bad.reshape(-1, 12), world).render_point(cam, scene.point_lights, smp)
    ok = (flat["band_primary"] == 0) & (inst["band_primary"] == 0)
    assert (flat["hit_id"][ok] != inst["hit_id"][ok]).sum() > 20
