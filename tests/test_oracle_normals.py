"""Pins of the oracle's smooth shading normal (vertex normals interpolated with the hit's barycentrics).

Face normals given as vertex normals reproduce flat shading; on a tessellated unit sphere whose vertices
are their own normals the interpolated normal at a hit p is p / |p| (the radiance is recomputed here from
the BRDF with that normal); the rotation of normals by moved bodies is the FP32 definition."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_05095_amd import scenegen as sg


def unwelded(scene):
    """Every triangle with its own three vertices (same geometry, same ids)."""
    pos = scene.positions[scene.indices.reshape(-1)].reshape(-1, 3)
    idx = np.arange(3 * scene.n_tris, dtype=np.uint32).reshape(-1, 3)
    return pos, idx


def test_face_normals_reproduce_flat_shading():
    scene = sg.small_random_scene(3, n_instances=12, width=40, height=30, ssaa=2, n_lights=3)
    pos, idx = unwelded(scene)
    nrm = sg.vertex_normals(pos, idx)       # = the face normal of each triangle's own vertices
    cam = scene.cameras[0]
    smp = np.arange(cam.n_samples)
    flat = O.OracleScene(pos, idx, scene.tri_material, scene.materials).render_point(cam, scene.point_lights, smp)
    smooth = O.OracleScene(pos, idx, scene.tri_material, scene.materials, normals=nrm).render_point(
        cam, scene.point_lights, smp)
    assert np.array_equal(flat["hit_id"], smooth["hit_id"]) and np.array_equal(flat["mask"], smooth["mask"])
    L = flat["rgb"]
    rel = np.abs(smooth["rgb"] - L) / np.maximum(np.abs(L), 1e-6 * L.max())
    assert (flat["hit_id"] != 0xFFFFFFFF).sum() > 0.3 * len(smp)
    assert rel.max() < 2e-6      # only the FP32 rounding of the stored normals


def sphere_scene(subdiv, smooth):
    v, f = sg.icosphere(subdiv)
    pos = v.astype(np.float32)
    idx = f.astype(np.uint32)
    mats = np.array([[0.7, 0.6, 0.5, 0.6, 0.0]], np.float32)
    nrm = v.astype(np.float32) if smooth else None       # the exact sphere normal at each vertex
    return O.OracleScene(pos, idx, np.zeros(len(idx), np.uint32), mats, normals=nrm), mats[0]


def sphere_error(subdiv, smooth):
    cam = sg.Camera(eye=(0.4, 0.9, -3.0), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), vfov_deg=40.0,
                    width=64, height=64, ssaa=1)
    light = np.array([[2.0, 3.0, -2.5, 50.0, 50.0, 50.0]], np.float32)
    osc, mat = sphere_scene(subdiv, smooth)
    smp = np.arange(cam.n_samples)
    out = osc.render_point(cam, light, smp)
    o, d = O.gen_rays(cam, smp)
    hit = out["hit_id"] != 0xFFFFFFFF
    p = o.astype(np.float64) + d.astype(np.float64) * np.where(hit, out["tuv"][:, 0], 1.0)[:, None]
    n_exact = p / np.linalg.norm(p, axis=1, keepdims=True)
    wi = light[0, :3].astype(np.float64) - p
    d2 = (wi * wi).sum(1)
    wi /= np.sqrt(d2)[:, None]
    cos = (n_exact * wi).sum(1)
    sel = hit & (cos > 0.2) & (out["mask"] == 1)
    want = np.array([O.brdf(n_exact[k], -d[k].astype(np.float64), wi[k], mat[:3], mat[3], mat[4]) * 50.0 * cos[k] / d2[k]
                     for k in np.nonzero(sel)[0]])
    got = out["rgb"][sel]
    return float(np.mean(np.abs(got - want) / want)), int(sel.sum())


@pytest.mark.parametrize("subdiv", [2, 4])
def test_interpolated_sphere_normals_point_along_the_hit_point(subdiv):
    """The vertices of the tessellated unit sphere are their own normals, and a hit point is the same
    barycentric combination of the vertices, so the interpolated normal is p / |p| at every hit: the radiance
    equals the BRDF evaluated with that normal to the rounding of the stored normals, while flat shading is
    off by percents (a wrong barycentric weight would be too)."""
    es, n = sphere_error(subdiv, True)
    ef, _ = sphere_error(subdiv, False)
    assert n > 800
    assert es < 1e-7 and ef > 0.01


def test_rotation_of_normals_is_the_fp32_definition():
    scene = sg.with_vertex_normals(sg.small_random_scene(5, n_instances=8))
    anim = sg.RigidAnimation(scene, n_bodies=4, seed=2, max_disp=0.5, max_rot_deg=30.0)
    xf = anim.transforms(3)
    got = O.rotate_f32(scene.normals, scene.body_vertex_range, anim.body_ids, xf)
    want = scene.normals.copy()
    for b, M in zip(anim.body_ids, xf.reshape(-1, 3, 4)):
        f0, c0 = scene.body_vertex_range[b]
        n = scene.normals[f0:f0 + c0]
        a, bb, cc = M[:, 0] * n[:, 0:1], M[:, 1] * n[:, 1:2], M[:, 2] * n[:, 2:3]
        want[f0:f0 + c0] = (a + bb) + cc
        rot = n.astype(np.float64) @ M[:, :3].astype(np.float64).T
        assert np.abs(rot - got[f0:f0 + c0]).max() < 1e-6
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
