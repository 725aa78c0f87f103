"""The GPU BVH build (RC_BUILD_DEVICE_LBVH) through the C ABI: the tree it produces must satisfy the same
invariants as the host build (exact FP32 child boxes, every triangle in exactly one leaf of at most
max_leaf triangles, breadth-first levels with consistent parent links), and renders through it must
match the oracle exactly as with the host build."""
import sys
import time

import numpy as np
import pytest

from paper_2410_05095_amd import scenegen as sg
from tests.parity import bvh_bound_errors
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


def check_tree(nodes, order, pos, idx, max_leaf, stats):
    """Structure of an exported BVH; returns the leaf-size histogram."""
    n = len(idx)
    assert np.array_equal(np.sort(order), np.arange(n, dtype=np.uint32))
    bad, hist = bvh_bound_errors(nodes, order, pos, idx)
    assert bad == 0
    assert hist[max_leaf + 1:].sum() == 0 and hist.sum() == stats["n_leaves"]
    child = nodes[:, 24:28].astype(np.int64)
    parent = nodes[:, 28].astype(np.int64)
    level = nodes[:, 29].astype(np.int64)
    empty = child == 0xFFFFFFFF
    leaf = ((child & 0x80000000) != 0) & ~empty
    inner = ~leaf & ~empty
    # breadth-first: levels non-decreasing, the root alone at level 0, depth = number of levels
    assert level[0] == 0 and parent[0] == 0xFFFFFFFF and (np.diff(level) >= 0).all()
    assert stats["depth"] == level.max() + 1 and stats["max_stack"] == 3 * stats["depth"] + 1
    # every node but the root is the child of exactly one node, whose index and level it records
    ni, ci = np.nonzero(inner)
    w = child[ni, ci]
    assert np.array_equal(np.sort(w), np.arange(1, len(nodes)))
    assert (parent[w] == ni).all() and (level[w] == level[ni] + 1).all()
    # leaves cover every slot exactly once
    ni, ci = np.nonzero(leaf)
    first = child[ni, ci] & 0x0FFFFFFF
    cnt = ((child[ni, ci] >> 28) & 7) + 1
    cover = np.zeros(n + 1, np.int64)
    np.add.at(cover, first, 1)
    np.add.at(cover, first + cnt, -1)
    assert (np.cumsum(cover)[:n] == 1).all()
    # child slots are filled from the front
    assert not (empty[:, :-1] & ~empty[:, 1:]).any()
    return hist


@pytest.mark.parametrize("seed,max_leaf", [(7, 4), (7, 1), (3, 2), (11, 3)])
def test_device_build_structure(ctx, seed, max_leaf):
    scene = sg.small_random_scene(seed, n_instances=40, width=8, height=8)
    gs = ctx.scene_from(scene).build(max_leaf=max_leaf, device=True)
    nodes, order = gs.export()
    st = gs.stats()
    say(f"[lbvh] seed={seed} max_leaf={max_leaf} tris={scene.n_tris}", st)
    hist = check_tree(nodes, order, scene.positions, scene.indices, max_leaf, st)
    say("[lbvh] leaf sizes", hist.tolist())
    host = ctx.scene_from(scene).build(max_leaf=max_leaf).stats()
    say(f"[lbvh] SAH device {st['sah_cost']:.2f} host {host['sah_cost']:.2f}")
    assert st["sah_cost"] < 3.0 * host["sah_cost"]
    gs.close()


def tri_scene(ctx, pos, idx):
    pos = np.ascontiguousarray(pos, np.float32)
    idx = np.ascontiguousarray(idx, np.uint32)
    mats = np.array([[0.5, 0.5, 0.5, 0.5, 0.0]], np.float32)
    return ctx.scene(pos, idx, np.zeros(len(idx), np.uint32), mats), pos, idx


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 9, 17])
def test_device_build_few_triangles(ctx, n):
    rng = np.random.default_rng(n)
    pos = rng.normal(size=(3 * n, 3))
    idx = np.arange(3 * n).reshape(n, 3)
    for max_leaf in (1, 4):
        gs, p, i = tri_scene(ctx, pos, idx)
        gs.build(max_leaf=max_leaf, device=True)
        nodes, order = gs.export()
        check_tree(nodes, order, p, i, max_leaf, gs.stats())
        gs.close()


def test_device_build_duplicate_codes_and_flat_extent(ctx):
    """All centroids equal (every Morton code the same: the radix tree splits by position), and a scene
    with zero extent along z (one axis of the centroid bounds empty)."""
    rng = np.random.default_rng(5)
    n = 300
    d = rng.normal(size=(n, 3)) * 0.1
    pos = np.stack([d, -d, np.zeros_like(d)], 1).reshape(-1, 3)          # every centroid at the origin
    idx = np.arange(3 * n).reshape(n, 3)
    gs, p, i = tri_scene(ctx, pos, idx)
    gs.build(device=True)
    nodes, order = gs.export()
    st = gs.stats()
    check_tree(nodes, order, p, i, 4, st)
    say("[lbvh] equal codes", st)
    gs.close()
    pos = rng.uniform(-5, 5, (3 * 2000, 3))
    pos[:, 2] = 1.25
    gs, p, i = tri_scene(ctx, pos, np.arange(3 * 2000).reshape(-1, 3))
    gs.build(max_leaf=2, device=True)
    nodes, order = gs.export()
    check_tree(nodes, order, p, i, 2, gs.stats())
    gs.close()


def test_device_build_deterministic(ctx):
    scene = sg.small_random_scene(9, n_instances=60)
    a = ctx.scene_from(scene).build(device=True)
    b = ctx.scene_from(scene).build(device=True)
    na, oa = a.export()
    nb, ob = b.export()
    assert np.array_equal(na, nb) and np.array_equal(oa, ob)
    a.close()
    b.close()


@pytest.mark.parametrize("seed,ssaa,w,h", [(0, 1, 37, 29), (2, 2, 64, 48)])
def test_device_build_render_parity(ctx, oracle_mod, seed, ssaa, w, h):
    scene = sg.small_random_scene(seed, n_instances=30, width=w, height=h, ssaa=ssaa, n_lights=3)
    render_and_compare(ctx, oracle_mod, scene, scene.cameras[0], device_build=True)


@pytest.mark.parametrize("seed,N,stream", [(0, 16, 0), (6, 64, 4)])
def test_device_build_rect_parity(ctx, oracle_mod, seed, N, stream):
    scene = sg.small_random_scene(seed, n_instances=40, width=40, height=32, ssaa=1)
    compare_rect(ctx, oracle_mod, scene, scene.cameras[0], N, stream, device_build=True)


def test_device_build_refit(ctx, oracle_mod):
    """Refit keeps working on a device-built tree: boxes exact after rigid motion."""
    import torch
    O = oracle_mod
    scene = sg.small_random_scene(4, n_instances=30)
    gs = ctx.scene_from(scene).build(device=True)
    anim = sg.RigidAnimation(scene, n_bodies=10, seed=2, max_disp=0.5, max_rot_deg=20.0)
    xf = anim.transforms(3)
    gs.set_transforms(torch.from_numpy(xf).cuda(), torch.from_numpy(anim.body_ids.astype(np.int32)).cuda())
    gs.refit()
    torch.cuda.synchronize()
    want = O.transform_f32(scene.positions, scene.body_vertex_range, anim.body_ids, xf)
    nodes, order = gs.export()
    assert bvh_bound_errors(nodes, order, want, scene.indices)[0] == 0
    gs.close()


def test_device_build_big_scene(ctx, oracle_mod):
    """7.3M triangles: the device-built tree is exact, and 2000 pixels of the 64-sample rect-light frame
    match the oracle."""
    import torch
    scene = sg.big_scene(0)
    gs = ctx.scene_from(scene)
    t0 = time.perf_counter()
    gs.build(device=True)
    dt = time.perf_counter() - t0
    st = gs.stats()
    say(f"[lbvh big] wall {dt * 1e3:.1f} ms", st)
    nodes, order = gs.export()
    check_tree(nodes, order, scene.positions, scene.indices, 4, st)
    gs.close()
    del nodes, order
    torch.cuda.empty_cache()
    cam = scene.cameras[0]
    rng = np.random.default_rng(2)
    pix = np.sort(rng.choice(cam.width * cam.height, 2000, replace=False))
    out, orc, s = compare_rect(ctx, oracle_mod, scene, cam, 64, 0, pixels=pix, device_build=True)
    assert s["band_primary"] < 0.01 * s["n"]
