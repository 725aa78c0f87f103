"""The two-level acceleration structure (RC_BUILD_TWO_LEVEL) through the C ABI against the oracle's
instanced queries: one bottom-level tree per body over rest positions, a top level over the bodies'
world boxes rebuilt from their rigid maps, rays mapped into each body.

Structure: instance maps bit-exact against the FP32 definition, exact bottom-level boxes, every body in
exactly one top-level leaf whose box holds the body's mapped vertices.  Renders (camera rays, point-light
and rect-light shadows, both rect kernels) match the two-level oracle exactly outside its FP32 band, for
bodies at rest and moved; a top level rebuilt on a second stream gives the same frame."""
import sys

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


def identity_o2w(n):
    x = np.zeros((n, 12), np.float32)
    x[:, 0] = x[:, 5] = x[:, 10] = 1.0
    return x


def move(gs, scene, frame, n_bodies=None, seed=1, max_disp=0.6, max_rot=25.0):
    """Move bodies on the GPU (transform + recorded maps); returns (o2w of all bodies, world positions)."""
    import torch
    from oracle import oracle as O
    nb = len(scene.body_tri_range)
    anim = sg.RigidAnimation(scene, n_bodies=n_bodies or nb // 2, seed=seed, max_disp=max_disp, max_rot_deg=max_rot)
    xf = anim.transforms(frame)
    gs.set_transforms(torch.from_numpy(xf).cuda(), torch.from_numpy(anim.body_ids.astype(np.int32)).cuda())
    torch.cuda.synchronize()
    o2w = identity_o2w(nb)
    o2w[anim.body_ids] = xf
    world = O.transform_f32(scene.positions, scene.body_vertex_range, anim.body_ids, xf)
    return o2w, world


def oracle_two_level(O, scene, o2w, world):
    return O.OracleScene.two_level(world, scene.positions, scene.indices, scene.tri_material, scene.materials,
                                   scene.body_tri_range, o2w)


def check_structure(gs, scene, o2w, world, max_leaf=4):
    from oracle import oracle as O
    st = gs.stats()
    nodes, order = gs.export()
    inst = gs.tlas_export()
    nb = len(scene.body_tri_range)
    root = int(st["tlas_root"])
    assert st["n_instances"] == nb and nodes.shape[0] == st["n_nodes"]
    # instance records: the FP32 world-to-object maps, bit for bit, and body b's tree rooted at node b
    assert np.array_equal(inst[:, :12].view(np.uint32), O.w2o_f32(o2w).view(np.uint32))
    assert np.array_equal(inst[:, 12].view(np.uint32), np.arange(nb, dtype=np.uint32))
    # bottom levels: exact boxes over rest positions, leaves of body b inside its own triangle range
    blas = nodes[:root]
    bad, hist = bvh_bound_errors(blas, order, scene.positions, scene.indices)
    assert bad == 0 and hist[max_leaf + 1:].sum() == 0
    assert np.array_equal(np.sort(order), np.arange(scene.n_tris, dtype=np.uint32))
    rng = scene.body_tri_range.astype(np.int64)
    for b in range(nb):
        lo, hi = rng[b, 0], rng[b, 0] + rng[b, 1]
        assert ((order[lo:hi] >= lo) & (order[lo:hi] < hi)).all()
    # body b's tree (from node b) reaches exactly the slots of its own triangle range, each once
    child_all = blas[:, 24:28].astype(np.int64)
    for b in range(nb):
        cover = np.zeros(scene.n_tris, np.int64)
        todo = [b]
        while todo:
            nd = todo.pop()
            for w in child_all[nd]:
                if w == 0xFFFFFFFF:
                    continue
                if w & 0x80000000:
                    f0, c0 = w & 0x0FFFFFFF, ((w >> 28) & 7) + 1
                    cover[f0:f0 + c0] += 1
                else:
                    assert nb <= w < root, (b, nd, w)
                    todo.append(int(w))
        lo, hi = rng[b, 0], rng[b, 0] + rng[b, 1]
        assert (cover[lo:hi] == 1).all() and cover[:lo].sum() == 0 and cover[hi:].sum() == 0, b
    # top level: each body in exactly one leaf, and that leaf's box holds the body's mapped vertices
    tl = nodes[root:]
    f = tl.view(np.float32)
    child = tl[:, 24:28]
    empty = child == 0xFFFFFFFF
    leaf = ((child & 0x80000000) != 0) & ~empty
    ni, ci = np.nonzero(leaf)
    body = (child[ni, ci] & 0x0FFFFFFF).astype(np.int64)
    assert np.array_equal(np.sort(body), np.arange(nb)) and (((child[ni, ci] >> 28) & 7) == 0).all()
    vr = scene.body_vertex_range.astype(np.int64)
    X = o2w.reshape(-1, 3, 4).astype(np.float64)
    for n_, c_, b in zip(ni, ci, body):
        v = scene.positions[vr[b, 0]:vr[b, 0] + vr[b, 1]].astype(np.float64) @ X[b, :, :3].T + X[b, :, 3]
        lo = np.array([f[n_, 0 + c_], f[n_, 8 + c_], f[n_, 16 + c_]])
        hi = np.array([f[n_, 4 + c_], f[n_, 12 + c_], f[n_, 20 + c_]])
        assert (v >= lo).all() and (v <= hi).all(), b
    # internal top-level children: exact unions of their child boxes
    ni, ci = np.nonzero(~leaf & ~empty)
    w = child[ni, ci].astype(np.int64) - root
    assert (w > 0).all() and (w < len(tl)).all()
    for k, (lo_off, hi_off) in enumerate(((0, 4), (8, 12), (16, 20))):
        cl = np.where(empty[w], np.inf, f[w, lo_off:lo_off + 4]).min(1)
        ch = np.where(empty[w], -np.inf, f[w, hi_off:hi_off + 4]).max(1)
        assert np.array_equal(f[ni, lo_off + ci], cl) and np.array_equal(f[ni, hi_off + ci], ch)
    return st


@pytest.mark.parametrize("seed,max_leaf", [(7, 4), (2, 1)])
def test_two_level_structure(ctx, seed, max_leaf):
    scene = sg.small_random_scene(seed, n_instances=40, width=8, height=8)
    gs = ctx.scene_from(scene).build(max_leaf=max_leaf, two_level=True)
    nb = len(scene.body_tri_range)
    st = check_structure(gs, scene, identity_o2w(nb), scene.positions, max_leaf)
    say(f"[two-level] seed={seed} rest", st)
    o2w, world = move(gs, scene, 3)
    gs.refit()
    st = check_structure(gs, scene, o2w, world, max_leaf)
    say(f"[two-level] seed={seed} moved", st)
    gs.close()


def test_two_level_single_body_and_tiny_bodies(ctx):
    """One body (a top level with one leaf), and bodies of one triangle."""
    from paper_2410_05095_amd import _native as N
    rng = np.random.default_rng(3)
    pos = rng.normal(size=(9, 3)).astype(np.float32)
    idx = np.arange(9, dtype=np.uint32).reshape(3, 3)
    mats = np.array([[0.5, 0.5, 0.5, 0.5, 0.0]], np.float32)
    for vr in (np.array([[0, 9]], np.uint32), np.array([[0, 3], [3, 3], [6, 3]], np.uint32)):
        gs = ctx.scene(pos, idx, np.zeros(3, np.uint32), mats, body_vertex_range=vr).build(two_level=True)
        sc = sg.Scene(pos, idx, np.zeros(3, np.uint32), mats, vr,
                      np.array([[0, 3]] if len(vr) == 1 else [[0, 1], [1, 1], [2, 1]], np.uint32),
                      np.zeros((0, 6), np.float32), None, [], "tiny")
        check_structure(gs, sc, identity_o2w(len(vr)), pos)
        gs.close()
    # a triangle shared between two bodies is rejected
    bad = np.array([[0, 4], [4, 5]], np.uint32)
    with pytest.raises(N.RcError) as e:
        ctx.scene(pos, idx, np.zeros(3, np.uint32), mats, body_vertex_range=bad).build(two_level=True)
    assert e.value.status == -2


@pytest.mark.parametrize("seed,ssaa,w,h,frame", [(0, 1, 37, 29, 0), (2, 2, 48, 36, 3), (5, 1, 64, 40, 5)])
def test_two_level_point_parity(ctx, oracle_mod, seed, ssaa, w, h, frame):
    O = oracle_mod
    scene = sg.small_random_scene(seed, n_instances=30, width=w, height=h, ssaa=ssaa, n_lights=3)
    gs = ctx.scene_from(scene).build(two_level=True)
    nb = len(scene.body_tri_range)
    o2w, world = identity_o2w(nb), scene.positions
    if frame:
        o2w, world = move(gs, scene, frame)
        gs.refit()
    osc = oracle_two_level(O, scene, o2w, world)
    render_and_compare(ctx, O, scene, scene.cameras[0], gs=gs, osc=osc)
    gs.close()


@pytest.mark.parametrize("seed,N,stream,frame", [(0, 16, 0, 0), (6, 64, 4, 4), (3, 7, 2, 2), (4, 130, 1, 6)])
def test_two_level_rect_parity(ctx, oracle_mod, seed, N, stream, frame):
    O = oracle_mod
    scene = sg.small_random_scene(seed, n_instances=40, width=40, height=32, ssaa=1)
    gs = ctx.scene_from(scene).build(two_level=True)
    nb = len(scene.body_tri_range)
    o2w, world = identity_o2w(nb), scene.positions
    if frame:
        o2w, world = move(gs, scene, frame)
        gs.refit()
    osc = oracle_two_level(O, scene, o2w, world)
    compare_rect(ctx, O, scene, scene.cameras[0], N, stream, gs=gs, osc=osc)
    gs.close()


def test_two_level_rebuild_on_second_stream(ctx):
    """The top level rebuilt on a side stream (ordered by events) renders the same frame as one rebuilt on
    the context stream."""
    import torch
    scene = sg.small_random_scene(8, n_instances=40, width=64, height=48, ssaa=1)
    cam = scene.cameras[0]
    kw = dict(rect=scene.rect_light, area_samples=64, area_stream=0)
    a = ctx.scene_from(scene).build(two_level=True)
    b = ctx.scene_from(scene).build(two_level=True)
    outs = []
    side = torch.cuda.Stream()
    for frame in (1, 2, 3):
        move(a, scene, frame)
        a.refit()
        ra = ctx.render(a, cam, (), **kw)
        ra = {k: v.clone() for k, v in ra.items()}
        move(b, scene, frame)
        ev = torch.cuda.Event()
        ev.record()
        side.wait_event(ev)
        b.tlas_rebuild(stream=side)
        done = torch.cuda.Event()
        done.record(side)
        torch.cuda.current_stream().wait_event(done)
        rb = ctx.render(b, cam, (), **kw)
        torch.cuda.synchronize()
        assert ctx.last_error() == 0
        for k in ra:
            assert torch.equal(ra[k], rb[k]), (frame, k)
        outs.append(float(ra["visibility"].float().mean()))
    say("[two-level side stream] mean visibility per frame", outs)
    a.close()
    b.close()


def test_two_level_big_scene_sampled(ctx, oracle_mod):
    """7.3M triangles in 1501 bodies, 300 of them moved: 1500 pixels of the 64-sample rect-light frame
    against the two-level oracle."""
    import time
    O = oracle_mod
    scene = sg.big_scene(0)
    cam = scene.cameras[0]
    gs = ctx.scene_from(scene)
    t0 = time.perf_counter()
    gs.build(two_level=True)
    say(f"[two-level big] build wall {(time.perf_counter() - t0) * 1e3:.1f} ms", gs.stats())
    o2w, world = move(gs, scene, 2, n_bodies=300, seed=3, max_disp=0.3, max_rot=10.0)
    gs.refit()
    osc = oracle_two_level(O, scene, o2w, world)
    rng = np.random.default_rng(4)
    pix = np.sort(rng.choice(cam.width * cam.height, 1500, replace=False))
    out, orc, s = compare_rect(ctx, O, scene, cam, 64, 0, pixels=pix, gs=gs, osc=osc)
    assert s["band_primary"] < 0.01 * s["n"]
    gs.close()
