"""The binned-SAH build on the GPU (RC_BUILD_DEVICE_SAH): the same splits as the host build (same bins,
costs, leaf rule), so the 4-wide node arrays are equal word for word and each leaf holds the same triangles
(their order inside a leaf may differ: the GPU partitions stably); the usual tree invariants hold on degenerate
inputs; renders through the tree match the oracle."""
import sys
import time

import numpy as np
import pytest

from paper_2410_05095_amd import scenegen as sg
from tests.test_gpu_build import check_tree, tri_scene
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


def leaf_sets(nodes, order):
    child = nodes[:, 24:28].astype(np.int64)
    empty = child == 0xFFFFFFFF
    leaf = ((child & 0x80000000) != 0) & ~empty
    ni, ci = np.nonzero(leaf)
    w = child[ni, ci]
    first, cnt = w & 0x0FFFFFFF, ((w >> 28) & 7) + 1
    return {(int(a), int(b)): frozenset(order[f:f + c].tolist()) for a, b, f, c in zip(ni, ci, first, cnt)}


def same_as_host(ctx, scene_or_arrays, **kw):
    if isinstance(scene_or_arrays, tuple):
        pos, idx = scene_or_arrays
        host, _, _ = tri_scene(ctx, pos, idx)
        dev, _, _ = tri_scene(ctx, pos, idx)
    else:
        host, dev = ctx.scene_from(scene_or_arrays), ctx.scene_from(scene_or_arrays)
    host.build(**kw)
    dev.build(device_sah=True, **kw)
    hs, ds = host.stats(), dev.stats()
    hn, ho = host.export()
    dn, do = dev.export()
    host.close()
    dev.close()
    return hs, ds, hn, ho, dn, do


@pytest.mark.parametrize("seed,n_inst,max_leaf,bins", [(7, 40, 4, 32), (3, 60, 2, 16), (11, 90, 4, 64),
                                                      (5, 30, 1, 32)])
def test_device_sah_equals_host_build(ctx, seed, n_inst, max_leaf, bins):
    scene = sg.small_random_scene(seed, n_instances=n_inst, tris_lo=50, tris_hi=400, width=8, height=8)
    hs, ds, hn, ho, dn, do = same_as_host(ctx, scene, max_leaf=max_leaf, bins=bins)
    say(f"[sah gpu] seed={seed} tris={scene.n_tris} max_leaf={max_leaf} bins={bins}: SAH host {hs['sah_cost']:.6f} "
        f"device {ds['sah_cost']:.6f}, nodes {hs['n_nodes']} / {ds['n_nodes']}")
    check_tree(dn, do, scene.positions, scene.indices, max_leaf, ds)
    assert ds["n_nodes"] == hs["n_nodes"] and ds["depth"] == hs["depth"] and ds["n_leaves"] == hs["n_leaves"]
    assert abs(ds["sah_cost"] - hs["sah_cost"]) <= 1e-12 * hs["sah_cost"]
    assert np.array_equal(dn, hn)
    assert leaf_sets(dn, do) == leaf_sets(hn, ho)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 9, 17, 5000])
def test_device_sah_few_and_many_triangles(ctx, n):
    """Sizes around the leaf size, and above the size (1024) where ranges switch from level-wise splitting to
    one wave per range."""
    rng = np.random.default_rng(n)
    pos = rng.normal(size=(3 * n, 3)) * np.array([3.0, 1.0, 2.0])
    idx = np.arange(3 * n).reshape(n, 3)
    for max_leaf in (1, 4):
        hs, ds, hn, ho, dn, do = same_as_host(ctx, (pos, idx), max_leaf=max_leaf)
        check_tree(dn, do, pos.astype(np.float32), idx, max_leaf, ds)
        assert np.array_equal(dn, hn), (n, max_leaf)
        assert leaf_sets(dn, do) == leaf_sets(hn, ho)


def test_device_sah_degenerate_inputs(ctx):
    """Every centroid at one point (no split exists: ranges are halved) with 300 and with 9000 triangles, and a
    scene flat along z (one axis without extent)."""
    rng = np.random.default_rng(5)
    for n in (300, 9000):
        d = rng.normal(size=(n, 3)) * 0.1
        pos = np.stack([d, -d, np.zeros_like(d)], 1).reshape(-1, 3)
        idx = np.arange(3 * n).reshape(n, 3)
        gs, p, i = tri_scene(ctx, pos, idx)
        gs.build(device_sah=True)
        check_tree(*gs.export(), p, i, 4, gs.stats())
        say(f"[sah gpu] {n} coinciding centroids:", gs.stats())
        gs.close()
    pos = rng.uniform(-5, 5, (3 * 6000, 3))
    pos[:, 2] = 1.25
    idx = np.arange(3 * 6000).reshape(-1, 3)
    hs, ds, hn, ho, dn, do = same_as_host(ctx, (pos, idx), max_leaf=2)
    check_tree(dn, do, pos.astype(np.float32), idx, 2, ds)
    assert np.array_equal(dn, hn)


@pytest.mark.parametrize("seed,ssaa,w,h", [(0, 1, 37, 29), (2, 2, 64, 48)])
def test_device_sah_render_parity(ctx, oracle_mod, seed, ssaa, w, h):
    scene = sg.small_random_scene(seed, n_instances=30, width=w, height=h, ssaa=ssaa, n_lights=3)
    gs = ctx.scene_from(scene).build(device_sah=True)
    render_and_compare(ctx, oracle_mod, scene, scene.cameras[0], gs=gs)
    compare_rect(ctx, oracle_mod, scene, scene.cameras[0], 16, 1, gs=gs) if ssaa == 1 else None


def test_device_sah_big_scene(ctx, oracle_mod):
    """7.3M triangles: the GPU build gives the host build's nodes (same SAH) in a fraction of its time; 2000
    pixels of the 64-sample rect-light frame through it match the oracle."""
    import torch
    scene = sg.big_scene(0)
    host = ctx.scene_from(scene)
    t0 = time.perf_counter()
    host.build()
    t_host = time.perf_counter() - t0
    dev = ctx.scene_from(scene)
    t0 = time.perf_counter()
    dev.build(device_sah=True)
    t_dev = time.perf_counter() - t0
    hs, ds = host.stats(), dev.stats()
    say(f"[sah gpu big] host {t_host * 1e3:.0f} ms (build_ms {hs['build_ms']:.0f}), device {t_dev * 1e3:.0f} ms "
        f"(build_ms {ds['build_ms']:.1f}); SAH host {hs['sah_cost']:.4f} device {ds['sah_cost']:.4f}")
    assert abs(ds["sah_cost"] - hs["sah_cost"]) <= 1e-3 * hs["sah_cost"]
    hn, _ = host.export()
    dn, do = dev.export()
    host.close()
    say(f"[sah gpu big] node words equal: {np.array_equal(dn, hn)}; differing nodes "
        f"{int((dn != hn).any(axis=1).sum()) if dn.shape == hn.shape else 'shape'}")
    check_tree(dn, do, scene.positions, scene.indices, 4, ds)
    del hn, dn, do
    torch.cuda.empty_cache()
    cam = scene.cameras[0]
    rng = np.random.default_rng(2)
    pix = np.sort(rng.choice(cam.width * cam.height, 2000, replace=False))
    out, orc, s = compare_rect(ctx, oracle_mod, scene, cam, 64, 0, pixels=pix, gs=dev)
    assert s["band_primary"] < 0.01 * s["n"]
    dev.close()
