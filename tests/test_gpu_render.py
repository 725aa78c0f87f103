"""GPU parity of the rendering path (through the C ABI) against the CPU oracle."""
import sys

import numpy as np
import pytest

from paper_2410_05095_amd import scenegen as sg
from tests.parity import NO_HIT, assert_clean, compare_point, to_np

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


def render_and_compare(ctx, O, scene, cam, rtol=1e-4, sample_idx=None, brute=False, device_build=False, gs=None,
                       osc=None):
    """Render with per-lane traversal, with the wave-uniform kernels forced, and with the library's own
    choice, and check each against one oracle run.  gs / osc: an already built GPU scene / oracle scene to use
    instead."""
    import torch
    say(f"[render] {scene.name} {cam.width}x{cam.height} ssaa={cam.ssaa} tris={scene.n_tris} "
        f"build={'given' if gs is not None else ('device' if device_build else 'host')}")
    if gs is None:
        gs = ctx.scene_from(scene).build(device=device_build)
    n = cam.n_samples
    smp = np.arange(n) if sample_idx is None else np.asarray(sample_idx)
    if osc is None:
        osc = O.OracleScene.from_scene(scene, use_bvh=not brute)
    orc = osc.render_point(cam, scene.point_lights, smp, brute=brute)
    for mode, kw in (("per-lane", dict(per_lane=True)), ("wave", dict(wave=True)), ("auto", {})):
        out = ctx.render(gs, cam, scene.point_lights, sample_rgba=True, **kw)
        torch.cuda.synchronize()
        assert ctx.last_error() == 0
        hit = to_np(out["hit"])[smp]
        mask = to_np(out["shadow"])[smp] if len(scene.point_lights) else None
        srgba = to_np(out["sample_rgba"])[smp]
        st = compare_point(hit, mask, srgba, orc, len(scene.point_lights), rtol=rtol)
        say("[parity]", mode, st)
        assert_clean(st)
    # resolve: bit-exact against the fixed FP32 order applied to the GPU's own samples
    spp = cam.ssaa ** 2
    want = O.resolve_f32(to_np(out["sample_rgba"]).reshape(-1, spp, 4), spp)
    got = to_np(out["rgba"]).reshape(-1, 4)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    return out, orc, st, gs


def test_camera_rays_bit_exact(ctx, oracle_mod):
    O = oracle_mod
    cams = [sg.tiny_box_scene(0).cameras[0],
            sg.Camera(eye=(0.0, 10.0, -28.0), target=(0.0, 5.0, 0.0), up=(0, 1, 0), vfov_deg=50.0,
                      width=333, height=197, ssaa=2, seed=11, frame=3),
            sg.Camera(eye=(1.5, -2.0, 7.25), target=(-3.0, 0.5, 1.0), up=(0.1, 1, 0.2), vfov_deg=71.5,
                      width=64, height=1, ssaa=1)]
    for cam in cams:
        o, d = ctx.camera_rays(cam)
        oo, od = O.gen_rays(cam, np.arange(cam.n_samples))
        go, gd = to_np(o), to_np(d)
        say(f"[rays] {cam.width}x{cam.height} ssaa={cam.ssaa}: dir mismatches "
            f"{int((gd.view(np.uint32) != od.view(np.uint32)).any(axis=1).sum())}")
        assert np.array_equal(go.view(np.uint32), oo.view(np.uint32))
        assert np.array_equal(gd.view(np.uint32), od.view(np.uint32))


def test_tiny_box_full_frame(ctx, oracle_mod):
    scene = sg.tiny_box_scene(0)
    out, orc, st, _ = render_and_compare(ctx, oracle_mod, scene, scene.cameras[0], brute=True)
    assert st["clean"] > 0.95 * st["n"]
    # the box interior: every ray hits something
    assert (to_np(out["hit"])[:, 0].view(np.uint32) != NO_HIT).all()


@pytest.mark.parametrize("seed,ssaa,w,h,ninst", [(0, 1, 37, 29, 8), (1, 2, 41, 23, 12), (2, 2, 67, 45, 30),
                                                   (3, 1, 130, 71, 60)])
def test_small_scenes_full_frame(ctx, oracle_mod, seed, ssaa, w, h, ninst):
    scene = sg.small_random_scene(seed, n_instances=ninst, width=w, height=h, ssaa=ssaa, n_lights=1 + seed)
    render_and_compare(ctx, oracle_mod, scene, scene.cameras[0])


def test_city_full_size_sampled(ctx, oracle_mod):
    """The 1.1M-triangle scene at 1920x1080 with 2x2 samples and 4 point lights: the whole frame is
    rendered in the benchmark's configuration; 30000 samples are checked against the oracle."""
    scene = sg.city_scene(0)
    cam = scene.cameras[0]
    rng = np.random.default_rng(0)
    smp = np.sort(rng.choice(cam.n_samples, 30000, replace=False))
    out, orc, st, gs = render_and_compare(ctx, oracle_mod, scene, cam, sample_idx=smp)
    assert st["clean"] > 0.9 * st["n"]
    hits = (orc["hit_id"] != NO_HIT).sum()
    assert hits > 10000


def test_bvh_invariants(ctx):
    scene = sg.small_random_scene(7, n_instances=40, width=8, height=8)
    gs = ctx.scene_from(scene).build()
    nodes, order = gs.export()
    st = gs.stats()
    say("[bvh]", st)
    assert sorted(order.tolist()) == list(range(scene.n_tris))
    f = nodes.view(np.float32)
    boxes = f[:, :24].reshape(-1, 6, 4)          # lo_x hi_x lo_y hi_y lo_z hi_z  x 4 children
    child = nodes[:, 24:28]
    pos = scene.positions
    seen = np.zeros(scene.n_tris, int)
    for ni in range(len(nodes)):
        for c in range(4):
            w = int(child[ni, c])
            if w == 0xFFFFFFFF:
                continue
            lo = boxes[ni, [0, 2, 4], c]
            hi = boxes[ni, [1, 3, 5], c]
            if w & 0x80000000:
                first, cnt = w & 0x0FFFFFFF, ((w >> 28) & 7) + 1
                assert cnt <= 4
                tris = order[first:first + cnt]
                seen[tris] += 1
                v = pos[scene.indices[tris].ravel()]
                assert np.array_equal(v.min(0), lo) and np.array_equal(v.max(0), hi)
            else:
                cb = boxes[w]
                valid = child[w] != 0xFFFFFFFF
                assert np.array_equal(cb[[0, 2, 4]][:, valid].min(1), lo)
                assert np.array_equal(cb[[1, 3, 5]][:, valid].max(1), hi)
    assert (seen == 1).all()
    assert st["depth"] >= 2 and st["max_stack"] == 3 * st["depth"] + 1


def test_render_deterministic(ctx):
    import torch
    scene = sg.small_random_scene(4, n_instances=30, width=96, height=64, ssaa=2, n_lights=3)
    gs = ctx.scene_from(scene).build()
    a = ctx.render(gs, scene.cameras[0], scene.point_lights)
    a = {k: v.clone() for k, v in a.items()}
    b = ctx.render(gs, scene.cameras[0], scene.point_lights)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_render_error_paths(ctx):
    from paper_2410_05095_amd import _native as N
    scene = sg.small_random_scene(1, n_instances=3, width=8, height=8)
    gs = ctx.scene_from(scene)
    with pytest.raises(N.RcError) as e:
        ctx.render(gs, scene.cameras[0], scene.point_lights)
    assert e.value.status == -5   # not built
    gs.build()
    bad = sg.Camera(eye=(0, 0, 0), target=(0, 0, 1), up=(0, 1, 0), vfov_deg=50, width=8, height=8, ssaa=3)
    with pytest.raises(N.RcError) as e:
        ctx.render(gs, bad, scene.point_lights)
    assert e.value.status == -8
    with pytest.raises(N.RcError) as e:
        ctx.scene(scene.positions * np.nan, scene.indices, scene.tri_material, scene.materials)
    assert e.value.status == -2
    with pytest.raises(N.RcError) as e:   # per-lane and wave-uniform kernels both forced
        ctx.render(gs, scene.cameras[0], scene.point_lights, per_lane=True, wave=True)
    assert e.value.status == -1
    assert ctx.last_error() == 0


def test_default_kernels_small_and_large_passes(ctx):
    """The library traces small shadow passes one ray per lane and large ones wave-uniformly: a small frame
    in the default mode equals the per-lane render bit for bit; rect-light frames above the ray threshold
    equal the forced wave-uniform render."""
    import dataclasses
    import torch
    scene = sg.small_random_scene(6, n_instances=40, width=96, height=64, n_lights=2)
    gs = ctx.scene_from(scene).build()
    cam = scene.cameras[0]
    rect = scene.rect_light
    cases = [(cam, dict(lights=scene.point_lights)), (cam, dict(rect=rect, area_samples=4, area_stream=0))]
    big = dataclasses.replace(cam, width=512, height=384)
    cases.append((big, dict(rect=rect, area_samples=16, area_stream=1)))   # 3.1M rays: the wave kernels
    for i, (c, kw) in enumerate(cases):
        res = {}
        for mode, extra in (("auto", {}), ("lane", dict(per_lane=True)), ("wave", dict(wave=True))):
            o = ctx.render(gs, c, shade=False, **kw, **extra)
            torch.cuda.synchronize()
            res[mode] = {k: v.clone() for k, v in o.items() if k in ("hit", "shadow", "visibility") and v is not None}
        want = "wave" if i == 2 else "lane"
        say(f"[kernels] case {i} {c.width}x{c.height}: default = {want}")
        for k in res["auto"]:
            assert torch.equal(res["auto"][k], res[want][k]), (i, k)
    assert ctx.last_error() == 0


def test_shade_rejects_foreign_hit_ids(ctx):
    """rc_shade and rc_pack_features take a caller's G-buffer: an id at or beyond the scene's triangle count
    (a buffer from a larger scene) is shaded and packed as a miss, and the context reports
    RC_ERR_INVALID_VALUE; the other pixels are unchanged.  rc_shade validates lights like rc_render."""
    import torch
    from paper_2410_05095_amd import _native as N
    scene = sg.small_random_scene(4, n_instances=4, width=16, height=12, ssaa=1)
    cam = scene.cameras[0]
    gs = ctx.scene_from(scene).build()
    out = ctx.render(gs, cam, scene.point_lights, rect=scene.rect_light, area_samples=4, area_stream=0)
    torch.cuda.synchronize()
    assert ctx.last_error() == 0
    ref = out["rgba"].clone()
    hit = out["hit"].view(torch.int32).view(-1, 4)
    ids = hit[:, 0].cpu().numpy().view(np.uint32)
    victim = int(np.nonzero(ids != 0xFFFFFFFF)[0][0])
    for bad_id in (scene.n_tris, 0x7FFFFFF0):
        hit[victim, 0] = int(np.array(bad_id, np.uint32).view(np.int32))
        ctx.shade(gs, cam, out, lights=scene.point_lights, rect=scene.rect_light)
        torch.cuda.synchronize()
        assert ctx.last_error() == -2, bad_id
        got = out["rgba"].cpu().numpy().reshape(-1, 4)
        want = ref.cpu().numpy().reshape(-1, 4)
        assert np.all(got[victim] == 0.0)
        others = np.arange(len(got)) != victim
        assert np.array_equal(got[others], want[others])
        feat = N.pack_features(ctx, gs, cam, out, depth_norm=60.0)
        torch.cuda.synchronize()
        assert ctx.last_error() == -2
        f = feat.float().cpu().numpy().reshape(-1, 8)
        assert np.array_equal(f[victim], np.array([1, 1, 0, 0, 0, 0, 0, 0], np.float32))
    assert ctx.last_error() == 0      # the flag was cleared when read
    lights = np.array(scene.point_lights, np.float32).copy()
    lights[0, 0] = np.nan
    with pytest.raises(N.RcError) as e:
        ctx.shade(gs, cam, out, lights=lights)
    assert e.value.status == -2


def test_render_without_shading_then_shade(ctx):
    """RC_FLAG_NO_SHADE: rc_render stops after the visibility stages and leaves the image untouched; rc_shade on
    its G-buffer, masks and visibility then gives the image of a full rc_render bit for bit (point lights with
    2x2 samples, and a rect light at 1 sample per pixel, the learned path's configuration)."""
    import torch
    for ssaa, use_rect in ((2, False), (1, True)):
        scene = sg.small_random_scene(6, n_instances=5, width=24, height=18, ssaa=ssaa)
        cam = scene.cameras[0]
        gs = ctx.scene_from(scene).build()
        lights = () if use_rect else scene.point_lights
        rect = scene.rect_light if use_rect else None
        kw = dict(rect=rect, area_samples=1 if use_rect else 0, area_stream=0)
        full = ctx.render(gs, cam, lights, **kw)
        part = ctx.render(gs, cam, lights, shade=False, **kw)
        part["rgba"].fill_(7.0)
        torch.cuda.synchronize()
        assert torch.all(part["rgba"] == 7.0)
        ctx.render(gs, cam, lights, out=part, shade=False, **kw)
        torch.cuda.synchronize()
        assert torch.all(part["rgba"] == 7.0), "the image was written without shading"
        assert torch.equal(part["hit"], full["hit"])
        ctx.shade(gs, cam, part, lights=lights, rect=rect)
        torch.cuda.synchronize()
        assert ctx.last_error() == 0
        assert torch.equal(part["rgba"], full["rgba"]), (ssaa, use_rect)


def compare_rect(ctx, O, scene, cam, N, stream, pixels=None, device_build=False, gs=None, osc=None):
    """Both rect-light kernels (wave-uniform traversal, the default; per-lane stacks)
    against one oracle run: hit ids and visible-sample counts exact outside the FP32 band, radiance within
    1e-4.  gs / osc: an already built GPU scene / oracle scene to use instead."""
    import torch
    say(f"[rect] {scene.name} {cam.width}x{cam.height} N={N} tris={scene.n_tris} "
        f"build={'given' if gs is not None else ('device' if device_build else 'host')}")
    if gs is None:
        gs = ctx.scene_from(scene).build(device=device_build)
    outs = {}
    for per_lane in (False, True):
        outs[per_lane] = ctx.render(gs, cam, (), rect=scene.rect_light, area_samples=N, area_stream=stream,
                                    sample_rgba=True, per_lane=per_lane, wave=not per_lane)
        torch.cuda.synchronize()
        assert ctx.last_error() == 0
    npix = cam.width * cam.height
    pix = np.arange(npix) if pixels is None else np.asarray(pixels)
    if osc is None:
        osc = O.OracleScene.from_scene(scene)
    orc = osc.render_rect(cam, scene.rect_light, N, stream, pix)
    bp = orc["band_primary"].astype(bool)
    ok = ~bp
    exact = ok & (orc["band_count"] == 0)
    cnts = {}
    for per_lane, out in outs.items():
        hit = to_np(out["hit"]).view(np.uint32)[pix]
        vis = to_np(out["visibility"]).reshape(-1)[pix]
        cnt = np.rint(vis.astype(np.float64) * N).astype(np.int64)
        cnts[per_lane] = cnt
        assert np.array_equal(cnt.astype(np.float32) / np.float32(N), vis)
        assert (hit[ok, 0] != orc["hit_id"][ok]).sum() == 0
        diff = np.abs(cnt - orc["vis_count"])
        assert (diff[ok] <= orc["band_count"][ok]).all()
        assert (diff[exact] == 0).all()
        # radiance = unshadowed centre-point term times the GPU visibility
        want = orc["rgb_unshadowed"] * vis[:, None].astype(np.float64)
        got = to_np(out["sample_rgba"])[pix, :3].astype(np.float64)
        lmax = max(float(want.max()), 1e-30)
        rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-6 * lmax)
        st = {"kernel": "per-lane" if per_lane else "wave", "n": len(pix), "band_primary": int(bp.sum()),
              "band_rays": int(orc["band_count"][ok].sum()),
              "pix_with_band_rays": int((orc["band_count"][ok] > 0).sum()), "rgb_max_rel": float(rel[ok].max()),
              "mean_V": float(vis[ok & (orc["hit_id"] != NO_HIT)].mean())}
        say("[rect parity]", st)
        assert st["rgb_max_rel"] <= 1e-4
    # the two kernels can differ only where a ray of the pixel is in the band
    kdiff = cnts[False] != cnts[True]
    say(f"[rect] pixels where the two kernels differ: {int(kdiff.sum())} (all with band rays)")
    assert not (kdiff & exact).any()
    return outs[False], orc, st


@pytest.mark.parametrize("seed,w,h,N,stream", [(0, 48, 40, 16, 0), (5, 61, 33, 7, 3), (3, 40, 24, 1, 1),
                                               (4, 20, 16, 130, 2), (6, 24, 20, 64, 4)])
def test_rect_light_small(ctx, oracle_mod, seed, w, h, N, stream):
    scene = sg.small_random_scene(seed, n_instances=40, width=w, height=h, ssaa=1)
    out, orc, st = compare_rect(ctx, oracle_mod, scene, scene.cameras[0], N, stream)
    assert 0.0 < st["mean_V"] < 1.0


def deep_scene(n=300, ratio=0.8):
    """A ground square and n triangles shrinking geometrically (factor `ratio`) towards a point above it:
    binned SAH gives a tree of depth 31, so the wave kernel's traversal stack needs its second register
    (3 x depth + 1 > 64 entries)."""
    tris = [[(-4, 0, -4), (4, 0, -4), (4, 0, 4)], [(-4, 0, -4), (4, 0, 4), (-4, 0, 4)]]
    for k in range(n):
        s = ratio ** k
        c = np.array([0.6 * s, 0.3 + 0.4 * s, 0.05 * s])
        tris.append([c + (-0.4 * s, 0, -0.4 * s), c + (0.4 * s, 0, -0.3 * s), c + (0.0, 0.0, 0.45 * s)])
    pos = np.asarray(tris, np.float32).reshape(-1, 3)
    nt = len(pos) // 3
    cam = sg.Camera(eye=(0.9, 1.4, -1.6), target=(0.1, 0.1, 0.1), up=(0.0, 1.0, 0.0), vfov_deg=50.0,
                    width=40, height=30, ssaa=1)
    rect = sg.RectLight(center=(0.1, 2.5, 0.1), edge_u=(1.0, 0.0, 0.0), edge_v=(0.0, 0.0, 1.0),
                        radiance=(40.0, 40.0, 40.0))
    return sg.Scene(positions=pos, indices=np.arange(3 * nt, dtype=np.uint32).reshape(nt, 3),
                    tri_material=np.zeros(nt, np.uint32), materials=np.array([[0.7, 0.6, 0.5, 0.4, 0.0]], np.float32),
                    body_vertex_range=np.array([[0, len(pos)]], np.uint32),
                    body_tri_range=np.array([[0, nt]], np.uint32), point_lights=np.zeros((0, 6), np.float32),
                    rect_light=rect, cameras=[cam], name="deep")


def test_rect_light_deep_tree(ctx, oracle_mod):
    """The wave kernel with its two-register stack (a flat tree deeper than 21 levels)."""
    scene = deep_scene()
    gs = ctx.scene_from(scene).build()
    depth = gs.stats()["depth"]
    say(f"[rect deep] depth {depth}, stack bound {3 * depth + 1}")
    assert 3 * depth + 1 > 64
    out, orc, st = compare_rect(ctx, oracle_mod, scene, scene.cameras[0], 64, 1, gs=gs)
    assert 0.0 < st["mean_V"] < 1.0
    gs.close()


def test_rect_light_big_scene_sampled(ctx, oracle_mod):
    """7.3M triangles at 1920x1080 with 64 light samples per pixel (the benchmark's plain path):
    4000 pixels checked against the oracle."""
    scene = sg.big_scene(0)
    cam = scene.cameras[0]
    rng = np.random.default_rng(1)
    pix = np.sort(rng.choice(cam.width * cam.height, 4000, replace=False))
    out, orc, st = compare_rect(ctx, oracle_mod, scene, cam, 64, 0, pixels=pix)
    assert st["band_primary"] < 0.01 * st["n"]
