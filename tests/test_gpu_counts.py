"""Own-path work counts: the per-lane rect-light kernel's node-visit and triangle-test counters against the
oracle's instrumented traversal of the library's exported BVH over the same shadow rays (the algorithmic
work per ray that the benchmark's roofline uses); the wave kernel's counters (union of the wave's paths)
are reported beside them."""
import sys

import numpy as np
import pytest

from paper_2410_05095_amd import scenegen as sg

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


@pytest.mark.parametrize("seed,n_inst,N", [(5, 40, 16), (6, 120, 7)])
def test_per_lane_counts_match_instrumented_oracle(ctx, oracle_mod, seed, n_inst, N):
    import torch
    O = oracle_mod
    scene = sg.small_random_scene(seed, n_instances=n_inst, width=48, height=36, ssaa=1)
    cam = scene.cameras[0]
    say(f"[counts] seed {seed} instances {n_inst} tris {scene.n_tris} N={N}")
    gs = ctx.scene_from(scene).build()
    got = {}
    for per_lane in (True, False):
        ctx.render(gs, cam, (), rect=scene.rect_light, area_samples=N, area_stream=0, per_lane=per_lane, wave=not per_lane, count=True)
        torch.cuda.synchronize()
        assert ctx.last_error() == 0
        st = ctx.stage_times()
        got[per_lane] = (st["shadow_rays"], st["shadow_nodes"], st["shadow_tris"])
    nodes, order = gs.export()
    orc = O.OracleScene.from_scene(scene).count_rect(cam, scene.rect_light, N, 0,
                                                      np.arange(cam.width * cam.height), nodes, order)
    rays, nn, nt = got[True]
    say(f"  per-lane kernel: rays {rays} nodes {nn} tris {nt}; oracle: {orc}; "
        f"wave kernel (union of paths): nodes {got[False][1]} tris {got[False][2]} "
        f"(x{got[False][1] / max(nn, 1):.2f}, x{got[False][2] / max(nt, 1):.2f})")
    assert orc["rays"] > 1000
    assert abs(rays - orc["rays"]) <= 0.002 * orc["rays"] + 2
    assert got[False][0] == rays
    assert abs(nn - orc["nodes"]) <= 0.02 * orc["nodes"]
    assert abs(nt - orc["tris"]) <= 0.02 * orc["tris"]
