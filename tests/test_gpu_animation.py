"""Animated frames (moving rigid bodies, BVH refit every frame, several views per frame, learned 1-spp path):
the BF16 denoiser against its FP32 copy and both against the 256-sample visibility, frame by frame.
Statistical for the trained network's error (parity unpinned); the geometry after motion and refit is
pinned by the refit tests."""
import sys

import numpy as np
import pytest

from paper_2410_05095_amd import scenegen as sg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_animated_frames_bf16_vs_fp32():
    import torch
    from paper_2410_05095_amd import _native as N
    from paper_2410_05095_amd import animate as A
    from paper_2410_05095_amd import denoise as D
    ctx = N.Context(0)
    kw = dict(n_instances=300, total_tris=1_460_000, width=512, height=288)
    train = [(sc, ctx.scene_from(sc).build()) for sc in (sg.big_scene(1, **kw),)]
    data = D.make_training_set(ctx, train, n_views=16, crops_per_view=8, crop=128, width=512, height=288, seed=0)
    den = N.Denoiser(ctx, seed=0)
    D.train(den, data, steps=300, batch=8, lr=2e-3)
    scene = sg.big_scene(0, **kw)
    gs = ctx.scene_from(scene).build()
    anim = sg.RigidAnimation(scene, n_bodies=60, seed=0)
    views = D.orbit_views(np.random.default_rng(5), 4, 512, 288, seed0=700)
    res = A.run(ctx, scene, gs, den, anim, views, n_frames=6, ref_views=lambda f: list(range(4)), log=say)
    say("[anim]", {k: v for k, v in res.items() if k != "per_frame"})
    assert res["reference_views"] == 24
    assert res["refit_ms_median"] > 0.0
    for r in res["per_frame"]:
        for m16, m32 in zip(r["mse_bf16"], r["mse_fp32"]):
            # BF16 storage changes the error by a small fraction of itself
            assert abs(m16 - m32) <= 0.05 * m32 + 1e-6, r
    assert res["max_abs_bf16_fp32"] < 0.05
    # the denoised estimate beats the raw 1-sample estimate it starts from, on every frame
    assert res["mse_bf16_mean"] < 0.6 * res["mse_raw_1spp_mean"]
    # the views dealt over three streams (the default) give the results of one stream, bit for bit: the same
    # per-view errors on a fresh copy of the scene
    gs1 = ctx.scene_from(scene).build()
    anim1 = sg.RigidAnimation(scene, n_bodies=60, seed=0)
    res1 = A.run(ctx, scene, gs1, den, anim1, views, n_frames=3, ref_views=lambda f: list(range(4)), lanes=1)
    for r2, r1 in zip(res["per_frame"][:3], res1["per_frame"]):
        assert r2["mse_bf16"] == r1["mse_bf16"] and r2["mse_fp32"] == r1["mse_fp32"], (r2, r1)
    torch.cuda.synchronize()
    assert ctx.last_error() == 0
