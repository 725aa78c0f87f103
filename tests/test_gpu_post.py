"""GPU display post pass (tone map, sRGB8, FXAA) against the oracle, bit for bit: random HDR images with
edges at ragged sizes, and a rendered frame."""
import sys

import numpy as np
import pytest

from oracle import post as P
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


def hdr_image(seed, h, w):
    """Random rectangles and diagonal bands of HDR colour over a noisy background."""
    rng = np.random.default_rng(seed)
    img = rng.uniform(0.0, 0.05, (h, w, 4)).astype(np.float32)
    yy, xx = np.mgrid[0:h, 0:w]
    for _ in range(max(2, (h * w) // 200)):
        c = rng.uniform(0.0, 4.0, 3)
        if rng.random() < 0.5:
            y0, x0 = rng.integers(0, h), rng.integers(0, w)
            m = (yy >= y0) & (yy < y0 + rng.integers(1, h + 1)) & (xx >= x0) & (xx < x0 + rng.integers(1, w + 1))
        else:
            a, b = rng.normal(size=2)
            m = np.abs(a * xx + b * yy + rng.uniform(-w, w)) < rng.uniform(0.5, 4.0)
        img[m, :3] = c
    img[..., 3] = (rng.random((h, w)) < 0.9).astype(np.float32)
    img[rng.random((h, w)) < 0.01, :3] = 1e5      # very bright pixels
    img[rng.random((h, w)) < 0.01, :3] = -0.5     # negatives clamp to 0
    return img


def compare(ctx, img, label):
    import torch
    t = torch.from_numpy(img).cuda().contiguous()
    for aa in (False, True):
        got = ctx.postprocess(t, fxaa=aa).cpu().numpy()
        want = P.postprocess(img, aa=aa)
        bad = np.argwhere(np.any(got != want, axis=-1))
        say(f"[post {label} fxaa={aa}] {img.shape[1]}x{img.shape[0]}: {len(bad)} pixels differ")
        assert len(bad) == 0, bad[:5]
    assert ctx.last_error() == 0


@pytest.mark.parametrize("seed,h,w", [(0, 37, 23), (1, 1, 1), (2, 1, 50), (3, 64, 64), (4, 120, 97), (5, 300, 17)])
def test_random_images_bit_exact(ctx, seed, h, w):
    compare(ctx, hdr_image(seed, h, w), f"random {seed}")


def test_rendered_frame_bit_exact(ctx):
    import torch
    scene = sg.small_random_scene(4, n_instances=40, width=160, height=96, ssaa=2, n_lights=3)
    gs = ctx.scene_from(scene).build()
    out = ctx.render(gs, scene.cameras[0], scene.point_lights)
    torch.cuda.synchronize()
    img = out["rgba"].cpu().numpy()
    compare(ctx, img, "rendered")
    # the anti-aliasing pass changes edge pixels only
    tm = P.postprocess(img, aa=False)
    aa = P.postprocess(img, aa=True)
    changed = np.any(tm != aa, axis=-1).mean()
    say(f"[post rendered] FXAA changed {100 * changed:.1f}% of pixels")
    assert 0.0 < changed < 0.5
