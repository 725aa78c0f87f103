"""rc_postprocess_noalloc (fixed per-GPU scratch, no allocation) against rc_postprocess through the C ABI:
identical bytes on consecutive calls whose sizes shrink (the scratch keeps the previous call's contents),
with and without FXAA, up to the maximum size; sizes beyond it are rejected."""
import sys

import numpy as np
import pytest

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


def blocky_hdr(seed, h, w):
    """HDR image with hard-edged blocks (FXAA has edges to work on) over low-level noise."""
    rng = np.random.default_rng(seed)
    bh, bw = (h + 6) // 7, (w + 6) // 7
    blocks = rng.uniform(0.0, 4.0, (bh, bw, 4)).astype(np.float32) * (rng.random((bh, bw, 1)) < 0.6)
    img = np.kron(blocks, np.ones((7, 7, 1), np.float32))[:h, :w]
    img += rng.uniform(0.0, 0.05, (h, w, 4)).astype(np.float32)
    img[..., 3] = rng.uniform(0.0, 1.2, (h, w)).astype(np.float32)
    return np.ascontiguousarray(img)


def test_noalloc_post_equals_allocating_post(ctx):
    import torch
    from paper_2410_05095_amd import _native as N
    for i, (h, w) in enumerate([(2048, 2048), (1080, 1920), (29, 37), (1, 1)]):
        say(f"[post noalloc] call {i}: {w}x{h}")
        rgba = torch.from_numpy(blocky_hdr(i, h, w)).cuda()
        for fxaa in (True, False):
            want = ctx.postprocess(rgba, fxaa=fxaa)
            got = torch.full((h, w, 4), 7, dtype=torch.uint8, device="cuda")
            ctx.postprocess_noalloc(rgba, got, fxaa=fxaa)
            torch.cuda.synchronize()
            assert ctx.last_error() == 0
            assert torch.equal(got, want), (h, w, fxaa)
    big = torch.zeros((2048, 2049, 4), dtype=torch.float32, device="cuda")
    out = torch.empty((2048, 2049, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(N.RcError) as e:
        ctx.postprocess_noalloc(big, out)
    assert e.value.status == -1
