"""How far BF16 rounding flips alone move the denoiser's gradients (test helper).

The oracle's BF16-emulating forward stores every activation rounded to bfloat16 from an FP64 sum.  A sum
evaluated in another precision or order (the GPU accumulates in FP32 on the matrix cores) can land on
the other side of a BF16 rounding boundary; each such flip changes a stored value by one BF16 ulp
(2^-8 relative) and propagates through the rest of the network and its backward pass.  On small
batches a few flips decide a tensor's gradient error.  `flip_scale` measures that effect inside the
oracle itself: the same network, inputs and BF16 storage points, with every convolution summed in FP32
(numpy order) instead of FP64, compared per parameter tensor (relative Frobenius norm)."""
import numpy as np

from oracle import unet as U


def conv3x3_f32(x, w, b):
    """conv3x3 with the products and sums in FP32 (inputs are BF16 values, exact in FP32)."""
    N, H, W, Ci = x.shape
    xp = np.pad(x.astype(np.float32), ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(b.astype(np.float32), (N, H, W, w.shape[0])).copy()
    for dy in range(3):
        for dx in range(3):
            out += xp[:, dy:dy + H, dx:dx + W, :] @ w[:, dy, dx, :].T.astype(np.float32)
    return out.astype(np.float64)


def rel_frob(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def flip_scale(params, x, target, mask):
    """Per-tensor relative Frobenius difference between the BF16-emulated oracle gradients with FP32 and
    with FP64 convolution sums, and the number of stored activations that differ between the two."""
    y64, c64 = U.forward(params, x, bf16=True)
    g64, _ = U.backward(params, c64, target, mask, bf16_grads=True)
    y32, c32 = U.forward(params, x, bf16=True, conv=conv3x3_f32)
    g32, _ = U.backward(params, c32, target, mask, bf16_grads=True)
    flips = sum(int((c32[k] != c64[k]).sum()) for k in c64 if k not in ("P", "y"))
    return {k: rel_frob(g32[k], g64[k]) for k in g64}, flips
