"""U-Net shadow-denoiser oracle in FP64 numpy — TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg use this module; the HIP library
never does.  The network (a learned replacement of the many-sample soft-shadow estimate; the paper's
Sec. IV-B mentions denoising as what makes real-time ray tracing practical) maps 8 feature channels
(1-sample visibility, log depth, normal xyz, albedo rgb) to a visibility in (0, 1):

  e1 = R(C(R(C(x))))            8 -> 32 -> 32
  e2 = R(C(R(C(P(e1)))))       32 -> 64 -> 64        P = 2x2 average pool
  b  = R(C(R(C(P(e2)))))       64 -> 128 -> 128
  d2 = R(C(R(C([U(b), e2]))))  192 -> 64 -> 64       U = nearest 2x upsample, [] = channel concat
  d1 = R(C(R(C([U(d2), e1])))) 96 -> 32 -> 32
  y  = sigmoid(d1 . w_h + b_h)                       1x1 head

C = 3x3 cross-correlation with zero "same" padding plus bias, R = ReLU.  Tensors are NHWC; weights
are (Cout, 3, 3, Cin).  With bf16=True the forward pass rounds the weights and every stored
activation (features, conv outputs, pools, concats) to bfloat16 (round to nearest even) at the same
points where the GPU stores BF16; arithmetic stays FP64.
"""
from __future__ import annotations

import numpy as np

LAYERS = [("e1a", 8, 32), ("e1b", 32, 32), ("e2a", 32, 64), ("e2b", 64, 64), ("bna", 64, 128),
          ("bnb", 128, 128), ("d2a", 192, 64), ("d2b", 64, 64), ("d1a", 96, 32), ("d1b", 32, 32)]
N_PARAMS = sum(9 * ci * co + co for _, ci, co in LAYERS) + 32 + 1


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def init_params(seed: int = 0) -> dict:
    """He-normal conv weights (fan-in 9 Cin), zero biases, head N(0, 1/32)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co in LAYERS:
        p[name + ".w"] = rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), (co, 3, 3, ci))
        p[name + ".b"] = np.zeros(co)
    p["head.w"] = rng.normal(0.0, np.sqrt(1.0 / 32), 32)
    p["head.b"] = np.zeros(1)
    return p


def conv3x3(x, w, b):
    """out[n,y,x,o] = b[o] + sum_{dy,dx,i} w[o,dy,dx,i] * xpad[n, y+dy, x+dx, i]"""
    N, H, W, Ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(b, (N, H, W, w.shape[0])).copy()
    for dy in range(3):
        for dx in range(3):
            out += xp[:, dy:dy + H, dx:dx + W, :] @ w[:, dy, dx, :].T
    return out


def conv3x3_backward(x, w, g):
    """Gradients of sum(g * conv3x3(x, w, b)) w.r.t. x, w, b."""
    N, H, W, Ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    g2 = g.reshape(-1, g.shape[-1])
    for dy in range(3):
        for dx in range(3):
            gxp[:, dy:dy + H, dx:dx + W, :] += g @ w[:, dy, dx, :]
            gw[:, dy, dx, :] = g2.T @ xp[:, dy:dy + H, dx:dx + W, :].reshape(-1, Ci)
    return gxp[:, 1:-1, 1:-1, :], gw, g2.sum(axis=0)


def pool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_backward(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(g):
    N, H, W, C = g.shape
    return g.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def forward(params: dict, x: np.ndarray, bf16: bool = False, conv=None):
    """Returns (y (N,H,W), cache of every stored tensor).  `conv` replaces conv3x3 (same signature),
    e.g. by a variant that sums in another precision, to measure how much BF16 rounding of the
    stored activations alone moves the result."""
    conv = conv3x3 if conv is None else conv
    rd = bf16_round if bf16 else (lambda a: a)
    P = {k: (rd(v) if k.endswith(".w") else v) for k, v in params.items()}
    c = {"x": rd(x)}

    def block(name_a, name_b, inp, tag):
        a = rd(np.maximum(conv(inp, P[name_a + ".w"], P[name_a + ".b"]), 0.0))
        b = rd(np.maximum(conv(a, P[name_b + ".w"], P[name_b + ".b"]), 0.0))
        c[tag + "_in"], c[tag + "_a"], c[tag + "_b"] = inp, a, b
        return b

    e1 = block("e1a", "e1b", c["x"], "e1")
    e2 = block("e2a", "e2b", rd(pool2(e1)), "e2")
    bn = block("bna", "bnb", rd(pool2(e2)), "bn")
    d2 = block("d2a", "d2b", np.concatenate([up2(bn), e2], axis=-1), "d2")
    d1 = block("d1a", "d1b", np.concatenate([up2(d2), e1], axis=-1), "d1")
    logit = d1 @ P["head.w"] + P["head.b"][0]
    y = 1.0 / (1.0 + np.exp(-logit))
    c["y"] = y
    c["P"] = P
    return y, c


def masked_mse(y, target, mask):
    """sum(mask (y - target)^2) / max(sum(mask), 1)"""
    m = np.asarray(mask, np.float64)
    return float((m * (y - target) ** 2).sum() / max(m.sum(), 1.0))


def backward(params: dict, cache: dict, target, mask, bf16_grads: bool = False):
    """Gradient of masked_mse w.r.t. every parameter (a dict like params) and the input features.

    With bf16_grads=True the activation gradients are rounded to bfloat16 where a BF16 pipeline
    stores them: the head's gradient into the last ReLU, every convolution's input gradient, the
    gradient of each upsampled tensor, and each pooled gradient plus its skip gradient."""
    rd = bf16_round if bf16_grads else (lambda a: a)
    P = cache["P"]
    y = cache["y"]
    m = np.asarray(mask, np.float64)
    dy = 2.0 * m * (y - target) / max(m.sum(), 1.0)
    dlogit = dy * y * (1.0 - y)
    g = {}
    d1 = cache["d1_b"]
    g["head.w"] = np.tensordot(dlogit, d1, axes=([0, 1, 2], [0, 1, 2]))
    g["head.b"] = np.array([dlogit.sum()])
    gd1 = rd(dlogit[..., None] * P["head.w"])

    def block_back(name_a, name_b, tag, gout):
        a, b, inp = cache[tag + "_a"], cache[tag + "_b"], cache[tag + "_in"]
        gpre = gout * (b > 0)
        ga, g[name_b + ".w"], g[name_b + ".b"] = conv3x3_backward(a, P[name_b + ".w"], gpre)
        gpre = rd(ga) * (a > 0)
        gin, g[name_a + ".w"], g[name_a + ".b"] = conv3x3_backward(inp, P[name_a + ".w"], gpre)
        return rd(gin)

    gu1 = block_back("d1a", "d1b", "d1", gd1)
    gd2 = rd(up2_backward(gu1[..., :64]))
    ge1_skip = gu1[..., 64:]
    gu2 = block_back("d2a", "d2b", "d2", gd2)
    gbn = rd(up2_backward(gu2[..., :128]))
    ge2_skip = gu2[..., 128:]
    gp2 = block_back("bna", "bnb", "bn", gbn)
    ge2 = rd(pool2_backward(gp2) + ge2_skip)
    gp1 = block_back("e2a", "e2b", "e2", ge2)
    ge1 = rd(pool2_backward(gp1) + ge1_skip)
    gx = block_back("e1a", "e1b", "e1", ge1)
    return g, gx


def adam_step(params, grads, state, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma & Ba) with bias correction; t counts from 1.  Updates in place."""
    for k in params:
        m = state.setdefault(k + ".m", np.zeros_like(params[k]))
        v = state.setdefault(k + ".v", np.zeros_like(params[k]))
        m *= b1
        m += (1 - b1) * grads[k]
        v *= b2
        v += (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] -= lr * mh / (np.sqrt(vh) + eps)


def flat(params: dict) -> np.ndarray:
    return np.concatenate([params[k].ravel() for k in param_names()])


def param_names():
    names = []
    for n, _, _ in LAYERS:
        names += [n + ".w", n + ".b"]
    return names + ["head.w", "head.b"]
