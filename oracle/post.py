"""Display post-processing oracle — TEST INFRASTRUCTURE ONLY.

Only tests and the benchmark's checks use this module; it shares no code with the HIP library.

The paper's frame ends in display space (Sec. IV-B, "Main Pass" and "Post-Processing Pass"): the linear
HDR colour is tone mapped with Reinhard's operator, brought back to sRGB gamma space, and a screen-space
anti-aliasing pass (FXAA, Sec. IV-B "Anti-Aliasing") blends across luma edges.  The paper gives neither
the tone-map variant nor FXAA's parameters; the readings used here:

* Reinhard per channel, r = c / (1 + c), in FP32 (negative inputs clamp to 0); the sRGB transfer
  function of IEC 61966-2-1 (linear segment 12.92 v below 0.0031308, else 1.055 v^(1/2.4) - 0.055),
  evaluated in FP64 and quantised to 8 bits with floor(255 s + 0.5).  Alpha (coverage) is quantised
  the same way without the curve.
* FXAA in the manner of Lottes' fast approximate anti-aliasing, on the 8-bit sRGB image, with integer
  luma so that every decision is exact: luma = 77 R + 150 G + 29 B (Rec. 601 weights x 256).
  A pixel is processed when its 4-neighbourhood luma range is at least 2048 (about 1/32 of full scale)
  and at least 1/8 of the neighbourhood maximum.  The edge runs along x when the second differences
  across rows (weights 1, 2, 1 over the three columns) are at least those across columns.  The side
  is the neighbour across the edge with the larger luma step (ties: north / west).  Along the edge the
  luma pair straddling the edge is followed up to 12 pixels each way until it departs from the centre
  pair by at least half the step; if the nearer end differs from the centre pair in the opposite
  direction to the centre pixel, the pixel is blended toward the side neighbour by 0.5 minus the
  distance to that end over the span between the two ends.  A sub-pixel term (FP32, fixed order)
  from the 3x3 weighted luma mean, s = clamp(|mean - centre| / range), t = (3 - 2 s) s s,
  0.75 t^2, is used when larger.  Blend: floor(a + w (b - a) + 0.5) per channel in FP32.  Image borders
  clamp.
"""
from __future__ import annotations

import numpy as np

LUMA_W = (77, 150, 29)
EDGE_MIN = 2048
EDGE_REL_SHIFT = 3
SEARCH = 12
F32 = np.float32


def srgb8(v: np.ndarray) -> np.ndarray:
    """FP64 sRGB encoding of linear values in [0, 1], quantised to 8 bits."""
    v = np.asarray(v, np.float64)
    s = np.where(v <= 0.0031308, 12.92 * v, 1.055 * np.power(np.maximum(v, 0.0), 1.0 / 2.4) - 0.055)
    return np.clip(np.floor(s * 255.0 + 0.5), 0, 255).astype(np.uint8)


def tonemap_srgb8(rgba: np.ndarray) -> np.ndarray:
    """(H, W, 4) linear float32 -> (H, W, 4) uint8: Reinhard per channel (FP32), sRGB, alpha quantised."""
    c = np.maximum(np.asarray(rgba, F32)[..., :3], F32(0.0))
    r = c / (F32(1.0) + c)
    out = np.empty(rgba.shape[:-1] + (4,), np.uint8)
    out[..., :3] = srgb8(r)
    a = np.clip(np.asarray(rgba, F32)[..., 3].astype(np.float64), 0.0, 1.0)
    out[..., 3] = np.floor(a * 255.0 + 0.5).astype(np.uint8)
    return out


def luma(img8: np.ndarray) -> np.ndarray:
    i = img8.astype(np.int64)
    return LUMA_W[0] * i[..., 0] + LUMA_W[1] * i[..., 1] + LUMA_W[2] * i[..., 2]


def fxaa(img8: np.ndarray) -> np.ndarray:
    """(H, W, 4) uint8 sRGB -> (H, W, 4) uint8 with the edge blending described in the module text."""
    H, W = img8.shape[:2]
    L = luma(img8)
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")

    def at(x, y):
        return L[np.clip(y, 0, H - 1), np.clip(x, 0, W - 1)]

    Lc = L
    Ln, Ls, Lw, Le = at(xx, yy - 1), at(xx, yy + 1), at(xx - 1, yy), at(xx + 1, yy)
    Lnw, Lne, Lsw, Lse = at(xx - 1, yy - 1), at(xx + 1, yy - 1), at(xx - 1, yy + 1), at(xx + 1, yy + 1)
    lmax = np.maximum.reduce([Lc, Ln, Ls, Lw, Le])
    lmin = np.minimum.reduce([Lc, Ln, Ls, Lw, Le])
    rng = lmax - lmin
    active = (rng >= EDGE_MIN) & ((rng << EDGE_REL_SHIFT) >= lmax)
    d_across_rows = np.abs(Lnw - 2 * Lw + Lsw) + 2 * np.abs(Ln - 2 * Lc + Ls) + np.abs(Lne - 2 * Le + Lse)
    d_across_cols = np.abs(Lnw - 2 * Ln + Lne) + 2 * np.abs(Lw - 2 * Lc + Le) + np.abs(Lsw - 2 * Ls + Lse)
    horiz = d_across_rows >= d_across_cols            # the edge runs along x: blend across rows
    L1 = np.where(horiz, Ln, Lw)
    L2 = np.where(horiz, Ls, Le)
    g1, g2 = np.abs(L1 - Lc), np.abs(L2 - Lc)
    first = g1 >= g2
    side_l = np.where(first, L1, L2)
    grad = np.maximum(g1, g2)
    S2 = Lc + side_l                                   # twice the mean of the pair straddling the edge
    sx = np.where(horiz, 0, np.where(first, -1, 1))    # offset to the side neighbour
    sy = np.where(horiz, np.where(first, -1, 1), 0)
    ax = np.where(horiz, 1, 0)                         # direction along the edge
    ay = np.where(horiz, 0, 1)

    def search(sign):
        dist = np.full(L.shape, SEARCH + 1, np.int64)
        mend = np.zeros(L.shape, np.int64)
        done = np.zeros(L.shape, bool)
        for i in range(1, SEARCH + 1):
            px, py = xx + sign * i * ax, yy + sign * i * ay
            m = at(px, py) + at(px + sx, py + sy)
            hit = ~done & (2 * np.abs(m - S2) >= grad)
            dist = np.where(hit, i, dist)
            mend = np.where(hit, m, mend)
            done |= hit
        return dist, mend, done

    dp, mp, fp = search(+1)
    dn, mn, fn = search(-1)
    near_pos = dp < dn
    dmin = np.minimum(dp, dn)
    mend = np.where(near_pos, mp, mn)
    found = np.where(near_pos, fp, fn)
    blend_edge = found & ((mend - S2 < 0) != (2 * Lc - S2 < 0))
    off_edge = np.where(blend_edge, F32(0.5) - dmin.astype(F32) / (dp + dn).astype(F32), F32(0.0)).astype(F32)
    a12 = 2 * (Ln + Ls + Le + Lw) + (Lne + Lnw + Lse + Lsw)
    num = np.abs(a12 - 12 * Lc).astype(F32)
    den = np.maximum(12 * rng, 1).astype(F32)
    s1 = np.minimum(num / den, F32(1.0)).astype(F32)
    t = (F32(-2.0) * s1).astype(F32)
    t = (t + F32(3.0)).astype(F32)
    t = (t * s1).astype(F32)
    t = (t * s1).astype(F32)
    sub = ((t * t).astype(F32) * F32(0.75)).astype(F32)
    w = np.maximum(off_edge, sub).astype(F32)
    out = img8.copy()
    nb = img8[np.clip(yy + sy, 0, H - 1), np.clip(xx + sx, 0, W - 1)]
    for c in range(3):
        a = img8[..., c].astype(F32)
        b = nb[..., c].astype(F32)
        v = (a + (w * (b - a)).astype(F32)).astype(F32)
        v = np.floor((v + F32(0.5)).astype(F32))
        out[..., c] = np.where(active, np.clip(v, 0, 255), img8[..., c]).astype(np.uint8)
    return out


def postprocess(rgba: np.ndarray, aa: bool = True) -> np.ndarray:
    img = tonemap_srgb8(rgba)
    return fxaa(img) if aa else img
