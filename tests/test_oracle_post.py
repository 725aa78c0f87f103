"""Pins of the display post-processing oracle (tone mapping, sRGB, FXAA): the sRGB standard's own
inverse, Reinhard's limits, and FXAA results derived by hand from the algorithm's definition for a long
one-pixel line and for a step edge that ends inside the search range."""
import numpy as np

from oracle import post as P


def gray(img):
    """(H, W) gray levels -> (H, W, 4) uint8 RGBA (luma = 256 x level for gray)."""
    out = np.empty(img.shape + (4,), np.uint8)
    out[..., :3] = img[..., None]
    out[..., 3] = 255
    return out


def test_srgb_encoding_inverts_the_standard_decoding():
    s8 = np.arange(256)
    s = s8 / 255.0
    lin = np.where(s <= 0.04045, s / 12.92, ((s + 0.055) / 1.055) ** 2.4)   # IEC 61966-2-1 decoding
    assert np.array_equal(P.srgb8(lin), s8.astype(np.uint8))
    # the two branches meet at the breakpoint
    v = 0.0031308
    assert abs(12.92 * v - (1.055 * v ** (1 / 2.4) - 0.055)) < 1e-6


def test_reinhard_limits_and_alpha():
    rgba = np.array([[[0.0, 1.0, 1e9, 0.0], [-1.0, 3.0, 1e-6, 1.0], [0.5, 0.5, 0.5, 0.5]]], np.float32)
    out = P.tonemap_srgb8(rgba)
    assert out[0, 0, 0] == 0 and out[0, 0, 2] == 255 and out[0, 0, 3] == 0
    assert out[0, 0, 1] == P.srgb8(np.array([0.5]))[0]           # c = 1 maps to 1/2
    assert out[0, 1, 0] == 0                                      # negative clamps to 0
    assert out[0, 1, 1] == P.srgb8(np.array([0.75]))[0]          # c = 3 maps to 3/4
    assert out[0, 1, 3] == 255 and out[0, 2, 3] == 128
    assert out[0, 2, 0] == P.srgb8(np.array([1.0 / 3.0]))[0]     # c = 1/2 maps to 1/3


def test_fxaa_leaves_flat_and_low_contrast_images():
    const = gray(np.full((9, 13), 140, np.uint8))
    assert np.array_equal(P.fxaa(const), const)
    rng = np.random.default_rng(0)
    low = gray((120 + rng.integers(0, 7, (11, 17))).astype(np.uint8))   # luma range < 2048 everywhere
    assert np.array_equal(P.fxaa(low), low)


def test_fxaa_long_line_known_answer():
    b, d = 200, 20
    img = np.full((9, 40), d, np.uint8)
    img[4, :] = b
    out = P.fxaa(gray(img))[..., 0].astype(int)
    # on the line: no edge end within 12 pixels, sub-pixel term s = 2/3 -> w = 0.75 ((3 - 4/3) (4/9))^2
    s = 2.0 / 3.0
    w_line = 0.75 * ((3 - 2 * s) * s * s) ** 2
    assert np.all(out[4, 13:27] == int(np.floor(b + w_line * (d - b) + 0.5)))     # 126
    # next to it: s = 1/3, blended toward the line
    s = 1.0 / 3.0
    w_side = 0.75 * ((3 - 2 * s) * s * s) ** 2
    want = int(np.floor(d + w_side * (b - d) + 0.5))                               # 29
    assert np.all(out[3, 13:27] == want) and np.all(out[5, 13:27] == want)
    # two rows away nothing changes
    assert np.all(out[:2] == d) and np.all(out[7:] == d)


def test_fxaa_step_edge_ending_in_range_known_answer():
    b, d = 200, 20
    img = np.full((20, 40), d, np.uint8)
    img[10:, :20] = b
    out = P.fxaa(gray(img))[..., 0].astype(int)
    # pixel (x=15, y=10): edge along x, side north, end found 5 pixels east (none within 12 west):
    # offset 0.5 - 5 / (5 + 13); the sub-pixel term (s = 1/3) is smaller
    w = 0.5 - 5.0 / 18.0
    assert out[10, 15] == int(np.floor(b + w * (d - b) + 0.5))                     # 160
    # the end of the edge is nearer for x = 18: offset 0.5 - 2 / (2 + 13)
    w = 0.5 - 2.0 / 15.0
    assert out[10, 18] == int(np.floor(b + w * (d - b) + 0.5))
