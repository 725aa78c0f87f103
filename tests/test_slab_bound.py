"""The FP32 slab test of the traversal kernels, emulated exactly on the CPU.

Every traversal kernel tests a box with one FMA per plane, p * inv + c, where inv = 1/dd (dd: the direction
clamped to |dd| >= 1e-20), the near offsets c are -o * inv moved down by 2^-21 |.| + 2^-120, and the far
planes use inv * (1 + 2^-20) with offsets moved up likewise.  A box is entered when max(near, 0) <=
min(far, bound).  The claim this pins: whenever the exact segment o + t dd, 0 <= t <= bound, meets the box,
the FP32 test passes, so no box on a ray's way is skipped.  Boxes that the segment misses by a clear margin
must fail, so the test is not trivially true.

FP32 arithmetic is emulated with exact rationals and one correct rounding per operation (the FMA rounds
once)."""
from fractions import Fraction

import numpy as np

F32 = np.float32


def rnd(x: Fraction) -> float:
    """x rounded to the nearest FP32 value (ties to even)."""
    c = F32(float(x))      # within one FP32 ulp of the correctly rounded value (double rounding at most)
    best = None
    for cand in (np.nextafter(c, F32(-np.inf)), c, np.nextafter(c, F32(np.inf))):
        e = abs(Fraction(float(cand)) - x)
        key = (e, int(np.frombuffer(F32(cand).tobytes(), np.uint32)[0]) & 1)
        if best is None or key < best[0]:
            best = (key, cand)
    return float(best[1])


def fr(v) -> Fraction:
    return Fraction(float(v))


def ray_consts(o, d):
    """FP32 per-ray constants: dd, inv, invf, cn, cf (exactly as the kernels round them)."""
    dd, inv, invf, cn, cf = [], [], [], [], []
    grow = fr(F32(1.000001))
    for a in range(3):
        x = float(d[a])
        if abs(x) < 1e-20:
            x = float(np.copysign(F32(1e-20), F32(x)))
        dd.append(x)
        i = rnd(1 / fr(x))
        g = rnd(fr(i) * grow)
        c = rnd(-(fr(o[a]) * fr(i)))
        m = rnd(abs(fr(c)) * Fraction(1, 2 ** 21) + Fraction(1, 2 ** 120))
        e = rnd(-(fr(o[a]) * fr(g)))
        mf = rnd(abs(fr(e)) * Fraction(1, 2 ** 21) + Fraction(1, 2 ** 120))
        inv.append(i), invf.append(g), cn.append(rnd(fr(c) - fr(m))), cf.append(rnd(fr(e) + fr(mf)))
    return dd, inv, invf, cn, cf


def slab_fp32(consts, lo, hi, bound):
    dd, inv, invf, cn, cf = consts
    near, far = [], []
    for a in range(3):
        n, f = (lo[a], hi[a]) if inv[a] >= 0 else (hi[a], lo[a])
        near.append(rnd(fr(n) * fr(inv[a]) + fr(cn[a])))
        far.append(rnd(fr(f) * fr(invf[a]) + fr(cf[a])))
    return max(max(near[0], near[1]), max(near[2], 0.0)) <= min(min(far[0], far[1]), min(far[2], bound))


def segment_box_exact(o, dd, lo, hi, bound):
    """Exact [t0, t1] overlap of the segment o + t dd (0 <= t <= bound) with the box; None if empty."""
    t0, t1 = Fraction(0), fr(bound)
    for a in range(3):
        p, q = (fr(lo[a]) - fr(o[a])) / fr(dd[a]), (fr(hi[a]) - fr(o[a])) / fr(dd[a])
        if p > q:
            p, q = q, p
        t0, t1 = max(t0, p), min(t1, q)
    return (t0, t1) if t0 <= t1 else None


def random_ray(rng):
    scale = 10.0 ** rng.integers(-3, 4)
    o = (rng.normal(size=3) * scale).astype(F32)
    d = rng.normal(size=3) * 10.0 ** rng.integers(-2, 3)
    kind = rng.integers(5)
    if kind == 0:
        d[rng.integers(3)] = 0.0                      # axis-parallel in one axis (clamped to 1e-20)
    elif kind == 1:
        d[rng.integers(3)] *= 1e-12                   # nearly parallel
    elif kind == 2:
        o[rng.integers(3)] = 0.0                      # origin on a coordinate plane
    return o, d.astype(F32)


def box_through(rng, o, dd, t, flat_axes=()):
    """An FP32 box containing the exact point o + t dd: each axis either tight around it (a flat box rounds
    the point outward to the two FP32 neighbours) or widened at random on one or both sides."""
    lo, hi = [], []
    for a in range(3):
        p = fr(o[a]) + t * fr(dd[a])
        c = F32(float(p))
        l = c if Fraction(float(c)) <= p else np.nextafter(c, F32(-np.inf))
        h = c if Fraction(float(c)) >= p else np.nextafter(c, F32(np.inf))
        if a not in flat_axes:
            w = abs(float(p)) * 10.0 ** rng.uniform(-7, 0) + 10.0 ** rng.uniform(-6, 0)
            s = rng.integers(3)
            if s != 1:
                l = F32(float(l) - w * rng.random())
            if s != 0:
                h = F32(float(h) + w * rng.random())
            if not (Fraction(float(l)) <= p <= Fraction(float(h))):
                l, h = min(l, F32(float(c))), max(h, F32(float(c)))
                l = l if Fraction(float(l)) <= p else np.nextafter(l, F32(-np.inf))
                h = h if Fraction(float(h)) >= p else np.nextafter(h, F32(np.inf))
        lo.append(float(l)), hi.append(float(h))
    return lo, hi


def test_boxes_on_the_segment_always_pass():
    rng = np.random.default_rng(7)
    n = 0
    for _ in range(1500):
        o, d = random_ray(rng)
        consts = ray_consts(o, d)
        dd = consts[0]
        for t in (Fraction(0), Fraction(1), Fraction(int(rng.integers(1, 2 ** 20)), 2 ** 20),
                  Fraction(1) - Fraction(1, 2 ** 22)):
            flat = tuple(a for a in range(3) if rng.random() < 0.3)
            lo, hi = box_through(rng, o, dd, t, flat)
            assert segment_box_exact(o, dd, lo, hi, 2.0) is not None
            # bound 2 leaves room above the segment's end, whose FP32 neighbourhood the oracle's band covers
            assert slab_fp32(consts, lo, hi, 2.0), (o, d, lo, hi, t)
            n += 1
    assert n == 6000


def test_boxes_clear_of_the_segment_fail():
    """Boxes the exact segment misses by a relative margin of 1e-4 (behind the origin, beyond the bound, or
    beside the ray) fail the test."""
    rng = np.random.default_rng(8)
    n_checked = 0
    for _ in range(1500):
        o, d = random_ray(rng)
        if min(abs(float(x)) for x in d) < 1e-6 * max(abs(float(x)) for x in d):
            continue   # nearly parallel rays: the clamp and the margins make the slabs of that axis wide
        consts = ray_consts(o, d)
        dd = consts[0]
        t = Fraction(int(rng.integers(0, 2 ** 20)), 2 ** 20)
        lo, hi = box_through(rng, o, dd, t)
        a = int(rng.integers(3))
        size = max(abs(float(o[k])) + abs(float(dd[k])) for k in range(3))
        gap = 1e-4 * size + (hi[a] - lo[a])
        shift = gap if rng.random() < 0.5 else -gap
        lo2, hi2 = list(lo), list(hi)
        lo2[a] = float(F32(lo[a] + shift))
        hi2[a] = float(F32(hi[a] + shift))
        ex = segment_box_exact(o, dd, lo2, hi2, 1.0)
        if ex is not None:
            continue   # the shifted box still meets the segment elsewhere
        # the exact distance by which the segment misses, in t: require a clear miss
        grown = [lo2[k] - 1e-5 * size for k in range(3)], [hi2[k] + 1e-5 * size for k in range(3)]
        if segment_box_exact(o, dd, grown[0], grown[1], 1.0) is not None:
            continue
        assert not slab_fp32(consts, lo2, hi2, 1.0), (o, d, lo2, hi2)
        n_checked += 1
    assert n_checked > 300, n_checked
