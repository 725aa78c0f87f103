"""The traversal kernels' FP32 Moller-Trumbore (Moller & Trumbore, JGT 1997) with fused multiply-adds, emulated
exactly on the CPU, against the oracle's band for that test.

The kernels evaluate each cross-product component as fma(a, b, -(c d)) and each dot product as
fma(z, z', fma(y, y', x x')), one rounding per FMA, and divide by multiplying with the reciprocal of the
determinant.  The oracle's certainty comes from a running forward-error bound that counts the rounding of
every product and every sum separately; the fused form rounds less, so every decision the oracle calls
certain must come out the same, and t, u, v must stay inside the oracle's bounds.  The unfused form is
checked the same way, so both sides of the comparison are pinned.

FP32 arithmetic is emulated with exact rationals and one correct rounding per operation (an FMA rounds
once); the reciprocal is the correctly rounded one (the kernels' hardware reciprocal is within 1 ulp, which
the band allows for)."""
from fractions import Fraction

import numpy as np

from oracle import oracle as O
from tests.test_oracle_watertight import random_cases
from tests.test_slab_bound import fr, rnd


def mul(a, b):
    return rnd(fr(a) * fr(b))


def add(a, b):
    return rnd(fr(a) + fr(b))


def fma(a, b, c):
    return rnd(fr(a) * fr(b) + fr(c))


def mt_emulated(o, d, tri, fused):
    """(hit, t, u, v) of the kernels' FP32 test on the packed triangle (v0, e1 = v1 - v0, e2 = v2 - v0)."""
    v0 = [float(x) for x in tri[0]]
    e1 = [rnd(fr(tri[1][k]) - fr(tri[0][k])) for k in range(3)]
    e2 = [rnd(fr(tri[2][k]) - fr(tri[0][k])) for k in range(3)]
    o, d = [float(x) for x in o], [float(x) for x in d]

    def cross(a, b):
        idx = ((1, 2), (2, 0), (0, 1))
        if fused:
            return [fma(a[i], b[j], -mul(a[j], b[i])) for i, j in idx]
        return [rnd(fr(mul(a[i], b[j])) - fr(mul(a[j], b[i]))) for i, j in idx]

    def dot(a, b):
        if fused:
            return fma(a[2], b[2], fma(a[1], b[1], mul(a[0], b[0])))
        return add(add(mul(a[0], b[0]), mul(a[1], b[1])), mul(a[2], b[2]))

    p = cross(d, e2)
    det = dot(e1, p)
    if det == 0.0:
        return False, 0.0, 0.0, 0.0
    idet = rnd(1 / fr(det))
    s = [rnd(fr(o[k]) - fr(v0[k])) for k in range(3)]
    u = mul(dot(s, p), idet)
    q = cross(s, e1)
    v = mul(dot(d, q), idet)
    t = mul(dot(e2, q), idet)
    hit = u >= 0.0 and v >= 0.0 and add(u, v) <= 1.0 and t > 0.0
    return hit, t, u, v


def oracle_for(tri):
    pos = np.asarray(tri, np.float32).reshape(3, 3)
    return O.OracleScene(pos, np.arange(3, dtype=np.uint32).reshape(1, 3), np.zeros(1, np.uint32),
                         np.array([[0.5, 0.5, 0.5, 0.5, 0.0]], np.float32), use_bvh=False, watertight=False)


def test_fused_and_unfused_mt_within_the_oracle_band():
    rng = np.random.default_rng(3)
    stats = {"pass": 0, "fail": 0, "unc": 0, "differ": 0}
    for tri, o, d in random_cases(rng, 1500):
        res = O_res = oracle_for(tri).tri_test(0, o, d)      # exact_hit, status, t, u, v, et, eu, ev
        status = int(O_res[1])
        out = [mt_emulated(o, d, tri, fused) for fused in (True, False)]
        stats["differ"] += out[0][0] != out[1][0]
        for hit, t, u, v in out:
            if status == 1:
                assert hit, (tri, o, d, res)
                assert abs(t - res[2]) <= res[5] and abs(u - res[3]) <= res[6] and abs(v - res[4]) <= res[7]
            elif status == 0:
                assert not hit, (tri, o, d, res)
        stats[("fail", "pass", "unc")[status]] += 1
    # every outcome is reached; rays aimed at edges and vertices make the band non-empty
    assert stats["pass"] > 100 and stats["fail"] > 100 and stats["unc"] > 20, stats
    # where the two forms decide differently the oracle called the case uncertain (checked above)
    assert stats["differ"] <= stats["unc"], stats


def test_fused_mt_differs_from_unfused_somewhere():
    """The emulation really evaluates a different rounding: on near-edge rays some results differ in the
    last bits (otherwise the test above would not say anything about the fused form)."""
    rng = np.random.default_rng(4)
    n_diff = 0
    for tri, o, d in random_cases(rng, 300):
        a, b = mt_emulated(o, d, tri, True), mt_emulated(o, d, tri, False)
        n_diff += a[1:] != b[1:]
    assert n_diff > 30, n_diff
