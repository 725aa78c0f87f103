"""Pins of the oracle's band model for the watertight ray/triangle test (Woop, Benthin and Wald, JCGT 2013).

The test decides the same geometric crossing as Moller-Trumbore in exact arithmetic; only the FP32
certainty differs.  An FP32 evaluation of the test written here in numpy (step by step, independent of the
oracle) must agree with every decision the oracle calls certain, and its t, u, v must lie within the
oracle's error bounds.  The same evaluation never lets a ray slip between two triangles that share an
edge, which is the property the test exists for.  Scenes rendered with the watertight band have the same
hits as with the Moller-Trumbore band wherever neither is uncertain."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_05095_amd import scenegen as sg

F = np.float32


def wt_fp32(o, d, v0, v1, v2):
    """FP32 watertight test: (hit, t, u, v) with the operation order of the kernels (t > 0 required)."""
    o, d = o.astype(F), d.astype(F)
    kz = 0
    if abs(d[1]) > abs(d[kz]):
        kz = 1
    if abs(d[2]) > abs(d[kz]):
        kz = 2
    kx, ky = (kz + 1) % 3, (kz + 2) % 3
    if d[kz] < 0:
        kx, ky = ky, kx
    Sx, Sy, Sz = F(d[kx] / d[kz]), F(d[ky] / d[kz]), F(F(1) / d[kz])
    A, B, C = (v0.astype(F) - o), (v1.astype(F) - o), (v2.astype(F) - o)
    Ax, Ay = F(A[kx] - F(Sx * A[kz])), F(A[ky] - F(Sy * A[kz]))
    Bx, By = F(B[kx] - F(Sx * B[kz])), F(B[ky] - F(Sy * B[kz]))
    Cx, Cy = F(C[kx] - F(Sx * C[kz])), F(C[ky] - F(Sy * C[kz]))
    U, V, W = F(F(Cx * By) - F(Cy * Bx)), F(F(Ax * Cy) - F(Ay * Cx)), F(F(Bx * Ay) - F(By * Ax))
    if U == 0 or V == 0 or W == 0:
        D = np.float64
        U = F(D(Cx) * D(By) - D(Cy) * D(Bx))
        V = F(D(Ax) * D(Cy) - D(Ay) * D(Cx))
        W = F(D(Bx) * D(Ay) - D(By) * D(Ax))
    if (U < 0 or V < 0 or W < 0) and (U > 0 or V > 0 or W > 0):
        return False, 0.0, 0.0, 0.0
    det = F(F(U + V) + W)
    if det == 0:
        return False, 0.0, 0.0, 0.0
    Az, Bz, Cz = F(Sz * A[kz]), F(Sz * B[kz]), F(Sz * C[kz])
    T = F(F(F(U * Az) + F(V * Bz)) + F(W * Cz))
    r = F(F(1) / det)
    t, u, v = F(T * r), F(V * r), F(W * r)
    return bool(t > 0), float(t), float(u), float(v)


def mt_fp32(o, d, a, b, c):
    """FP32 Moller-Trumbore in the kernels' order (edges rounded first); hit with t > 0."""
    a, b, c = a.astype(F), b.astype(F), c.astype(F)
    e1, e2 = b - a, c - a
    px, py, pz = F(d[1] * e2[2]) - F(d[2] * e2[1]), F(d[2] * e2[0]) - F(d[0] * e2[2]), F(d[0] * e2[1]) - F(d[1] * e2[0])
    det = F(F(e1[0] * px) + F(e1[1] * py)) + F(e1[2] * pz)
    idet = F(1) / det
    s = o - a
    u = F(F(F(F(s[0] * px) + F(s[1] * py)) + F(s[2] * pz)) * idet)
    qx, qy, qz = F(s[1] * e1[2]) - F(s[2] * e1[1]), F(s[2] * e1[0]) - F(s[0] * e1[2]), F(s[0] * e1[1]) - F(s[1] * e1[0])
    v = F(F(F(F(d[0] * qx) + F(d[1] * qy)) + F(d[2] * qz)) * idet)
    t = F(F(F(F(e2[0] * qx) + F(e2[1] * qy)) + F(e2[2] * qz)) * idet)
    return bool(u >= 0 and v >= 0 and u + v <= 1 and t > 0)


def oracle_for(tri, watertight=True):
    pos = np.asarray(tri, F).reshape(3, 3)
    return O.OracleScene(pos, np.arange(3, dtype=np.uint32).reshape(1, 3), np.zeros(1, np.uint32),
                         np.array([[0.5, 0.5, 0.5, 0.5, 0.0]], F), use_bvh=False, watertight=watertight)


def random_cases(rng, n):
    for _ in range(n):
        tri = rng.normal(size=(3, 3)) * rng.choice([0.01, 1.0, 30.0])
        o = rng.normal(size=3) * 20.0
        kind = rng.integers(4)
        if kind == 0:      # towards a random point of the triangle's plane near it
            w = rng.dirichlet([1, 1, 1]) * 1.4 - 0.13
            target = w @ tri
        elif kind == 1:    # exactly towards an edge point (in FP64; the FP32 ray rounds it)
            a, b = rng.choice(3, 2, replace=False)
            s = rng.random()
            target = tri[a] + s * (tri[b] - tri[a])
        elif kind == 2:    # towards a vertex
            target = tri[rng.integers(3)]
        else:              # a random direction
            target = o + rng.normal(size=3)
        d = target - o
        d = d / np.linalg.norm(d)
        yield tri.astype(F), o.astype(F), d.astype(F)


def test_certain_decisions_agree_with_an_fp32_evaluation():
    rng = np.random.default_rng(0)
    stats = {"pass": 0, "fail": 0, "unc": 0}
    for tri, o, d in random_cases(rng, 4000):
        osc = oracle_for(tri)
        res = osc.tri_test(0, o, d)      # exact_hit, status, t, u, v, et, eu, ev
        hit, t, u, v = wt_fp32(o, d, tri[0], tri[1], tri[2])
        status = int(res[1])
        if status == 1:
            stats["pass"] += 1
            assert hit, (tri, o, d, res)
            assert abs(t - res[2]) <= res[5] and abs(u - res[3]) <= res[6] and abs(v - res[4]) <= res[7]
        elif status == 0:
            stats["fail"] += 1
            assert not hit, (tri, o, d, res)
        else:
            stats["unc"] += 1
        assert bool(res[0]) == (status == 1) or status == 2
    # the cases reach every outcome, and rays aimed at edges and vertices make the band non-empty
    assert stats["pass"] > 300 and stats["fail"] > 300 and stats["unc"] > 50, stats


def test_no_ray_slips_between_triangles_sharing_an_edge():
    """Rays aimed at points of the shared edge of two triangles (the FP32 ray rounds them to either side):
    the watertight test reports a hit on at least one of the two."""
    rng = np.random.default_rng(1)
    n_both_miss_wt = n_both_miss_mt = 0
    for _ in range(3000):
        a, b = rng.normal(size=3), rng.normal(size=3)
        nrm = rng.normal(size=3)
        c1 = (a + b) / 2 + rng.normal(size=3) * 0.3 + nrm
        c2 = (a + b) / 2 + rng.normal(size=3) * 0.3 - nrm
        s = rng.random()
        target = a + s * (b - a)
        o = target + rng.normal(size=3) * 10.0
        d = (target - o) / np.linalg.norm(target - o)
        o, d = o.astype(F), d.astype(F)
        h1 = wt_fp32(o, d, a, b, c1)[0]
        h2 = wt_fp32(o, d, b, a, c2)[0]
        # skip rays whose crossing of the two triangles' plane pair is behind the origin or grazing
        n1, n2 = np.cross(b - a, c1 - a), np.cross(a - b, c2 - b)
        if abs(np.dot(n1, d)) < 1e-3 * np.linalg.norm(n1) or abs(np.dot(n2, d)) < 1e-3 * np.linalg.norm(n2):
            continue
        if np.dot(n1, d) * np.dot(n2, d) < 0:
            continue   # the two faces are seen from opposite sides: the ray can pass by the edge's outside
        n_both_miss_wt += (not h1) and (not h2)
        n_both_miss_mt += (not mt_fp32(o, d, a, b, c1)) and (not mt_fp32(o, d, b, a, c2))
    assert n_both_miss_wt == 0
    assert n_both_miss_mt > 50      # the same rays slip through with Moller-Trumbore in FP32


@pytest.mark.parametrize("seed", [0, 2])
def test_watertight_band_scene_matches_mt_band_scene(seed):
    scene = sg.small_random_scene(seed, n_instances=10, width=40, height=30, ssaa=2, n_lights=2)
    cam = scene.cameras[0]
    smp = np.arange(cam.n_samples)
    mt = O.OracleScene.from_scene(scene).render_point(cam, scene.point_lights, smp)
    wt = O.OracleScene.from_scene(scene, watertight=True).render_point(cam, scene.point_lights, smp)
    ok = (mt["band_primary"] == 0) & (wt["band_primary"] == 0)
    assert (mt["hit_id"][ok] != wt["hit_id"][ok]).sum() == 0
    sh = ok & (mt["band_shadow"] == 0) & (wt["band_shadow"] == 0)
    assert (mt["mask"][sh] != wt["mask"][sh]).sum() == 0
    assert ok.sum() > 0.97 * len(smp)
