"""Python front end of the CPU oracle — TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It marshals numpy arrays into the plain-C FP64 oracle
(``oracle.c``) and spreads independent samples over host threads (each C call
releases the GIL).  No function here touches the GPU library.
"""
from __future__ import annotations

import ctypes as C
import math
import threading
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # noqa: F401  (oracle/build.py)
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


class OrScene(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("nv", C.c_int64), ("idx", C.c_void_p), ("nt", C.c_int64),
                ("tri_mat", C.c_void_p), ("mats", C.c_void_p), ("nmat", C.c_int64), ("inst", C.c_void_p),
                ("flags", C.c_int64), ("nrm", C.c_void_p)]


class OrCamera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("ssaa", C.c_int32), ("seed", C.c_uint32), ("frame", C.c_uint32)]


P = C.c_void_p


def _declare(L):
    L.or_philox4x32_10.argtypes = [P, P, P]
    L.or_gen_rays.argtypes = [P, P, C.c_int64, P, P]
    L.or_bvh_build.argtypes = [P]
    L.or_bvh_build.restype = P
    L.or_bvh_free.argtypes = [P]
    L.or_bvh_nodes.argtypes = [P]
    L.or_bvh_nodes.restype = C.c_int64
    L.or_bvh_depth.argtypes = [P]
    L.or_bvh_depth.restype = C.c_int
    L.or_closest.argtypes = [P, P, P, P, C.c_double, C.c_double, C.c_double, P, P, P, P, P]
    L.or_any.argtypes = [P, P, P, P, C.c_double, C.c_double, C.c_double, P]
    L.or_inst_create.argtypes = [P, C.c_int64, P, P, C.c_int]
    L.or_inst_create.restype = P
    L.or_inst_free.argtypes = [P]
    L.or_w2o_f32.argtypes = [P, C.c_int64, P]
    L.or_rotate_f32.argtypes = [P, P, P, P, C.c_int64, P]
    L.or_transform_f32.argtypes = [P, P, P, P, C.c_int64, P]
    L.or_any.restype = C.c_int
    L.or_brdf.argtypes = [P, P, P, P, C.c_double, C.c_double, P]
    L.or_brdf_k.argtypes = [P, P, P, P, C.c_double, C.c_double, C.c_double, P]
    L.or_render_point.argtypes = [P, P, P, P, C.c_int, C.c_double, P, C.c_int64,
                                  P, P, P, P, P, P, P, P]
    L.or_render_rect.argtypes = [P, P, P, P, C.c_int, C.c_uint32, C.c_double, P, C.c_int64,
                                 P, P, P, P, P, P]
    L.or_count_rect.argtypes = [P, P, P, P, P, P, C.c_int, C.c_uint32, P, C.c_int64, P]
    L.or_count_any.argtypes = [P, P, P, P, P, C.c_int64, P, P]
    L.or_resolve_f32.argtypes = [P, C.c_int64, C.c_int, P]
    L.or_transform_f32.argtypes = [P, P, P, P, C.c_int64, P]
    L.or_ggx_D.argtypes = [P, P, C.c_double]
    L.or_ggx_D.restype = C.c_double
    L.or_schlick_g1.argtypes = [C.c_double, C.c_double]
    L.or_schlick_g1.restype = C.c_double
    L.or_schlick_f.argtypes = [C.c_double, C.c_double]
    L.or_schlick_f.restype = C.c_double
    L.or_rect_vis_point.argtypes = [P, P, P, P, P, C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_double, P]
    L.or_rect_vis_point.restype = C.c_int
    L.or_tri_test.argtypes = [P, C.c_uint32, P, P, C.c_double, C.c_double, C.c_double, P]


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def n_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


# ----------------------------------------------------------------------------
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def camera_struct(cam) -> OrCamera:
    c = OrCamera()
    c.eye[:] = [float(x) for x in cam.eye]
    c.target[:] = [float(x) for x in cam.target]
    c.up[:] = [float(x) for x in cam.up]
    c.vfov_deg = float(cam.vfov_deg)
    c.width, c.height, c.ssaa = int(cam.width), int(cam.height), int(cam.ssaa)
    c.seed, c.frame = int(cam.seed), int(cam.frame)
    return c


def gen_rays(cam, samples: np.ndarray):
    s = np.ascontiguousarray(samples, dtype=np.int64)
    o = np.zeros((len(s), 3), np.float32)
    d = np.zeros((len(s), 3), np.float32)
    cs = camera_struct(cam)
    lib().or_gen_rays(C.byref(cs), _p(s), len(s), _p(o), _p(d))
    return o, d


class OracleScene:
    """Holds the FP32 arrays of a scene and (optionally) the oracle's own BVH."""

    def __init__(self, positions, indices, tri_material, materials, use_bvh: bool = True, watertight: bool = False,
                 normals=None):
        self.pos = np.ascontiguousarray(positions, dtype=np.float32)
        self.idx = np.ascontiguousarray(indices, dtype=np.uint32)
        self.tri_mat = np.ascontiguousarray(tri_material, dtype=np.uint32)
        self.mats = np.ascontiguousarray(materials, dtype=np.float32)
        self.s = OrScene(_p(self.pos).value, self.pos.shape[0], _p(self.idx).value, self.idx.shape[0],
                         _p(self.tri_mat).value, _p(self.mats).value, self.mats.shape[0], None,
                         1 if watertight else 0, None)
        self.nrm = None if normals is None else np.ascontiguousarray(normals, dtype=np.float32)
        if self.nrm is not None:
            self.s.nrm = _p(self.nrm).value
        self.watertight = watertight
        self.bvh = lib().or_bvh_build(C.byref(self.s)) if use_bvh else None
        self.inst = None

    @classmethod
    def from_scene(cls, scene, use_bvh: bool = True, watertight: bool = False):
        """watertight: the FP32 side tests triangles with the watertight test (its band model).  The scene's
        vertex normals, if any, give the shading normal."""
        return cls(scene.positions, scene.indices, scene.tri_material, scene.materials, use_bvh, watertight,
                   getattr(scene, "normals", None))

    @classmethod
    def two_level(cls, world_positions, rest_positions, indices, tri_material, materials, tri_range, o2w,
                  use_bvh: bool = True, watertight: bool = False, world_normals=None):
        """A scene whose hit queries go through instances: instance i is triangles tri_range[i] =
        (first, count) of the rest-frame positions, placed by the rigid map [R | t] = o2w[i] (3x4, FP32)
        and tested in its own frame through the world-to-object map w2o_f32(o2w).  Surfaces and
        materials come from the world positions (the FP32 transform of the rest positions)."""
        self = cls(world_positions, indices, tri_material, materials, use_bvh=False, watertight=watertight,
                   normals=world_normals)
        self.rest = cls(rest_positions, indices, tri_material, materials, use_bvh=False, watertight=watertight)
        self.tri_range = np.ascontiguousarray(tri_range, np.uint32).reshape(-1, 2)
        self.w2o = w2o_f32(o2w)
        self.inst = lib().or_inst_create(C.byref(self.rest.s), self.tri_range.shape[0], _p(self.tri_range),
                                         _p(self.w2o), int(use_bvh))
        self.s.inst = self.inst
        self._inst_bvh = use_bvh
        return self

    def _query_bvh(self, brute: bool):
        if self.inst:   # for instanced scenes a non-null pointer selects the per-instance BVHs
            return None if (brute or not self._inst_bvh) else self.inst
        return None if brute else self.bvh

    def set_positions(self, positions):
        """Replace vertex positions (same topology) and rebuild the oracle BVH."""
        self.__init__(positions, self.idx, self.tri_mat, self.mats, self.bvh is not None, self.watertight, self.nrm)

    def __del__(self):
        if getattr(self, "inst", None):
            lib().or_inst_free(self.inst)
            self.inst = None
        if getattr(self, "bvh", None):
            lib().or_bvh_free(self.bvh)
            self.bvh = None

    # -- single-ray queries ------------------------------------------------
    def closest(self, o, d, tmin=0.0, tmax=math.inf, c=4.0, brute=False):
        of = np.ascontiguousarray(o, np.float32)
        df = np.ascontiguousarray(d, np.float32)
        hid = C.c_uint32()
        tuv = np.zeros(3)
        err = np.zeros(3)
        band = C.c_int()
        nc = C.c_int64()
        lib().or_closest(C.byref(self.s), self._query_bvh(brute), _p(of), _p(df), tmin, tmax, c,
                         C.byref(hid), _p(tuv), _p(err), C.byref(band), C.byref(nc))
        return int(hid.value), tuv, err, bool(band.value)

    def tri_test(self, tri, o, d, tmin=0.0, tmax=math.inf, c=4.0):
        """(exact_hit, status 0=certain miss/1=certain hit/2=uncertain, t, u, v, et, eu, ev)"""
        of = np.ascontiguousarray(o, np.float32)
        df = np.ascontiguousarray(d, np.float32)
        out = np.zeros(8)
        lib().or_tri_test(C.byref(self.s), int(tri), _p(of), _p(df), tmin, tmax, c, _p(out))
        return out

    def any_hit(self, o, d, tmin=0.0, tmax=1.0, c=4.0, brute=False):
        od = np.ascontiguousarray(o, np.float64)
        dd = np.ascontiguousarray(d, np.float64)
        band = C.c_int()
        occ = lib().or_any(C.byref(self.s), self._query_bvh(brute), _p(od), _p(dd), tmin, tmax, c,
                           C.byref(band))
        return bool(occ), bool(band.value)

    def rect_vis_point(self, p, n, rect, N, stream=0, pixel=0, seed=0, frame=0, c=4.0, brute=False):
        """(visible count of N light samples, band count) at surface point p with normal n."""
        pp = np.ascontiguousarray(p, np.float64)
        nn = np.ascontiguousarray(n, np.float64)
        R = rect_array(rect)
        bc = C.c_int()
        v = lib().or_rect_vis_point(C.byref(self.s), self._query_bvh(brute), _p(pp), _p(nn), _p(R), int(N),
                                    int(stream), int(pixel), int(seed), int(frame), c, C.byref(bc))
        return int(v), int(bc.value)

    # -- rendering ------------------------------------------------------------
    def render_point(self, cam, lights: np.ndarray, samples: np.ndarray, c: float = 4.0,
                     brute: bool = False, threads: Optional[int] = None):
        """Per-sample primary hit, shadow mask, FP64 radiance and the mask of cast shadow rays (light above the
        surface) for point lights."""
        samples = np.ascontiguousarray(samples, dtype=np.int64)
        n = len(samples)
        L = np.ascontiguousarray(lights, dtype=np.float32).reshape(-1, 6)
        out = dict(hit_id=np.zeros(n, np.uint32), tuv=np.zeros((n, 3)), tuv_err=np.zeros((n, 3)),
                   band_primary=np.zeros(n, np.uint8), mask=np.zeros(n, np.uint32),
                   band_shadow=np.zeros(n, np.uint32), rgb=np.zeros((n, 3)), cast=np.zeros(n, np.uint32))
        cs = camera_struct(cam)
        bvh = self._query_bvh(brute)

        def run(a, b):
            if b <= a:
                return
            lib().or_render_point(C.byref(self.s), bvh, C.byref(cs), _p(L), L.shape[0], c,
                                  _p(samples[a:b]), b - a,
                                  _p(out["hit_id"][a:b]), _p(out["tuv"][a:b]), _p(out["tuv_err"][a:b]),
                                  _p(out["band_primary"][a:b]), _p(out["mask"][a:b]),
                                  _p(out["band_shadow"][a:b]), _p(out["rgb"][a:b]), _p(out["cast"][a:b]))

        _parallel(run, n, threads)
        return out

    def render_rect(self, cam, rect, n_light_samples: int, stream: int, pixels: np.ndarray,
                    c: float = 4.0, brute: bool = False, threads: Optional[int] = None):
        """Per-pixel area-light visibility count (of n_light_samples), band counts and
        the unshadowed centre-point radiance."""
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        n = len(pixels)
        R = rect_array(rect)
        out = dict(hit_id=np.zeros(n, np.uint32), band_primary=np.zeros(n, np.uint8),
                   vis_count=np.zeros(n, np.int32), band_count=np.zeros(n, np.int32),
                   cast_count=np.zeros(n, np.int32), rgb_unshadowed=np.zeros((n, 3)))
        cs = camera_struct(cam)
        bvh = self._query_bvh(brute)

        def run(a, b):
            if b <= a:
                return
            lib().or_render_rect(C.byref(self.s), bvh, C.byref(cs), _p(R), int(n_light_samples), int(stream), c,
                                 _p(pixels[a:b]), b - a, _p(out["hit_id"][a:b]), _p(out["band_primary"][a:b]),
                                 _p(out["vis_count"][a:b]), _p(out["band_count"][a:b]),
                                 _p(out["cast_count"][a:b]), _p(out["rgb_unshadowed"][a:b]))

        _parallel(run, n, threads)
        return out


    def count_rect(self, cam, rect, n_light_samples: int, stream: int, pixels: np.ndarray, nodes: np.ndarray,
                   order: np.ndarray, threads: Optional[int] = None) -> dict:
        """Own-path work of the rect-light shadow rays of `pixels` through a BVH in the library's exported layout
        (nodes: n x 32 uint32, order: slot -> triangle id): rays cast, node visits and triangle tests of each
        ray's own near-first any-hit traversal (FP64)."""
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        nodes = np.ascontiguousarray(nodes, dtype=np.uint32)
        order = np.ascontiguousarray(order, dtype=np.uint32)
        R = rect_array(rect)
        cs = camera_struct(cam)
        bvh = self._query_bvh(False)
        n = len(pixels)
        parts = []
        lock = threading.Lock()

        def run(a, b):
            if b <= a:
                return
            acc = np.zeros(3, np.int64)
            lib().or_count_rect(C.byref(self.s), bvh, _p(nodes), _p(order), C.byref(cs), _p(R), int(n_light_samples),
                                int(stream), _p(pixels[a:b]), b - a, _p(acc))
            with lock:
                parts.append(acc)

        _parallel(run, n, threads)
        tot = np.sum(parts, axis=0) if parts else np.zeros(3, np.int64)
        return {"rays": int(tot[0]), "nodes": int(tot[1]), "tris": int(tot[2])}


    def count_any(self, o, d, nodes: np.ndarray, order: np.ndarray):
        """Instrumented any-hit traversal of segments o + t d (0 < t < 1) through an exported BVH:
        (occluded per segment, node visits, triangle tests)."""
        o = np.ascontiguousarray(np.asarray(o, np.float64).reshape(-1, 3))
        d = np.ascontiguousarray(np.asarray(d, np.float64).reshape(-1, 3))
        nodes = np.ascontiguousarray(nodes, dtype=np.uint32)
        order = np.ascontiguousarray(order, dtype=np.uint32)
        occ = np.zeros(len(o), np.uint8)
        acc = np.zeros(2, np.int64)
        lib().or_count_any(C.byref(self.s), _p(nodes), _p(order), _p(o), _p(d), len(o), _p(occ), _p(acc))
        return occ.astype(bool), int(acc[0]), int(acc[1])


def rect_array(rect) -> np.ndarray:
    return np.ascontiguousarray(np.concatenate([rect.center, rect.edge_u, rect.edge_v, rect.radiance]),
                                dtype=np.float32)


def _parallel(fn, n: int, threads: Optional[int]):
    t = threads or n_threads()
    if t <= 1 or n < 64:
        fn(0, n)
        return
    chunk = max(16, (n + 8 * t - 1) // (8 * t))
    with ThreadPoolExecutor(max_workers=t) as ex:
        list(ex.map(lambda a: fn(a, min(n, a + chunk)), range(0, n, chunk)))


def brdf(n, wo, wi, albedo, rough, metal, k: Optional[float] = None) -> np.ndarray:
    out = np.zeros(3)
    a = [np.ascontiguousarray(x, np.float64) for x in (n, wo, wi, albedo)]
    if k is None:
        lib().or_brdf(_p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]), float(rough), float(metal), _p(out))
    else:
        lib().or_brdf_k(_p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]), float(rough), float(metal), float(k), _p(out))
    return out


def ggx_D(n, h, alpha) -> float:
    a = np.ascontiguousarray(n, np.float64)
    b = np.ascontiguousarray(h, np.float64)
    return float(lib().or_ggx_D(_p(a), _p(b), float(alpha)))


def schlick_g1(x, k) -> float:
    return float(lib().or_schlick_g1(float(x), float(k)))


def schlick_f(f0, c) -> float:
    return float(lib().or_schlick_f(float(f0), float(c)))


def resolve_f32(samples: np.ndarray, n_per: int) -> np.ndarray:
    s = np.ascontiguousarray(samples, dtype=np.float32)
    n_pix = s.size // (4 * n_per)
    out = np.zeros((n_pix, 4), np.float32)
    lib().or_resolve_f32(_p(s), n_pix, n_per, _p(out))
    return out


def w2o_f32(o2w) -> np.ndarray:
    """World-to-object maps [M | m] (n, 12) of rigid maps [R | t] (FP32 mirror: M = R^T, m = -(R^T t))."""
    x = np.ascontiguousarray(o2w, np.float32).reshape(-1, 12)
    out = np.zeros_like(x)
    lib().or_w2o_f32(_p(x), x.shape[0], _p(out))
    return out


def rotate_f32(rest_normals, body_vrange, body_ids, xforms) -> np.ndarray:
    """Vertex normals of moved bodies: the FP32 rotation of the rest normals (no translation)."""
    rest = np.ascontiguousarray(rest_normals, np.float32)
    out = rest.copy()
    vr = np.ascontiguousarray(body_vrange, np.uint32)
    ids = np.ascontiguousarray(body_ids, np.uint32)
    xf = np.ascontiguousarray(xforms, np.float32)
    lib().or_rotate_f32(_p(rest), _p(vr), _p(ids), _p(xf), len(ids), _p(out))
    return out


def transform_f32(rest, body_vrange, body_ids, xforms) -> np.ndarray:
    rest = np.ascontiguousarray(rest, np.float32)
    out = rest.copy()
    vr = np.ascontiguousarray(body_vrange, np.uint32)
    ids = np.ascontiguousarray(body_ids, np.uint32)
    xf = np.ascontiguousarray(xforms, np.float32)
    lib().or_transform_f32(_p(rest), _p(vr), _p(ids), _p(xf), len(ids), _p(out))
    return out
