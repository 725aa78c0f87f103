"""Seeded synthetic scenes, lights and cameras.

This module only *describes inputs*: triangle meshes, instance layouts,
materials, lights and cameras, drawn from ``numpy.random.default_rng(seed)``.
It holds none of the rendering arithmetic (ray generation, intersection,
shading, resolve, refit, denoising); both the HIP library and the CPU oracle
receive the arrays it returns.

The paper's own scenes (surgical robot arms and a suturing phantom of 223K and
550K triangles, and a duplicated scene of more than 7M triangles; Sec. V,
Table I) are not available.  The scenes below stand in for them at the same
triangle scales: hundreds to thousands of rigid mesh instances (the paper's
scene nodes with world transforms, Sec. IV-C) made of procedural spheres,
boxes and tori, over a ground plane, with per-instance metallic-roughness
materials (Sec. IV-B).

Every preset is a pure function of (preset name, seed, overrides).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

F32 = np.float32
U32 = np.uint32


# ----------------------------------------------------------------------------
# Procedural meshes (unit size, FP64), outward winding unless stated.
# ----------------------------------------------------------------------------

def icosphere(subdiv: int):
    """Icosahedron subdivided ``subdiv`` times: 20*4**subdiv triangles on the unit sphere."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / math.sqrt(1 + t * t) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache: Dict[tuple, int] = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts, dtype=np.float64), np.array(faces, dtype=np.int64)


def uv_sphere(n_lat: int, n_lon: int):
    """Unit UV sphere; 2*n_lon*(n_lat-1) triangles, single triangles at the poles."""
    n_lat = max(n_lat, 3)
    n_lon = max(n_lon, 3)
    verts = [(0.0, 1.0, 0.0)]
    for i in range(1, n_lat):
        th = math.pi * i / n_lat
        for j in range(n_lon):
            ph = 2.0 * math.pi * j / n_lon
            verts.append((math.sin(th) * math.cos(ph), math.cos(th), math.sin(th) * math.sin(ph)))
    verts.append((0.0, -1.0, 0.0))
    south = len(verts) - 1

    def ring(i, j):
        return 1 + (i - 1) * n_lon + (j % n_lon)

    faces = []
    for j in range(n_lon):
        faces.append((0, ring(1, j + 1), ring(1, j)))
    for i in range(1, n_lat - 1):
        for j in range(n_lon):
            a, b = ring(i, j), ring(i, j + 1)
            c, d = ring(i + 1, j), ring(i + 1, j + 1)
            faces.append((a, b, d))
            faces.append((a, d, c))
    for j in range(n_lon):
        faces.append((south, ring(n_lat - 1, j), ring(n_lat - 1, j + 1)))
    return np.array(verts, dtype=np.float64), np.array(faces, dtype=np.int64)


def subdivided_box(n: int):
    """Cube [-1,1]^3, each face an n x n grid of quads: 12*n*n triangles."""
    n = max(n, 1)
    verts, faces = [], []
    g = np.linspace(-1.0, 1.0, n + 1)
    # (normal axis, sign): the two tangent axes are chosen so that (a, b, normal) is right-handed
    for axis in range(3):
        for sign in (-1.0, 1.0):
            ta, tb = (axis + 1) % 3, (axis + 2) % 3
            if sign < 0:
                ta, tb = tb, ta
            base = len(verts)
            for i in range(n + 1):
                for j in range(n + 1):
                    p = [0.0, 0.0, 0.0]
                    p[axis] = sign
                    p[ta] = g[i]
                    p[tb] = g[j]
                    verts.append(tuple(p))
            for i in range(n):
                for j in range(n):
                    a = base + i * (n + 1) + j
                    b = a + (n + 1)
                    faces.append((a, b, b + 1))
                    faces.append((a, b + 1, a + 1))
    return np.array(verts, dtype=np.float64), np.array(faces, dtype=np.int64)


def torus(n_u: int, n_v: int, minor: float):
    """Torus of major radius 1 and minor radius ``minor`` about the y axis: 2*n_u*n_v triangles."""
    n_u = max(n_u, 3)
    n_v = max(n_v, 3)
    verts = []
    for i in range(n_u):
        u = 2.0 * math.pi * i / n_u
        for j in range(n_v):
            v = 2.0 * math.pi * j / n_v
            r = 1.0 + minor * math.cos(v)
            verts.append((r * math.cos(u), minor * math.sin(v), r * math.sin(u)))
    faces = []
    for i in range(n_u):
        for j in range(n_v):
            a = i * n_v + j
            b = ((i + 1) % n_u) * n_v + j
            c = ((i + 1) % n_u) * n_v + (j + 1) % n_v
            d = i * n_v + (j + 1) % n_v
            faces.append((a, d, c))
            faces.append((a, c, b))
    return np.array(verts, dtype=np.float64), np.array(faces, dtype=np.int64)


def closed_box_inward(half: float = 0.5):
    """The 12-triangle closed box [-half, half]^3 with inward-facing winding."""
    v, f = subdivided_box(1)
    f = f[:, [0, 2, 1]]  # flip winding -> inward
    return v * half, f


def ground_plane(half: float = 20.0, y: float = 0.0):
    v = np.array([(-half, y, -half), (half, y, -half), (half, y, half), (-half, y, half)], dtype=np.float64)
    f = np.array([(0, 2, 1), (0, 3, 2)], dtype=np.int64)  # normal +y
    return v, f


def _mesh_dims(kind: str, target: int):
    if kind == "sphere":
        n_lat = max(3, int(round(math.sqrt(target / 4.0))))
        return n_lat, 2 * n_lat
    if kind == "box":
        return (max(1, int(round(math.sqrt(target / 12.0)))),)
    if kind == "torus":
        n_v = max(3, int(round(math.sqrt(target / 4.0))))
        return 2 * n_v, n_v
    raise ValueError(kind)


def tri_count(kind: str, target: int) -> int:
    """Exact triangle count of ``mesh_with_tris(kind, target)``."""
    d = _mesh_dims(kind, target)
    if kind == "sphere":
        return 2 * d[1] * (d[0] - 1)
    if kind == "box":
        return 12 * d[0] * d[0]
    return 2 * d[0] * d[1]


def mesh_with_tris(kind: str, target: int, minor: float = 0.3):
    """A procedural mesh of the given kind with roughly ``target`` triangles."""
    d = _mesh_dims(kind, target)
    if kind == "sphere":
        return uv_sphere(*d)
    if kind == "box":
        return subdivided_box(d[0])
    return torus(d[0], d[1], minor)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation (Shoemake's subgroup algorithm, Graphics Gems III)."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1 - u1), math.sqrt(u1)
    x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def random_material(rng: np.random.Generator) -> np.ndarray:
    """albedo ~ U[0.2,0.9]^3, roughness ~ U[0.05,1], metallic ~ Bernoulli(0.3)."""
    alb = rng.uniform(0.2, 0.9, 3)
    r = rng.uniform(0.05, 1.0)
    m = 1.0 if rng.random() < 0.3 else 0.0
    return np.array([alb[0], alb[1], alb[2], r, m], dtype=np.float64)


# ----------------------------------------------------------------------------
# Scene container
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Camera:
    eye: tuple
    target: tuple
    up: tuple
    vfov_deg: float
    width: int
    height: int
    ssaa: int = 1          # 1 = one centred sample, 2 = 2x2 stratified jitter
    seed: int = 0
    frame: int = 0

    @property
    def spp(self) -> int:
        return self.ssaa * self.ssaa

    @property
    def n_samples(self) -> int:
        return self.width * self.height * self.spp


@dataclasses.dataclass
class RectLight:
    center: tuple
    edge_u: tuple
    edge_v: tuple
    radiance: tuple


@dataclasses.dataclass
class Scene:
    positions: np.ndarray            # (Nv, 3) float32, world space
    indices: np.ndarray              # (Nt, 3) uint32
    tri_material: np.ndarray         # (Nt,) uint32
    materials: np.ndarray            # (M, 5) float32: albedo rgb, roughness, metallic
    body_vertex_range: np.ndarray    # (B, 2) uint32: first vertex, count (one body per instance)
    body_tri_range: np.ndarray       # (B, 2) uint32
    point_lights: np.ndarray         # (L, 6) float32: position xyz, intensity rgb
    rect_light: Optional[RectLight]
    cameras: List[Camera]
    name: str = ""
    normals: Optional[np.ndarray] = None   # (Nv, 3) float32 vertex normals, or None (flat shading)

    @property
    def n_tris(self) -> int:
        return int(self.indices.shape[0])

    @property
    def n_verts(self) -> int:
        return int(self.positions.shape[0])


class _Builder:
    def __init__(self):
        self.v: List[np.ndarray] = []
        self.f: List[np.ndarray] = []
        self.mat: List[np.ndarray] = []
        self.vr: List[tuple] = []
        self.tr: List[tuple] = []
        self.nv = 0
        self.nt = 0

    def add(self, verts: np.ndarray, faces: np.ndarray, mat_id: int, body: bool = True):
        self.v.append(verts)
        self.f.append(faces + self.nv)
        self.mat.append(np.full(len(faces), mat_id, dtype=np.int64))
        if body:
            self.vr.append((self.nv, len(verts)))
            self.tr.append((self.nt, len(faces)))
        self.nv += len(verts)
        self.nt += len(faces)

    def finish(self, materials, lights, rect, cams, name) -> Scene:
        pos = np.concatenate(self.v).astype(F32)
        idx = np.concatenate(self.f).astype(U32)
        return Scene(
            positions=np.ascontiguousarray(pos),
            indices=np.ascontiguousarray(idx),
            tri_material=np.concatenate(self.mat).astype(U32),
            materials=np.asarray(materials, dtype=F32).reshape(-1, 5),
            body_vertex_range=np.asarray(self.vr, dtype=U32).reshape(-1, 2),
            body_tri_range=np.asarray(self.tr, dtype=U32).reshape(-1, 2),
            point_lights=np.asarray(lights, dtype=F32).reshape(-1, 6),
            rect_light=rect,
            cameras=cams,
            name=name,
        )


def vertex_normals(positions: np.ndarray, indices: np.ndarray) -> np.ndarray:
    """Area-weighted average of the faces' normals at each vertex (FP64, unit, stored FP32): smooth on
    meshes that share vertices (spheres, tori), the face normal where faces own their vertices (boxes)."""
    p = positions.astype(np.float64)
    f = indices.astype(np.int64)
    fn = np.cross(p[f[:, 1]] - p[f[:, 0]], p[f[:, 2]] - p[f[:, 0]])
    acc = np.zeros_like(p)
    for k in range(3):
        np.add.at(acc, f[:, k], fn)
    ln = np.linalg.norm(acc, axis=1, keepdims=True)
    acc = np.where(ln > 0, acc / np.where(ln > 0, ln, 1.0), np.array([0.0, 1.0, 0.0]))
    return np.ascontiguousarray(acc.astype(F32))


def with_vertex_normals(scene: "Scene") -> "Scene":
    """The scene with vertex normals computed from its current positions (smooth shading)."""
    return dataclasses.replace(scene, normals=vertex_normals(scene.positions, scene.indices),
                               name=scene.name + "_smooth")


def tiny_box_scene(seed: int = 0, width: int = 128, height: int = 128) -> Scene:
    """Closed 12-triangle box (inward normals) + 1280-triangle icosphere of radius 0.3; one point light."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    bv, bf = closed_box_inward(0.5)
    b.add(bv, bf, 0)
    sv, sf = icosphere(3)
    b.add(sv * 0.3, sf, 1)
    mats = [random_material(rng), random_material(rng)]
    lights = [(0.0, 0.45, 0.0, 1.0, 1.0, 1.0)]
    cam = Camera(eye=(0.35, 0.2, 0.45), target=(0.0, -0.15, 0.0), up=(0.0, 1.0, 0.0),
                 vfov_deg=75.0, width=width, height=height, ssaa=1, seed=seed)
    return b.finish(mats, lights, None, [cam], "tiny_box")


KINDS = ("sphere", "box", "torus")


def draw_instances(n_instances: int, rng: np.random.Generator):
    """Per-instance kind, torus minor radius, size, rotation and position (drawn before any mesh is built)."""
    out = []
    for _ in range(n_instances):
        kind = KINDS[int(rng.integers(len(KINDS)))]
        minor = float(rng.uniform(0.2, 0.45))
        size = float(rng.uniform(0.2, 1.0))
        rot = random_rotation(rng)
        pos = rng.uniform((-10.0, 0.0, -10.0), (10.0, 20.0, 10.0))
        out.append((kind, minor, size, rot, pos))
    return out


def instanced_scene(params, tri_counts) -> _Builder:
    """Instances of procedural meshes at rigid poses in [-10,10]x[0,20]x[-10,10], over a 40x40 m ground."""
    b = _Builder()
    gv, gf = ground_plane(20.0)
    b.add(gv, gf, 0)
    for i, (kind, minor, size, rot, pos) in enumerate(params):
        v, f = mesh_with_tris(kind, int(tri_counts[i]), minor)
        b.add(v * size @ rot.T + pos, f, 1 + i)
    return b


def random_point_lights(rng: np.random.Generator, n: int, intensity: float = 400.0):
    out = []
    for _ in range(n):
        p = rng.uniform((-10.0, 15.0, -10.0), (10.0, 25.0, 10.0))
        out.append((p[0], p[1], p[2], intensity, intensity, intensity))
    return out


# A 1x1 m light on the camera side of the instance volume, tilted to face it (normal edge_u x edge_v
# = (0.5, -0.707, 0.5)).  Directly above the 20 m cube of instances almost every visible point would be
# in shadow (the instances leave a ~5 m mean free path), so the light sits outside the volume.
_S = 0.7071067811865476
DEFAULT_RECT = RectLight(center=(-12.0, 26.0, -22.0), edge_u=(_S, 0.0, -_S), edge_v=(0.5, _S, 0.5),
                         radiance=(100.0, 100.0, 100.0))
# A horizontal 1x1 m light facing down, for closed-form checks.
OVERHEAD_RECT = RectLight(center=(0.0, 21.0, 0.0), edge_u=(1.0, 0.0, 0.0), edge_v=(0.0, 0.0, 1.0),
                          radiance=(100.0, 100.0, 100.0))


def city_scene(seed: int = 0, n_instances: int = 400, width: int = 1920, height: int = 1080,
               ssaa: int = 2, n_lights: int = 4) -> Scene:
    """~1.1M triangles: 400 instances of 500-5000 triangles, 4 point lights, 1080p with 2x2 jitter."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(500, 5001, n_instances)
    b = instanced_scene(draw_instances(n_instances, rng), counts)
    mats = [random_material(rng) for _ in range(n_instances + 1)]
    lights = random_point_lights(rng, n_lights)
    cam = Camera(eye=(0.0, 10.0, -28.0), target=(0.0, 5.0, 0.0), up=(0.0, 1.0, 0.0),
                 vfov_deg=50.0, width=width, height=height, ssaa=ssaa, seed=seed)
    return b.finish(mats, lights, None, [cam], "city_1M")


def big_scene(seed: int = 0, n_instances: int = 1500, total_tris: int = 7_300_000,
              width: int = 1920, height: int = 1080) -> Scene:
    """~7.3M triangles: 1500 instances, log-uniform 2k-10k triangles rescaled to the total; one rect light."""
    rng = np.random.default_rng(seed)
    raw = np.exp(rng.uniform(math.log(2000.0), math.log(10000.0), n_instances))
    params = draw_instances(n_instances, rng)
    scale = total_tris / raw.sum()
    for _ in range(8):  # rescale so that the realised total is within 0.1% of the target
        counts = np.maximum(raw * scale, 12).astype(np.int64)
        got = 2 + sum(tri_count(p[0], int(c)) for p, c in zip(params, counts))
        if abs(got - total_tris) <= 1e-3 * total_tris:
            break
        scale *= total_tris / got
    b = instanced_scene(params, counts)
    mats = [random_material(rng) for _ in range(n_instances + 1)]
    cam = Camera(eye=(0.0, 10.0, -28.0), target=(0.0, 5.0, 0.0), up=(0.0, 1.0, 0.0),
                 vfov_deg=50.0, width=width, height=height, ssaa=1, seed=seed)
    return b.finish(mats, [], DEFAULT_RECT, [cam], "big_7M")


def orbit_cameras(rng: np.random.Generator, n: int, radius: float = 30.0, center=(0.0, 10.0, 0.0),
                  sizes=(256, 384, 512, 768, 1024), seed: int = 0) -> List[Camera]:
    """Cameras on the upper half of a sphere around ``center``, square resolutions drawn from ``sizes``."""
    cams = []
    for i in range(n):
        while True:
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            if d[1] > 0.05:
                break
        eye = np.asarray(center) + radius * d
        r = int(sizes[int(rng.integers(len(sizes)))])
        cams.append(Camera(eye=tuple(float(x) for x in eye), target=tuple(center), up=(0.0, 1.0, 0.0),
                           vfov_deg=50.0, width=r, height=r, ssaa=1, seed=seed + i))
    return cams


def batch_scenes(seed: int = 0, scale: float = 1.0, n_views: int = 64):
    """Four scenes of 0.1M/0.5M/1M/2M triangles (36/182/364/727 instances), 1-4 point lights each,
    and ``n_views`` orbit cameras; camera i renders scene i mod 4."""
    rng = np.random.default_rng(seed)
    scenes = []
    for k, n_inst in enumerate((36, 182, 364, 727)):
        n_inst = max(1, int(round(n_inst * scale)))
        counts = rng.integers(500, 5001, n_inst)
        b = instanced_scene(draw_instances(n_inst, rng), counts)
        mats = [random_material(rng) for _ in range(n_inst + 1)]
        lights = random_point_lights(rng, int(rng.integers(1, 5)))
        scenes.append(b.finish(mats, lights, None, [], f"batch_{k}"))
    cams = orbit_cameras(rng, n_views, seed=seed)
    for i, c in enumerate(cams):
        scenes[i % 4].cameras.append(c)
    return scenes, cams


def small_random_scene(seed: int, n_instances: int = 6, tris_lo: int = 20, tris_hi: int = 300,
                       width: int = 37, height: int = 29, ssaa: int = 1, n_lights: int = 2) -> Scene:
    """A small instanced scene for brute-force and parity checks (ragged image sizes on purpose)."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(tris_lo, tris_hi + 1, n_instances)
    b = instanced_scene(draw_instances(n_instances, rng), counts)
    mats = [random_material(rng) for _ in range(n_instances + 1)]
    lights = random_point_lights(rng, n_lights)
    cam = Camera(eye=(0.0, 10.0, -28.0), target=(0.0, 5.0, 0.0), up=(0.0, 1.0, 0.0),
                 vfov_deg=50.0, width=width, height=height, ssaa=ssaa, seed=seed)
    return b.finish(mats, lights, DEFAULT_RECT, [cam], f"small_{seed}")


# ----------------------------------------------------------------------------
# Animated rigid bodies: per-frame 3x4 transforms applied to rest positions.
# ----------------------------------------------------------------------------

def _axis_angle(axis: np.ndarray, ang: float) -> np.ndarray:
    x, y, z = axis
    c, s = math.cos(ang), math.sin(ang)
    C = 1 - c
    return np.array([[c + x * x * C, x * y * C - z * s, x * z * C + y * s],
                     [y * x * C + z * s, c + y * y * C, y * z * C - x * s],
                     [z * x * C - y * s, z * y * C + x * s, c + z * z * C]])


class RigidAnimation:
    """Per-frame rigid motion of ``n_bodies`` bodies chosen by seed.

    Each frame composes onto each moving body a displacement of uniform direction and
    magnitude U[0, max_disp] and a rotation about a uniform axis through the body's
    current centroid by U[0, max_rot_deg].  ``transforms(frame)`` returns, for every
    moving body, the FP32 3x4 matrix [R | t] that maps the body's rest positions to
    frame ``frame`` (rest = the scene as generated)."""

    def __init__(self, scene: Scene, n_bodies: int, seed: int = 0,
                 max_disp: float = 0.05, max_rot_deg: float = 2.0):
        rng = np.random.default_rng(seed + 7919)
        n_all = scene.body_vertex_range.shape[0]
        self.body_ids = np.sort(rng.choice(np.arange(1, n_all), size=min(n_bodies, n_all - 1), replace=False)).astype(U32)
        self.centroids = np.stack([
            scene.positions[int(a):int(a) + int(n)].astype(np.float64).mean(axis=0)
            for a, n in scene.body_vertex_range[self.body_ids]])
        self.seed = seed
        self.max_disp = max_disp
        self.max_rot = math.radians(max_rot_deg)
        self._R = np.tile(np.eye(3), (len(self.body_ids), 1, 1))
        self._t = np.zeros((len(self.body_ids), 3))
        self._frame = 0
        self._rng = np.random.default_rng(seed + 104729)

    def _step(self):
        rng = self._rng
        for i in range(len(self.body_ids)):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            disp = d * rng.uniform(0.0, self.max_disp)
            ax = rng.normal(size=3)
            ax /= np.linalg.norm(ax)
            dR = _axis_angle(ax, rng.uniform(0.0, self.max_rot))
            c = self._R[i] @ self.centroids[i] + self._t[i]      # current centroid
            # x' = dR (x - c) + c + disp  composed with x = R x0 + t
            self._R[i] = dR @ self._R[i]
            self._t[i] = dR @ (self._t[i] - c) + c + disp
        self._frame += 1

    def transforms(self, frame: int) -> np.ndarray:
        if frame < self._frame:
            raise ValueError("frames must be requested in increasing order")
        while self._frame < frame:
            self._step()
        out = np.concatenate([self._R, self._t[:, :, None]], axis=2)  # (B, 3, 4)
        return np.ascontiguousarray(out.reshape(-1, 12).astype(F32))


# ----------------------------------------------------------------------------
# Presets mirroring the five workloads.
# ----------------------------------------------------------------------------

PRESETS = {
    "tiny_box": "12-triangle closed box + 1280-triangle icosphere, 128x128, 1 spp, one point light",
    "city_1M": "~1.1M triangles, 400 instances, 1920x1080 with 2x2 jitter, 4 point lights",
    "big_7M": "~7.3M triangles, 1500 instances, 1920x1080, one 1x1 m rect light",
    "batch_64": "64 views (256..1024 square) over 4 scenes of 0.1M/0.5M/1M/2M triangles",
    "anim_7M": "big_7M with 300 rigid bodies moving per frame, 16 views",
}


def make(preset: str, seed: int = 0, **kw):
    if preset == "tiny_box":
        return tiny_box_scene(seed, **kw)
    if preset == "city_1M":
        return city_scene(seed, **kw)
    if preset == "big_7M":
        return big_scene(seed, **kw)
    if preset == "batch_64":
        return batch_scenes(seed, **kw)
    raise KeyError(preset)
