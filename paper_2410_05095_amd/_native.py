"""ctypes binding of libraycast.so (the C ABI in include/raycast.h).

Argument marshalling only: torch provides device memory and the current HIP stream; every
step of the rendering path runs in the library's HIP kernels.  There is no fallback: if the
library is not built or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libraycast.so")

RC_FLAG_TIMING = 1
RC_FLAG_PER_LANE = 4
RC_FLAG_GRAPH = 2
RC_FLAG_NO_SHADE = 8
RC_FLAG_COUNT = 16
RC_FLAG_WAVE = 32
NO_HIT = 0xFFFFFFFF


class RcError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


F3 = C.c_float * 3


class RcSceneDesc(C.Structure):
    _fields_ = [("positions", C.c_void_p), ("n_vertices", C.c_uint32), ("indices", C.c_void_p),
                ("n_tris", C.c_uint32), ("tri_material", C.c_void_p), ("materials", C.c_void_p),
                ("n_materials", C.c_uint32), ("body_vertex_range", C.c_void_p), ("n_bodies", C.c_uint32),
                ("normals", C.c_void_p)]


class RcBuildOpts(C.Structure):
    _fields_ = [("bins", C.c_uint32), ("max_leaf", C.c_uint32), ("node_cost", C.c_float), ("method", C.c_uint32),
                ("flags", C.c_uint32)]


class RcBvhStats(C.Structure):
    _fields_ = [("n_nodes", C.c_uint64), ("n_leaves", C.c_uint64), ("n_tris", C.c_uint64),
                ("depth", C.c_uint32), ("max_stack", C.c_uint32), ("sah_cost", C.c_double),
                ("build_ms", C.c_double), ("n_instances", C.c_uint32), ("tlas_levels", C.c_uint32),
                ("tlas_root", C.c_uint32), ("reserved", C.c_uint32)]


class RcCamera(C.Structure):
    _fields_ = [("eye", F3), ("target", F3), ("up", F3), ("vfov_deg", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32), ("ssaa", C.c_int32), ("seed", C.c_uint32), ("frame", C.c_uint32)]


class RcPointLight(C.Structure):
    _fields_ = [("position", F3), ("intensity", F3)]


class RcRectLight(C.Structure):
    _fields_ = [("center", F3), ("edge_u", F3), ("edge_v", F3), ("radiance", F3)]


class RcRenderOpts(C.Structure):
    _fields_ = [("area_samples", C.c_uint32), ("area_stream", C.c_uint32), ("flags", C.c_uint32)]


class RcOutputs(C.Structure):
    _fields_ = [("d_rgba", C.c_void_p), ("d_hit", C.c_void_p), ("d_shadow", C.c_void_p),
                ("d_visibility", C.c_void_p), ("d_sample_rgba", C.c_void_p)]


class RcView(C.Structure):
    _fields_ = [("scene", C.c_uint32), ("camera", RcCamera), ("light_first", C.c_uint32), ("n_lights", C.c_uint32),
                ("d_rgba", C.c_void_p), ("d_hit", C.c_void_p), ("d_shadow", C.c_void_p)]


class RcTune(C.Structure):
    _fields_ = [("tile_w", C.c_uint32), ("tile_h", C.c_uint32), ("queue_depth", C.c_uint32),
                ("min_rays", C.c_uint32), ("waves_per_simd", C.c_uint32), ("passes", C.c_uint32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class RcStageTimes(C.Structure):
    _fields_ = [("ms", C.c_float * 8), ("rays", C.c_uint64 * 2), ("node_visits", C.c_uint64 * 2),
                ("tri_tests", C.c_uint64 * 2)]


P = C.c_void_p
PP = C.POINTER(C.c_void_p)

# name -> (restype, argtypes); every symbol declared in include/raycast.h
SIGNATURES = {
    "rc_status_string": (C.c_char_p, [C.c_int]),
    "rc_version": (C.c_int, []),
    "rc_create": (C.c_int, [PP, C.c_int, P]),
    "rc_destroy": (C.c_int, [P]),
    "rc_set_stream": (C.c_int, [P, P]),
    "rc_get_last_error": (C.c_int, [P]),
    "rc_scene_create": (C.c_int, [P, C.POINTER(RcSceneDesc), PP]),
    "rc_scene_destroy": (C.c_int, [P, P]),
    "rc_bvh_build": (C.c_int, [P, P, C.POINTER(RcBuildOpts)]),
    "rc_scene_set_transforms": (C.c_int, [P, P, P, P, C.c_uint32]),
    "rc_bvh_refit": (C.c_int, [P, P]),
    "rc_tlas_rebuild": (C.c_int, [P, P, P]),
    "rc_tlas_export": (C.c_int, [P, P, P]),
    "rc_bvh_get_stats": (C.c_int, [P, P, C.POINTER(RcBvhStats)]),
    "rc_bvh_export": (C.c_int, [P, P, P, P]),
    "rc_render": (C.c_int, [P, P, C.POINTER(RcCamera), C.POINTER(RcPointLight), C.c_uint32,
                            C.POINTER(RcRectLight), C.POINTER(RcRenderOpts), C.POINTER(RcOutputs)]),
    "rc_get_stage_times": (C.c_int, [P, C.POINTER(RcStageTimes)]),
    "rc_camera_rays": (C.c_int, [P, C.POINTER(RcCamera), P, P]),
    "rc_scene_get_positions": (C.c_int, [P, P, P]),
    "rc_denoiser_n_params": (C.c_int, []),
    "rc_denoiser_create": (C.c_int, [P, C.c_uint32, PP]),
    "rc_denoiser_destroy": (C.c_int, [P, P]),
    "rc_denoiser_get_params": (C.c_int, [P, P, P]),
    "rc_denoiser_set_params": (C.c_int, [P, P, P]),
    "rc_denoiser_get_grads": (C.c_int, [P, P, P]),
    "rc_postprocess": (C.c_int, [P, P, C.c_uint32, C.c_uint32, C.c_uint32, P]),
    "rc_postprocess_noalloc": (C.c_int, [P, P, C.c_uint32, C.c_uint32, C.c_uint32, P]),
    "rc_denoiser_infer": (C.c_int, [P, P, P, C.c_uint32, C.c_uint32, C.c_uint32, P]),
    "rc_denoiser_infer_fp32": (C.c_int, [P, P, P, C.c_uint32, C.c_uint32, C.c_uint32, P]),
    "rc_denoiser_train_step": (C.c_int, [P, P, P, P, P, C.c_uint32, C.c_uint32, C.c_uint32, C.c_float,
                                         C.POINTER(C.c_float)]),
    "rc_denoiser_save": (C.c_int, [P, P, C.c_char_p]),
    "rc_denoiser_load": (C.c_int, [P, P, C.c_char_p]),
    "rc_pack_features": (C.c_int, [P, P, C.POINTER(RcCamera), P, P, C.c_float, P]),
    "rc_shade": (C.c_int, [P, P, C.POINTER(RcCamera), C.POINTER(RcPointLight), C.c_uint32, C.POINTER(RcRectLight),
                           P, P, P, P, P]),
    "rc_render_batch": (C.c_int, [P, P, C.c_uint32, C.POINTER(RcView), C.c_uint32, C.POINTER(RcPointLight),
                                  C.c_uint32, C.POINTER(RcTune), C.c_uint32]),
    "rc_autotune": (C.c_int, [P, P, C.c_uint32, C.POINTER(RcView), C.c_uint32, C.POINTER(RcPointLight), C.c_uint32,
                              C.POINTER(RcTune), C.c_uint32, C.c_uint32, C.c_char_p, C.POINTER(RcTune),
                              C.POINTER(C.c_float)]),
}

_lib = None


def lib():
    """Load libraycast.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first (paper_2410_05095_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().rc_status_string(int(status)).decode()


def check(status: int, where: str):
    if status != 0:
        raise RcError(status, where)


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _dptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def camera_struct(cam) -> RcCamera:
    c = RcCamera()
    c.eye[:] = [float(x) for x in cam.eye]
    c.target[:] = [float(x) for x in cam.target]
    c.up[:] = [float(x) for x in cam.up]
    c.vfov_deg = float(cam.vfov_deg)
    c.width, c.height, c.ssaa = int(cam.width), int(cam.height), int(cam.ssaa)
    c.seed, c.frame = int(cam.seed), int(cam.frame)
    return c


def rect_struct(rect) -> RcRectLight:
    r = RcRectLight()
    r.center[:] = [float(x) for x in rect.center]
    r.edge_u[:] = [float(x) for x in rect.edge_u]
    r.edge_v[:] = [float(x) for x in rect.edge_v]
    r.radiance[:] = [float(x) for x in rect.radiance]
    return r


def light_array(lights) -> Optional[C.Array]:
    L = np.asarray(lights, np.float32).reshape(-1, 6)
    if len(L) == 0:
        return None
    arr = (RcPointLight * len(L))()
    for i, row in enumerate(L):
        arr[i].position[:] = [float(x) for x in row[:3]]
        arr[i].intensity[:] = [float(x) for x in row[3:]]
    return arr


class Context:
    """A library context bound to a device and to torch's current stream at each call."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to torch: the HIP rendering path needs an MI355X (gfx950)")
        self.device = device
        torch.cuda.set_device(device)
        h = C.c_void_p()
        check(lib().rc_create(C.byref(h), device, C.c_void_p(torch.cuda.current_stream(device).cuda_stream)),
              "rc_create")
        self.h = h

    def _sync_stream(self):
        st = self.torch.cuda.current_stream(self.device).cuda_stream
        check(lib().rc_set_stream(self.h, C.c_void_p(st)), "rc_set_stream")

    def close(self):
        if getattr(self, "h", None):
            lib().rc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> int:
        return int(lib().rc_get_last_error(self.h))

    def scene(self, positions, indices, tri_material, materials, body_vertex_range=None, normals=None) -> "Scene":
        return Scene(self, positions, indices, tri_material, materials, body_vertex_range, normals)

    def scene_from(self, sc) -> "Scene":
        return Scene(self, sc.positions, sc.indices, sc.tri_material, sc.materials, sc.body_vertex_range,
                     getattr(sc, "normals", None))

    def render(self, scene: "Scene", cam, lights=(), rect=None, area_samples: int = 0, area_stream: int = 0,
               timing: bool = False, sample_rgba: bool = False, out: Optional[dict] = None,
               per_lane: bool = False, shade: bool = True, count: bool = False, wave: bool = False) -> dict:
        """One view through rc_render: camera rays, shadow rays (point lights, and the rect light with
        `area_samples` samples per pixel), shading and resolve into `out` (allocated when missing).
        per_lane / wave force the per-lane or the wave-uniform shadow kernels (by default the library picks by
        pass size); count gathers ray, node and triangle counts for stage_times(); shade=False stops after the
        visibility stages."""
        torch = self.torch
        self._sync_stream()
        W, H, S = int(cam.width), int(cam.height), int(cam.ssaa) ** 2
        Larr = light_array(lights)
        nl = 0 if Larr is None else len(Larr)
        dev = torch.device("cuda", self.device)
        if out is None:
            out = {}
        def get(name, shape, dtype):
            t = out.get(name)
            if t is None or tuple(t.shape) != shape or t.dtype != dtype:
                t = torch.empty(shape, dtype=dtype, device=dev)
                out[name] = t
            return t
        rgba = get("rgba", (H, W, 4), torch.float32)
        hit = get("hit", (H * W * S, 4), torch.int32)
        shadow = get("shadow", (H * W * S,), torch.int32) if nl else None
        vis = get("visibility", (H, W), torch.float32) if rect is not None else None
        srgba = get("sample_rgba", (H * W * S, 4), torch.float32) if sample_rgba else None
        o = RcOutputs(_dptr(rgba), _dptr(hit), _dptr(shadow), _dptr(vis), _dptr(srgba))
        flags = (RC_FLAG_TIMING if timing else 0) | (RC_FLAG_PER_LANE if per_lane else 0) | \
            (0 if shade else RC_FLAG_NO_SHADE) | (RC_FLAG_COUNT if count else 0) | (RC_FLAG_WAVE if wave else 0)
        opts = RcRenderOpts(int(area_samples), int(area_stream), flags)
        camc = camera_struct(cam)
        rc = rect_struct(rect) if rect is not None else None
        check(lib().rc_render(self.h, scene.h, C.byref(camc), Larr, nl, C.byref(rc) if rc is not None else None,
                              C.byref(opts), C.byref(o)), "rc_render")
        return out

    def shade(self, scene: "Scene", cam, out: dict, lights=(), rect=None, visibility=None):
        """Re-run shading + resolve into out["rgba"] from out["hit"], out["shadow"] and `visibility`."""
        self._sync_stream()
        Larr = light_array(lights)
        nl = 0 if Larr is None else len(Larr)
        vis = visibility if visibility is not None else out.get("visibility")
        camc = camera_struct(cam)
        rc = rect_struct(rect) if rect is not None else None
        check(lib().rc_shade(self.h, scene.h, C.byref(camc), Larr, nl, C.byref(rc) if rc is not None else None,
                             C.c_void_p(out["hit"].data_ptr()), _dptr(out.get("shadow")) if nl else None,
                             _dptr(vis), C.c_void_p(out["rgba"].data_ptr()), None), "rc_shade")
        return out

    def camera_rays(self, cam):
        torch = self.torch
        self._sync_stream()
        n = int(cam.width) * int(cam.height) * int(cam.ssaa) ** 2
        o = torch.empty((n, 3), dtype=torch.float32, device=torch.device("cuda", self.device))
        d = torch.empty_like(o)
        camc = camera_struct(cam)
        check(lib().rc_camera_rays(self.h, C.byref(camc), C.c_void_p(o.data_ptr()), C.c_void_p(d.data_ptr())),
              "rc_camera_rays")
        return o, d

    # -- batched rendering ----------------------------------------------------
    def _batch_args(self, scenes, views, outs):
        """views: list of (scene index, camera, light_first, n_lights); outs: list of dicts (allocated
        here when empty).  Returns the ctypes arrays."""
        torch = self.torch
        dev = torch.device("cuda", self.device)
        sarr = (C.c_void_p * len(scenes))(*[s.h.value for s in scenes])
        varr = (RcView * len(views))()
        for i, (si, cam, lf, nl) in enumerate(views):
            W, H, S = int(cam.width), int(cam.height), int(cam.ssaa) ** 2
            o = outs[i]
            if o.get("rgba") is None or tuple(o["rgba"].shape) != (H, W, 4):
                o["rgba"] = torch.empty((H, W, 4), dtype=torch.float32, device=dev)
                o["hit"] = torch.empty((H * W * S, 4), dtype=torch.int32, device=dev)
                o["shadow"] = torch.empty((H * W * S,), dtype=torch.int32, device=dev) if nl else None
            varr[i].scene = int(si)
            varr[i].camera = camera_struct(cam)
            varr[i].light_first = int(lf)
            varr[i].n_lights = int(nl)
            varr[i].d_rgba = o["rgba"].data_ptr()
            varr[i].d_hit = o["hit"].data_ptr()
            varr[i].d_shadow = o["shadow"].data_ptr() if nl else None
        return sarr, varr

    def render_batch(self, scenes, views, lights, tune: Optional[dict] = None, graph: bool = False,
                     timing: bool = False, outs: Optional[list] = None, count: bool = False) -> list:
        self._sync_stream()
        if outs is None:
            outs = [{} for _ in views]
        sarr, varr = self._batch_args(scenes, views, outs)
        Larr = light_array(lights)
        nl = 0 if Larr is None else len(Larr)
        t = RcTune(**tune) if tune else None
        flags = (RC_FLAG_GRAPH if graph else 0) | (RC_FLAG_TIMING if timing else 0) | (RC_FLAG_COUNT if count else 0)
        check(lib().rc_render_batch(self.h, sarr, len(scenes), varr, len(views), Larr, nl,
                                    C.byref(t) if t is not None else None, flags), "rc_render_batch")
        return outs

    def autotune(self, scenes, views, lights, candidates=None, reps: int = 3, cache_path: Optional[str] = None,
                 outs: Optional[list] = None):
        self._sync_stream()
        if outs is None:
            outs = [{} for _ in views]
        sarr, varr = self._batch_args(scenes, views, outs)
        Larr = light_array(lights)
        nl = 0 if Larr is None else len(Larr)
        cand = None
        if candidates:
            cand = (RcTune * len(candidates))(*[RcTune(**c) for c in candidates])
        best = RcTune()
        ms = C.c_float()
        check(lib().rc_autotune(self.h, sarr, len(scenes), varr, len(views), Larr, nl, cand,
                                len(candidates) if candidates else 0, int(reps),
                                cache_path.encode() if cache_path else None, C.byref(best), C.byref(ms)),
              "rc_autotune")
        return best.as_dict(), float(ms.value)

    def postprocess(self, rgba, fxaa: bool = True, out=None):
        """Display post pass: (H, W, 4) float32 linear RGBA on the GPU -> (H, W, 4) uint8 sRGB (Reinhard tone
        map, sRGB encoding, then FXAA unless fxaa=False)."""
        torch = self.torch
        assert rgba.dtype == torch.float32 and rgba.is_contiguous() and rgba.shape[-1] == 4
        H, W = int(rgba.shape[0]), int(rgba.shape[1])
        if out is None:
            out = torch.empty((H, W, 4), dtype=torch.uint8, device=rgba.device)
        self._sync_stream()
        check(lib().rc_postprocess(self.h, C.c_void_p(rgba.data_ptr()), W, H, 1 if fxaa else 0,
                                   C.c_void_p(out.data_ptr())), "rc_postprocess")
        return out

    def postprocess_noalloc(self, rgba, out, fxaa: bool = True):
        """rc_postprocess_noalloc: the display post pass into the caller's (H, W, 4) uint8 `out`, with the FXAA
        intermediate in the library's fixed per-GPU scratch (no allocation)."""
        assert rgba.dtype == self.torch.float32 and rgba.is_contiguous() and rgba.shape[-1] == 4
        assert out.dtype == self.torch.uint8 and out.is_contiguous() and out.shape == rgba.shape
        H, W = int(rgba.shape[0]), int(rgba.shape[1])
        self._sync_stream()
        check(lib().rc_postprocess_noalloc(self.h, C.c_void_p(rgba.data_ptr()), W, H, 1 if fxaa else 0,
                                           C.c_void_p(out.data_ptr())), "rc_postprocess_noalloc")
        return out

    def stage_times(self) -> dict:
        t = RcStageTimes()
        check(lib().rc_get_stage_times(self.h, C.byref(t)), "rc_get_stage_times")
        return {"primary_ms": t.ms[0], "shadow_ms": t.ms[1], "shade_ms": t.ms[2], "total_ms": t.ms[3],
                "primary_rays": int(t.rays[0]), "shadow_rays": int(t.rays[1]),
                "primary_nodes": int(t.node_visits[0]), "shadow_nodes": int(t.node_visits[1]),
                "primary_tris": int(t.tri_tests[0]), "shadow_tris": int(t.tri_tests[1])}


class Scene:
    def __init__(self, ctx: Context, positions, indices, tri_material, materials, body_vertex_range=None,
                 normals=None):
        self.ctx = ctx
        self.pos = np.ascontiguousarray(positions, np.float32)
        self.idx = np.ascontiguousarray(indices, np.uint32)
        self.tm = np.ascontiguousarray(tri_material, np.uint32)
        self.mats = np.ascontiguousarray(materials, np.float32)
        self.bvr = None if body_vertex_range is None else np.ascontiguousarray(body_vertex_range, np.uint32)
        nb = 0 if self.bvr is None else self.bvr.shape[0]
        self.nrm = None if normals is None else np.ascontiguousarray(normals, np.float32)
        d = RcSceneDesc(_ptr(self.pos), self.pos.shape[0], _ptr(self.idx), self.idx.shape[0], _ptr(self.tm),
                        _ptr(self.mats), self.mats.shape[0], None if nb == 0 else _ptr(self.bvr), nb,
                        None if self.nrm is None else _ptr(self.nrm))
        ctx._sync_stream()
        h = C.c_void_p()
        check(lib().rc_scene_create(ctx.h, C.byref(d), C.byref(h)), "rc_scene_create")
        self.h = h
        self.n_tris = self.idx.shape[0]

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            lib().rc_scene_destroy(self.ctx.h, self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build(self, bins: int = 32, max_leaf: int = 4, node_cost: float = 4.0, device: bool = False,
              two_level: bool = False, watertight: bool = False, device_sah: bool = False):
        """Host binned-SAH build; device=True: the GPU LBVH build (RC_BUILD_DEVICE_LBVH); device_sah=True: the
        binned SAH built on the GPU (RC_BUILD_DEVICE_SAH); two_level=True: one GPU-built tree per body under a top
        level over the bodies (RC_BUILD_TWO_LEVEL); watertight=True: the scene's ray/triangle tests use the
        watertight test (RC_BUILD_WATERTIGHT)."""
        self.ctx._sync_stream()
        method = 2 if two_level else (3 if device_sah else (1 if device else 0))
        opts = RcBuildOpts(bins, max_leaf, node_cost, method, 1 if watertight else 0)
        check(lib().rc_bvh_build(self.ctx.h, self.h, C.byref(opts)), "rc_bvh_build")
        return self

    def tlas_rebuild(self, stream=None):
        """Rebuild the top level of a two-level structure from the bodies' current maps, enqueued on `stream`
        (a torch.cuda.Stream; None = the context stream) without host synchronisation."""
        h = None if stream is None else C.c_void_p(stream.cuda_stream)
        if stream is None:
            self.ctx._sync_stream()
        check(lib().rc_tlas_rebuild(self.ctx.h, self.h, h), "rc_tlas_rebuild")

    def tlas_export(self) -> np.ndarray:
        """Instance records (n_bodies, 16) float32: world-to-object map [M | m] then the root index bits."""
        n = int(self.stats()["n_instances"])
        out = np.zeros((n, 16), np.float32)
        check(lib().rc_tlas_export(self.ctx.h, self.h, _ptr(out)), "rc_tlas_export")
        return out

    def refit(self):
        self.ctx._sync_stream()
        check(lib().rc_bvh_refit(self.ctx.h, self.h), "rc_bvh_refit")

    def set_transforms(self, d_xforms, d_body_ids):
        """d_xforms: (n, 12) float32 device tensor, d_body_ids: (n,) int32/uint32 device tensor."""
        assert d_xforms.is_contiguous() and d_body_ids.is_contiguous()
        self.ctx._sync_stream()
        check(lib().rc_scene_set_transforms(self.ctx.h, self.h, C.c_void_p(d_xforms.data_ptr()),
                                            C.c_void_p(d_body_ids.data_ptr()), int(d_body_ids.numel())),
              "rc_scene_set_transforms")

    def positions(self) -> np.ndarray:
        out = np.zeros_like(self.pos)
        check(lib().rc_scene_get_positions(self.ctx.h, self.h, _ptr(out)), "rc_scene_get_positions")
        return out

    def stats(self) -> dict:
        s = RcBvhStats()
        check(lib().rc_bvh_get_stats(self.ctx.h, self.h, C.byref(s)), "rc_bvh_get_stats")
        return {k: getattr(s, k) for k, _ in RcBvhStats._fields_}

    def export(self):
        st = self.stats()
        nodes = np.zeros((int(st["n_nodes"]), 32), np.uint32)
        order = np.zeros(self.n_tris, np.uint32)
        check(lib().rc_bvh_export(self.ctx.h, self.h, _ptr(nodes), _ptr(order)), "rc_bvh_export")
        return nodes, order


class Denoiser:
    """The U-Net shadow denoiser of the library (BF16 MFMA kernels, FP32 master weights, Adam)."""

    def __init__(self, ctx: Context, seed: int = 0):
        self.ctx = ctx
        self.n_params = int(lib().rc_denoiser_n_params())
        ctx._sync_stream()
        h = C.c_void_p()
        check(lib().rc_denoiser_create(ctx.h, int(seed), C.byref(h)), "rc_denoiser_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            lib().rc_denoiser_destroy(self.ctx.h, self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        check(lib().rc_denoiser_get_params(self.ctx.h, self.h, _ptr(out)), "rc_denoiser_get_params")
        return out

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, np.float32)
        assert p.size == self.n_params
        self.ctx._sync_stream()
        check(lib().rc_denoiser_set_params(self.ctx.h, self.h, _ptr(p)), "rc_denoiser_set_params")

    def grads(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        check(lib().rc_denoiser_get_grads(self.ctx.h, self.h, _ptr(out)), "rc_denoiser_get_grads")
        return out

    def infer(self, feat, out=None, fp32: bool = False):
        """feat: (N, H, W, 8) torch.bfloat16 on the GPU -> (N, H, W) float32.  fp32: evaluate the FP32 copy of
        the network (FP32 master weights and activations) instead of the BF16 one."""
        torch = self.ctx.torch
        assert feat.dtype == torch.bfloat16 and feat.is_contiguous() and feat.shape[-1] == 8
        n, h, w = (int(x) for x in feat.shape[:3])
        if out is None:
            out = torch.empty((n, h, w), dtype=torch.float32, device=feat.device)
        self.ctx._sync_stream()
        fn = lib().rc_denoiser_infer_fp32 if fp32 else lib().rc_denoiser_infer
        check(fn(self.ctx.h, self.h, C.c_void_p(feat.data_ptr()), n, h, w, C.c_void_p(out.data_ptr())),
              "rc_denoiser_infer_fp32" if fp32 else "rc_denoiser_infer")
        return out

    def train_step(self, feat, target, mask, lr: float, want_loss: bool = True):
        torch = self.ctx.torch
        assert feat.dtype == torch.bfloat16 and feat.is_contiguous()
        assert target.dtype == torch.float32 and mask.dtype == torch.float32
        n, h, w = (int(x) for x in feat.shape[:3])
        loss = C.c_float(float("nan"))
        self.ctx._sync_stream()
        check(lib().rc_denoiser_train_step(self.ctx.h, self.h, C.c_void_p(feat.data_ptr()),
                                           C.c_void_p(target.data_ptr()), C.c_void_p(mask.data_ptr()), n, h, w,
                                           float(lr), C.byref(loss) if want_loss else None),
              "rc_denoiser_train_step")
        return float(loss.value)

    def save(self, path: str):
        check(lib().rc_denoiser_save(self.ctx.h, self.h, path.encode()), "rc_denoiser_save")

    def load(self, path: str):
        self.ctx._sync_stream()
        check(lib().rc_denoiser_load(self.ctx.h, self.h, path.encode()), "rc_denoiser_load")


def pack_features(ctx: Context, scene: Scene, cam, out: dict, depth_norm: float, feat=None):
    """Denoiser features (H, W, 8) bfloat16 from a 1-spp rect-light render `out`."""
    torch = ctx.torch
    H, W = int(cam.height), int(cam.width)
    if feat is None:
        feat = torch.empty((H, W, 8), dtype=torch.bfloat16, device=out["hit"].device)
    camc = camera_struct(cam)
    ctx._sync_stream()
    check(lib().rc_pack_features(ctx.h, scene.h, C.byref(camc), C.c_void_p(out["hit"].data_ptr()),
                                 C.c_void_p(out["visibility"].data_ptr()), float(depth_norm),
                                 C.c_void_p(feat.data_ptr())), "rc_pack_features")
    return feat
