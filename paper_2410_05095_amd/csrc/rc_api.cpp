// Host runtime behind the C ABI (include/raycast.h): contexts, scenes, BVH build and refit,
// and the render pipeline  primary traversal -> shadow traversal -> shade + resolve.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "../../include/raycast.h"
#include "rc_internal.h"

struct rc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int grid = 0;                         // persistent traversal grid (blocks)
    uint32_t* d_counters = nullptr;       // [0..7] work queues, [8] error flag
    unsigned long long* d_rays = nullptr; // [0] primary, [1] shadow rays cast
    uint32_t* d_overflow = nullptr;
    size_t overflow_words = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool timed = false;
    int sticky = RC_OK;
};

struct rc_scene {
    std::vector<float> pos;
    std::vector<uint32_t> idx, tri_mat, body_vr;
    std::vector<float> mats;
    uint32_t nv = 0, nt = 0, nm = 0, nb = 0, max_body_verts = 0;
    float* d_pos = nullptr;
    float* d_rest = nullptr;
    uint32_t* d_idx = nullptr;
    uint32_t* d_tri_mat = nullptr;
    float* d_mats = nullptr;
    uint32_t* d_body_vr = nullptr;
    bool host_pos_stale = false;
    // BVH
    bool built = false;
    HostBvh hb;
    Node4* d_nodes = nullptr;
    uint32_t* d_order = nullptr;
    float4* d_tris = nullptr;
    double build_ms = 0.0;
    float scale = 1.0f;
    bool sah_stale = false;   // boxes refit on the device since the host copy was made
};

namespace {

int hip_status(hipError_t e) { return e == hipErrorOutOfMemory ? RC_ERR_OUT_OF_MEMORY : RC_ERR_HIP; }

#define RC_HIP(call)                              \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) return hip_status(e_); \
    } while (0)

template <class T>
int dev_alloc(T** p, size_t n)
{
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
    if (e != hipSuccess) { *p = nullptr; return hip_status(e); }
    return RC_OK;
}

template <class T>
void dev_free(T*& p)
{
    if (p) hipFree(p);
    p = nullptr;
}

void free_bvh(rc_scene* s)
{
    dev_free(s->d_nodes);
    dev_free(s->d_order);
    dev_free(s->d_tris);
    s->built = false;
    s->hb = HostBvh();
}

// FP32 camera frame, in the fixed operation order used by every consumer of these rays.
void f_normalize(float v[3])
{
    float n2 = v[0] * v[0] + v[1] * v[1];
    n2 = n2 + v[2] * v[2];
    float len = sqrtf(n2);
    v[0] = v[0] / len; v[1] = v[1] / len; v[2] = v[2] / len;
}

void f_cross(const float a[3], const float b[3], float o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

DevCamera make_camera(const rc_camera* c)
{
    DevCamera d;
    memset(&d, 0, sizeof(d));
    for (int k = 0; k < 3; ++k) { d.eye[k] = c->eye[k]; d.f[k] = c->target[k] - c->eye[k]; }
    f_normalize(d.f);
    f_cross(d.f, c->up, d.r);
    f_normalize(d.r);
    f_cross(d.r, d.f, d.u);
    d.tan_half = (float)tan((double)c->vfov_deg * (3.14159265358979323846 / 360.0));
    float aspect = (float)c->width / (float)c->height;
    d.x_scale = d.tan_half * aspect;
    d.width = c->width;
    d.height = c->height;
    d.ssaa = c->ssaa;
    d.seed = c->seed;
    d.frame = c->frame;
    return d;
}

bool finite3(const float* p) { return isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]); }

DevScene dev_scene(const rc_scene* s)
{
    DevScene d;
    memset(&d, 0, sizeof(d));
    d.pos = s->d_pos;
    d.idx = s->d_idx;
    d.tri_mat = s->d_tri_mat;
    d.mats = s->d_mats;
    d.nodes = s->d_nodes;
    d.tris = s->d_tris;
    d.n_tris = s->nt;
    d.n_nodes = (uint32_t)s->hb.nodes.size();
    d.max_stack = s->hb.max_stack;
    d.scale = s->scale;
    return d;
}

int ensure_overflow(rc_ctx* c, uint32_t max_stack)
{
    uint32_t depth = max_stack > RC_STACK_LDS ? max_stack - RC_STACK_LDS : 0;
    size_t words = (size_t)c->grid * RC_TRACE_BLOCK * depth * 2;
    if (words <= c->overflow_words && c->d_overflow) return RC_OK;
    dev_free(c->d_overflow);
    c->overflow_words = 0;
    int st = dev_alloc(&c->d_overflow, words);
    if (st != RC_OK) return st;
    c->overflow_words = words;
    return RC_OK;
}

}  // namespace

extern "C" {

const char* rc_status_string(int s)
{
    switch (s) {
    case RC_OK: return "ok";
    case RC_ERR_INVALID_ARG: return "invalid argument";
    case RC_ERR_INVALID_VALUE: return "invalid value in input data";
    case RC_ERR_OUT_OF_MEMORY: return "out of device memory";
    case RC_ERR_HIP: return "HIP runtime error";
    case RC_ERR_NOT_BUILT: return "acceleration structure not built";
    case RC_ERR_QUEUE_OVERFLOW: return "device queue or stack bound exceeded";
    case RC_ERR_BAD_CHECKPOINT: return "bad checkpoint";
    case RC_ERR_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

int rc_version(void) { return 10000; }

int rc_create(rc_ctx** out, int device, void* hip_stream)
{
    if (!out) return RC_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return RC_ERR_HIP;
    if (device < 0 || device >= n) return RC_ERR_INVALID_ARG;
    RC_HIP(hipSetDevice(device));
    rc_ctx* c = new (std::nothrow) rc_ctx();
    if (!c) return RC_ERR_OUT_OF_MEMORY;
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->grid = rc_trace_grid(device);
    int st = dev_alloc(&c->d_counters, 16);
    if (st == RC_OK) st = dev_alloc(&c->d_rays, 8);
    for (int i = 0; i < 4 && st == RC_OK; ++i)
        if (hipEventCreate(&c->ev[i]) != hipSuccess) st = RC_ERR_HIP;
    if (st == RC_OK && hipMemset(c->d_counters, 0, 16 * sizeof(uint32_t)) != hipSuccess) st = RC_ERR_HIP;
    if (st == RC_OK && hipMemset(c->d_rays, 0, 8 * sizeof(unsigned long long)) != hipSuccess) st = RC_ERR_HIP;
    if (st != RC_OK) { rc_destroy(c); return st; }
    *out = c;
    return RC_OK;
}

int rc_destroy(rc_ctx* c)
{
    if (!c) return RC_ERR_INVALID_ARG;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    dev_free(c->d_counters);
    dev_free(c->d_rays);
    dev_free(c->d_overflow);
    for (int i = 0; i < 4; ++i)
        if (c->ev[i]) hipEventDestroy(c->ev[i]);
    delete c;
    return RC_OK;
}

int rc_set_stream(rc_ctx* c, void* hip_stream)
{
    if (!c) return RC_ERR_INVALID_ARG;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return RC_OK;
}

int rc_get_last_error(rc_ctx* c)
{
    if (!c) return RC_ERR_INVALID_ARG;
    hipSetDevice(c->device);
    int st = c->sticky;
    c->sticky = RC_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return RC_ERR_HIP;
    uint32_t flag = 0;
    if (hipMemcpy(&flag, c->d_counters + 8, sizeof(flag), hipMemcpyDeviceToHost) != hipSuccess) return RC_ERR_HIP;
    if (flag) {
        uint32_t zero = 0;
        hipMemcpy(c->d_counters + 8, &zero, sizeof(zero), hipMemcpyHostToDevice);
        if (st == RC_OK) st = RC_ERR_QUEUE_OVERFLOW;
    }
    return st;
}

int rc_scene_create(rc_ctx* c, const rc_scene_desc* d, rc_scene** out)
{
    if (!c || !d || !out) return RC_ERR_INVALID_ARG;
    *out = nullptr;
    if (!d->positions || !d->indices || !d->tri_material || !d->materials) return RC_ERR_INVALID_ARG;
    if (d->n_vertices == 0 || d->n_tris == 0 || d->n_materials == 0) return RC_ERR_INVALID_ARG;
    if (d->n_tris >= (1u << 28)) return RC_ERR_UNSUPPORTED;
    if (d->n_bodies > 0 && !d->body_vertex_range) return RC_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < d->n_vertices; ++i)
        if (!finite3(d->positions + 3 * (size_t)i)) return RC_ERR_INVALID_VALUE;
    for (size_t i = 0; i < 3 * (size_t)d->n_tris; ++i)
        if (d->indices[i] >= d->n_vertices) return RC_ERR_INVALID_VALUE;
    for (uint32_t t = 0; t < d->n_tris; ++t)
        if (d->tri_material[t] >= d->n_materials) return RC_ERR_INVALID_VALUE;
    for (uint32_t m = 0; m < d->n_materials; ++m) {
        const float* p = d->materials + 5 * (size_t)m;
        for (int k = 0; k < 3; ++k)
            if (!(p[k] >= 0.0f && p[k] <= 1.0f)) return RC_ERR_INVALID_VALUE;
        if (!(p[3] >= 0.01f && p[3] <= 1.0f) || !(p[4] >= 0.0f && p[4] <= 1.0f)) return RC_ERR_INVALID_VALUE;
    }
    uint32_t max_body = 0;
    for (uint32_t b = 0; b < d->n_bodies; ++b) {
        uint64_t f = d->body_vertex_range[2 * (size_t)b], n = d->body_vertex_range[2 * (size_t)b + 1];
        if (f + n > d->n_vertices) return RC_ERR_INVALID_VALUE;
        max_body = std::max<uint32_t>(max_body, (uint32_t)n);
    }
    RC_HIP(hipSetDevice(c->device));
    rc_scene* s = new (std::nothrow) rc_scene();
    if (!s) return RC_ERR_OUT_OF_MEMORY;
    s->nv = d->n_vertices; s->nt = d->n_tris; s->nm = d->n_materials; s->nb = d->n_bodies;
    s->max_body_verts = max_body;
    s->pos.assign(d->positions, d->positions + 3 * (size_t)s->nv);
    s->idx.assign(d->indices, d->indices + 3 * (size_t)s->nt);
    s->tri_mat.assign(d->tri_material, d->tri_material + s->nt);
    s->mats.assign(d->materials, d->materials + 5 * (size_t)s->nm);
    if (s->nb) s->body_vr.assign(d->body_vertex_range, d->body_vertex_range + 2 * (size_t)s->nb);
    float scale = 1.0f;
    for (float x : s->pos) scale = std::max(scale, fabsf(x));
    s->scale = scale;
    int st = dev_alloc(&s->d_pos, s->pos.size());
    if (st == RC_OK) st = dev_alloc(&s->d_idx, s->idx.size());
    if (st == RC_OK) st = dev_alloc(&s->d_tri_mat, s->tri_mat.size());
    if (st == RC_OK) st = dev_alloc(&s->d_mats, s->mats.size());
    if (st == RC_OK && s->nb) st = dev_alloc(&s->d_rest, s->pos.size());
    if (st == RC_OK && s->nb) st = dev_alloc(&s->d_body_vr, s->body_vr.size());
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (st == RC_OK && hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess) st = RC_ERR_HIP;
    };
    up(s->d_pos, s->pos.data(), s->pos.size() * 4);
    up(s->d_idx, s->idx.data(), s->idx.size() * 4);
    up(s->d_tri_mat, s->tri_mat.data(), s->tri_mat.size() * 4);
    up(s->d_mats, s->mats.data(), s->mats.size() * 4);
    if (s->nb) {
        up(s->d_rest, s->pos.data(), s->pos.size() * 4);
        up(s->d_body_vr, s->body_vr.data(), s->body_vr.size() * 4);
    }
    if (st == RC_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = RC_ERR_HIP;
    if (st != RC_OK) { rc_scene_destroy(c, s); return st; }
    *out = s;
    return RC_OK;
}

int rc_scene_destroy(rc_ctx* c, rc_scene* s)
{
    if (!c || !s) return RC_ERR_INVALID_ARG;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    free_bvh(s);
    dev_free(s->d_pos);
    dev_free(s->d_rest);
    dev_free(s->d_idx);
    dev_free(s->d_tri_mat);
    dev_free(s->d_mats);
    dev_free(s->d_body_vr);
    delete s;
    return RC_OK;
}

int rc_bvh_build(rc_ctx* c, rc_scene* s, const rc_build_opts* o)
{
    if (!c || !s) return RC_ERR_INVALID_ARG;
    uint32_t bins = o && o->bins ? o->bins : 32u;
    uint32_t max_leaf = o && o->max_leaf ? o->max_leaf : 4u;
    if (bins < 2 || bins > 256 || max_leaf < 1 || max_leaf > 4) return RC_ERR_INVALID_ARG;
    RC_HIP(hipSetDevice(c->device));
    if (s->host_pos_stale) {
        RC_HIP(hipMemcpyAsync(s->pos.data(), s->d_pos, s->pos.size() * 4, hipMemcpyDeviceToHost, c->stream));
        RC_HIP(hipStreamSynchronize(c->stream));
        s->host_pos_stale = false;
    }
    free_bvh(s);
    auto t0 = std::chrono::steady_clock::now();
    HostBvh hb;
    if (!rc_build_bvh_host(s->pos.data(), s->idx.data(), s->nt, bins, max_leaf, hb)) return RC_ERR_INVALID_VALUE;
    s->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int st = dev_alloc(&s->d_nodes, hb.nodes.size());
    if (st == RC_OK) st = dev_alloc(&s->d_order, hb.tri_order.size());
    if (st == RC_OK) st = dev_alloc(&s->d_tris, 3 * (size_t)s->nt);
    if (st == RC_OK && hipMemcpyAsync(s->d_nodes, hb.nodes.data(), hb.nodes.size() * sizeof(Node4),
                                      hipMemcpyHostToDevice, c->stream) != hipSuccess) st = RC_ERR_HIP;
    if (st == RC_OK && hipMemcpyAsync(s->d_order, hb.tri_order.data(), hb.tri_order.size() * 4,
                                      hipMemcpyHostToDevice, c->stream) != hipSuccess) st = RC_ERR_HIP;
    if (st != RC_OK) { free_bvh(s); return st; }
    rc_launch_pack(s->d_pos, s->d_idx, s->d_order, s->nt, s->d_tris, c->stream);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) { free_bvh(s); return RC_ERR_HIP; }
    s->hb = std::move(hb);
    s->built = true;
    return ensure_overflow(c, s->hb.max_stack);
}

int rc_scene_set_transforms(rc_ctx* c, rc_scene* s, const float* d_xforms, const uint32_t* d_body_ids, uint32_t n)
{
    if (!c || !s) return RC_ERR_INVALID_ARG;
    if (n == 0) return RC_OK;
    if (!d_xforms || !d_body_ids || n > s->nb || s->nb == 0) return RC_ERR_INVALID_ARG;
    RC_HIP(hipSetDevice(c->device));
    rc_launch_transform(s->d_rest, s->d_pos, s->d_body_vr, d_xforms, d_body_ids, n, s->max_body_verts, c->stream);
    RC_HIP(hipGetLastError());
    s->host_pos_stale = true;
    return RC_OK;
}

int rc_bvh_refit(rc_ctx* c, rc_scene* s)
{
    if (!c || !s) return RC_ERR_INVALID_ARG;
    if (!s->built) return RC_ERR_NOT_BUILT;
    RC_HIP(hipSetDevice(c->device));
    rc_launch_pack(s->d_pos, s->d_idx, s->d_order, s->nt, s->d_tris, c->stream);
    const auto& ls = s->hb.level_start;
    for (int lv = (int)s->hb.depth - 1; lv >= 0; --lv)
        rc_launch_refit_level(s->d_nodes, s->d_pos, s->d_idx, s->d_order, ls[lv], ls[lv + 1] - ls[lv], c->stream);
    RC_HIP(hipGetLastError());
    s->sah_stale = true;
    return RC_OK;
}

int rc_scene_get_positions(rc_ctx* c, const rc_scene* s, float* out)
{
    if (!c || !s || !out) return RC_ERR_INVALID_ARG;
    RC_HIP(hipSetDevice(c->device));
    RC_HIP(hipMemcpyAsync(out, s->d_pos, (size_t)s->nv * 12, hipMemcpyDeviceToHost, c->stream));
    RC_HIP(hipStreamSynchronize(c->stream));
    return RC_OK;
}

int rc_bvh_get_stats(rc_ctx* c, const rc_scene* s_, rc_bvh_stats* o)
{
    if (!c || !s_ || !o) return RC_ERR_INVALID_ARG;
    if (!s_->built) return RC_ERR_NOT_BUILT;
    rc_scene* s = const_cast<rc_scene*>(s_);
    if (s->sah_stale) {
        RC_HIP(hipSetDevice(c->device));
        RC_HIP(hipMemcpyAsync(s->hb.nodes.data(), s->d_nodes, s->hb.nodes.size() * sizeof(Node4),
                              hipMemcpyDeviceToHost, c->stream));
        RC_HIP(hipStreamSynchronize(c->stream));
        s->hb.sah_cost = rc_bvh_sah(s->hb.nodes);
        s->sah_stale = false;
    }
    o->n_nodes = s->hb.nodes.size();
    o->n_leaves = s->hb.n_leaves;
    o->n_tris = s->nt;
    o->depth = s->hb.depth;
    o->max_stack = s->hb.max_stack;
    o->sah_cost = s->hb.sah_cost;
    o->build_ms = s->build_ms;
    return RC_OK;
}

int rc_bvh_export(rc_ctx* c, const rc_scene* s, uint32_t* nodes_out, uint32_t* order_out)
{
    if (!c || !s) return RC_ERR_INVALID_ARG;
    if (!s->built) return RC_ERR_NOT_BUILT;
    RC_HIP(hipSetDevice(c->device));
    if (nodes_out)
        RC_HIP(hipMemcpyAsync(nodes_out, s->d_nodes, s->hb.nodes.size() * sizeof(Node4), hipMemcpyDeviceToHost, c->stream));
    if (order_out)
        RC_HIP(hipMemcpyAsync(order_out, s->d_order, (size_t)s->nt * 4, hipMemcpyDeviceToHost, c->stream));
    RC_HIP(hipStreamSynchronize(c->stream));
    return RC_OK;
}

int rc_render(rc_ctx* c, rc_scene* s, const rc_camera* cam, const rc_point_light* lights, uint32_t n_lights,
              const rc_rect_light* rect, const rc_render_opts* opts, const rc_outputs* out)
{
    if (!c || !s || !cam || !out) return RC_ERR_INVALID_ARG;
    if (cam->width <= 0 || cam->height <= 0 || (int64_t)cam->width * cam->height > (1ll << 28)) return RC_ERR_INVALID_ARG;
    if (cam->ssaa != 1 && cam->ssaa != 2) return RC_ERR_UNSUPPORTED;
    if (!(cam->vfov_deg > 0.0f && cam->vfov_deg < 180.0f) || !finite3(cam->eye) || !finite3(cam->target) ||
        !finite3(cam->up))
        return RC_ERR_INVALID_VALUE;
    if (n_lights > 16 || (n_lights > 0 && !lights)) return RC_ERR_INVALID_ARG;
    if (!out->d_rgba || !out->d_hit) return RC_ERR_INVALID_ARG;
    if (n_lights > 0 && !out->d_shadow) return RC_ERR_INVALID_ARG;
    if (rect) {
        if (!out->d_visibility || !opts || opts->area_samples == 0) return RC_ERR_INVALID_ARG;
        if (cam->ssaa != 1) return RC_ERR_UNSUPPORTED;
    }
    if ((reinterpret_cast<uintptr_t>(out->d_rgba) | reinterpret_cast<uintptr_t>(out->d_hit) |
         reinterpret_cast<uintptr_t>(out->d_sample_rgba)) & 15u)
        return RC_ERR_INVALID_ARG;
    if (!s->built) return RC_ERR_NOT_BUILT;
    RC_HIP(hipSetDevice(c->device));

    DevCamera dc = make_camera(cam);
    DevScene ds = dev_scene(s);
    DevLights L;
    memset(&L, 0, sizeof(L));
    L.n_point = (int)n_lights;
    for (uint32_t l = 0; l < n_lights; ++l) {
        if (!finite3(lights[l].position) || !finite3(lights[l].intensity)) return RC_ERR_INVALID_VALUE;
        for (int k = 0; k < 3; ++k) { L.point[l][k] = lights[l].position[k]; L.point[l][3 + k] = lights[l].intensity[k]; }
    }
    if (rect) {
        L.has_rect = 1;
        memcpy(L.rect, rect, sizeof(float) * 12);
        for (int k = 0; k < 12; ++k)
            if (!isfinite(L.rect[k])) return RC_ERR_INVALID_VALUE;
        L.area_samples = (int)opts->area_samples;
        L.area_stream = opts->area_stream;
    }
    bool timing = opts && (opts->flags & RC_FLAG_TIMING);

    TraceWork w;
    w.counters = c->d_counters;
    w.overflow = c->d_overflow;
    w.overflow_depth = s->hb.max_stack > RC_STACK_LDS ? s->hb.max_stack - RC_STACK_LDS : 0;
    w.n_lanes = (uint32_t)c->grid * RC_TRACE_BLOCK;
    w.error_flag = c->d_counters + 8;
    int st = ensure_overflow(c, s->hb.max_stack);
    if (st != RC_OK) return st;
    w.overflow = c->d_overflow;

    hipStream_t q = c->stream;
    rc_launch_fill_u32(c->d_counters, 0u, 8, q);
    rc_launch_fill_u32(reinterpret_cast<uint32_t*>(c->d_rays), 0u, 16, q);
    uint4* gbuf = reinterpret_cast<uint4*>(out->d_hit);
    if (timing) RC_HIP(hipEventRecord(c->ev[0], q));
    w.ray_count = c->d_rays + 0;
    rc_launch_primary(ds, dc, gbuf, w, c->grid, q);
    if (timing) RC_HIP(hipEventRecord(c->ev[1], q));
    if (n_lights > 0 || rect) {
        w.ray_count = c->d_rays + 1;
        rc_launch_shadow(ds, dc, L, gbuf, out->d_shadow, out->d_visibility, w, c->grid, q);
    }
    if (timing) RC_HIP(hipEventRecord(c->ev[2], q));
    rc_launch_shade(ds, dc, L, gbuf, n_lights ? out->d_shadow : nullptr, out->d_visibility, out->d_rgba,
                    out->d_sample_rgba, q);
    if (timing) RC_HIP(hipEventRecord(c->ev[3], q));
    c->timed = timing;
    RC_HIP(hipGetLastError());
    return RC_OK;
}

int rc_camera_rays(rc_ctx* c, const rc_camera* cam, float* d_o, float* d_d)
{
    if (!c || !cam || !d_o || !d_d) return RC_ERR_INVALID_ARG;
    if (cam->width <= 0 || cam->height <= 0 || (int64_t)cam->width * cam->height > (1ll << 28)) return RC_ERR_INVALID_ARG;
    if (cam->ssaa != 1 && cam->ssaa != 2) return RC_ERR_UNSUPPORTED;
    RC_HIP(hipSetDevice(c->device));
    DevCamera dc = make_camera(cam);
    rc_launch_camera_rays(dc, d_o, d_d, (uint32_t)(cam->width * cam->height * cam->ssaa * cam->ssaa), c->stream);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

int rc_get_stage_times(rc_ctx* c, rc_stage_times* o)
{
    if (!c || !o) return RC_ERR_INVALID_ARG;
    memset(o, 0, sizeof(*o));
    RC_HIP(hipSetDevice(c->device));
    RC_HIP(hipStreamSynchronize(c->stream));
    if (c->timed) {
        RC_HIP(hipEventElapsedTime(&o->ms[0], c->ev[0], c->ev[1]));
        RC_HIP(hipEventElapsedTime(&o->ms[1], c->ev[1], c->ev[2]));
        RC_HIP(hipEventElapsedTime(&o->ms[2], c->ev[2], c->ev[3]));
        RC_HIP(hipEventElapsedTime(&o->ms[3], c->ev[0], c->ev[3]));
    }
    unsigned long long r[6] = {0, 0, 0, 0, 0, 0};
    RC_HIP(hipMemcpy(r, c->d_rays, sizeof(r), hipMemcpyDeviceToHost));
    for (int k = 0; k < 2; ++k) {
        o->rays[k] = r[k];
        o->node_visits[k] = r[2 + k];
        o->tri_tests[k] = r[4 + k];
    }
    return RC_OK;
}

}  // extern "C"
