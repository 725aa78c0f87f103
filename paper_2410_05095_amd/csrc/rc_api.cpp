// Host runtime behind the C ABI (include/raycast.h): contexts, scenes, BVH build and refit,
// and the render pipeline  primary traversal -> shadow traversal -> shade + resolve.
#include <math.h>
#include <string.h>

#include <stdio.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <string>
#include <vector>

#include "../../include/raycast.h"
#include "rc_internal.h"
#include "rc_objects.h"

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
    dev_free(s->d_inst);
    dev_free(s->d_tri_node);
    dev_free(s->d_dirty);
    rc_tlas_free(s->tlas);
    s->two_level = false;
    s->refit_nodes = 0;
    s->blas_nodes = s->blas_depth = 0;
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
    // allocated node count (a two-level scene's array has room for its largest top level)
    d.n_nodes = s->two_level ? s->blas_nodes + s->tlas.cap : (uint32_t)s->hb.nodes.size();
    d.max_stack = s->hb.max_stack;
    d.scale = s->scale;
    d.inst = s->two_level ? s->d_inst : nullptr;
    d.tlas_root = s->blas_nodes;
    d.watertight = s->watertight ? 1u : 0u;
    d.nrm = s->d_nrm;
    return d;
}

int ensure_overflow(rc_ctx* c, uint32_t max_stack)
{
    uint32_t depth = max_stack > RC_STACK_LDS ? max_stack - RC_STACK_LDS : 0;
    size_t words = (size_t)c->grid * RC_TRACE_BLOCK * depth * 2;
    if (words <= c->overflow_words && c->d_overflow) return RC_OK;
    RC_HIP(hipStreamSynchronize(c->stream));
    dev_free(c->d_overflow);
    c->overflow_words = 0;
    c->graph_key = 0;   // a captured batch graph points at the old buffer
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
    int st = dev_alloc(&c->d_counters, RC_COUNTER_WORDS);
    if (st == RC_OK) st = dev_alloc(&c->d_rays, 8);
    for (int i = 0; i < 4 && st == RC_OK; ++i)
        if (hipEventCreate(&c->ev[i]) != hipSuccess) st = RC_ERR_HIP;
    if (st == RC_OK && hipMemset(c->d_counters, 0, RC_COUNTER_WORDS * sizeof(uint32_t)) != hipSuccess) st = RC_ERR_HIP;
    if (st == RC_OK && hipMemset(c->d_rays, 0, 8 * sizeof(unsigned long long)) != hipSuccess) st = RC_ERR_HIP;
    if (st != RC_OK) { rc_destroy(c); return st; }
    // the fixed scratch of rc_postprocess_noalloc on this device; should its address be unavailable, that entry
    // point reports RC_ERR_HIP and everything else works
    if (rc_post_scratch_init(device) != hipSuccess) (void)hipGetLastError();
    *out = c;
    return RC_OK;
}

int rc_destroy(rc_ctx* c)
{
    if (!c) return RC_ERR_INVALID_ARG;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
    if (c->graph) hipGraphDestroy(c->graph);
    if (c->capture_stream) hipStreamDestroy(c->capture_stream);
    if (c->ev_staging) hipEventDestroy(c->ev_staging);
    if (c->h_table) hipHostFree(c->h_table);
    dev_free(c->d_table);
    dev_free(c->d_counters);
    dev_free(c->d_rays);
    dev_free(c->d_overflow);
    dev_free(c->d_post);
    dev_free(c->d_counts);
    dev_free(c->d_bsetup);
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
    uint32_t flag[2] = {0, 0};   // [0] a queue or stack bound was exceeded, [1] a kernel met an invalid input value
    if (hipMemcpy(flag, c->d_counters + 8, sizeof(flag), hipMemcpyDeviceToHost) != hipSuccess) return RC_ERR_HIP;
    if (flag[0] | flag[1]) {
        const uint32_t zero[2] = {0, 0};
        hipMemcpy(c->d_counters + 8, zero, sizeof(zero), hipMemcpyHostToDevice);
        if (st == RC_OK) st = flag[0] ? RC_ERR_QUEUE_OVERFLOW : RC_ERR_INVALID_VALUE;
    }
    return st;
}

// Per body, the triangles with a vertex in the body's vertex range (CSR), for the dirty-node refit.  Left
// empty (full refits) when vertex ranges overlap, so that every moved vertex maps to one body.
static int upload_body_tris(rc_ctx* c, rc_scene* s)
{
    const uint32_t NONE = 0xFFFFFFFFu;
    std::vector<uint32_t> vb(s->nv, NONE);
    for (uint32_t b = 0; b < s->nb; ++b) {
        const uint32_t f = s->body_vr[2 * (size_t)b], n = s->body_vr[2 * (size_t)b + 1];
        for (uint32_t v = f; v < f + n; ++v) {
            if (vb[v] != NONE) return RC_OK;
            vb[v] = b;
        }
    }
    std::vector<uint32_t> off(s->nb + 1, 0);
    auto bodies_of = [&](uint32_t t, uint32_t out[3]) {
        int k = 0;
        for (int j = 0; j < 3; ++j) {
            const uint32_t b = vb[s->idx[3 * (size_t)t + j]];
            bool seen = b == NONE;
            for (int q = 0; q < k; ++q) seen = seen || out[q] == b;
            if (!seen) out[k++] = b;
        }
        return k;
    };
    uint32_t bs[3];
    for (uint32_t t = 0; t < s->nt; ++t)
        for (int q = 0, k = bodies_of(t, bs); q < k; ++q) ++off[bs[q] + 1];
    for (uint32_t b = 0; b < s->nb; ++b) s->max_body_tris = std::max(s->max_body_tris, off[b + 1]);
    for (uint32_t b = 0; b < s->nb; ++b) off[b + 1] += off[b];
    std::vector<uint32_t> tris(off[s->nb]), fill(off.begin(), off.end() - 1);
    for (uint32_t t = 0; t < s->nt; ++t)
        for (int q = 0, k = bodies_of(t, bs); q < k; ++q) tris[fill[bs[q]]++] = t;
    int st = dev_alloc(&s->d_body_tri_off, off.size());
    if (st == RC_OK) st = dev_alloc(&s->d_body_tris, tris.size());
    if (st == RC_OK && (hipMemcpy(s->d_body_tri_off, off.data(), off.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
                        (!tris.empty() && hipMemcpy(s->d_body_tris, tris.data(), tris.size() * 4,
                                                    hipMemcpyHostToDevice) != hipSuccess)))
        st = RC_ERR_HIP;
    if (st != RC_OK) {
        dev_free(s->d_body_tri_off);
        dev_free(s->d_body_tris);
    }
    return st;
}

// After a flat build of a scene with bodies: the node of each triangle's leaf, and clear dirty flags.
static int prepare_dirty_refit(rc_ctx* c, rc_scene* s, uint32_t n_nodes)
{
    if (!s->d_body_tri_off) return RC_OK;
    int st = dev_alloc(&s->d_tri_node, s->nt);
    const size_t words = n_nodes;   // one mark per node
    if (st == RC_OK) st = dev_alloc(&s->d_dirty, words);
    if (st != RC_OK) return st;
    s->refit_nodes = n_nodes;
    rc_launch_fill_u32(s->d_tri_node, 0xFFFFFFFFu, s->nt, c->stream);
    rc_launch_tri_nodes(s->d_nodes, n_nodes, s->d_order, s->d_tri_node, c->stream);
    rc_launch_fill_u32(s->d_dirty, 0u, (uint32_t)words, c->stream);
    return hipGetLastError() == hipSuccess ? RC_OK : RC_ERR_HIP;
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
    if (d->normals)
        for (uint32_t i = 0; i < d->n_vertices; ++i) {
            const float* q = d->normals + 3 * (size_t)i;
            if (!finite3(q) || (q[0] == 0.0f && q[1] == 0.0f && q[2] == 0.0f)) return RC_ERR_INVALID_VALUE;
        }
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
    if (d->normals) s->nrm.assign(d->normals, d->normals + 3 * (size_t)s->nv);
    float scale = 1.0f;
    for (float x : s->pos) scale = std::max(scale, fabsf(x));
    s->scale = scale;
    int st = dev_alloc(&s->d_pos, s->pos.size());
    if (st == RC_OK) st = dev_alloc(&s->d_idx, s->idx.size());
    if (st == RC_OK) st = dev_alloc(&s->d_tri_mat, s->tri_mat.size());
    if (st == RC_OK) st = dev_alloc(&s->d_mats, s->mats.size());
    if (st == RC_OK && s->nb) st = dev_alloc(&s->d_rest, s->pos.size());
    if (st == RC_OK && s->nb) st = dev_alloc(&s->d_body_vr, s->body_vr.size());
    if (st == RC_OK && s->nb) st = dev_alloc(&s->d_o2w, 12 * (size_t)s->nb);
    if (st == RC_OK && !s->nrm.empty()) st = dev_alloc(&s->d_nrm, s->nrm.size());
    if (st == RC_OK && !s->nrm.empty() && s->nb) st = dev_alloc(&s->d_nrm_rest, s->nrm.size());
    std::vector<float> ident;
    if (s->nb) {
        ident.assign(12 * (size_t)s->nb, 0.0f);
        for (uint32_t b = 0; b < s->nb; ++b) ident[12 * (size_t)b] = ident[12 * (size_t)b + 5] = ident[12 * (size_t)b + 10] = 1.0f;
    }
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
        up(s->d_o2w, ident.data(), ident.size() * 4);
    }
    if (!s->nrm.empty()) {
        up(s->d_nrm, s->nrm.data(), s->nrm.size() * 4);
        if (s->nb) up(s->d_nrm_rest, s->nrm.data(), s->nrm.size() * 4);
    }
    if (st == RC_OK && s->nb) st = upload_body_tris(c, s);
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
    dev_free(s->d_o2w);
    dev_free(s->d_nrm);
    dev_free(s->d_nrm_rest);
    dev_free(s->d_body_tri_off);
    dev_free(s->d_body_tris);
    delete s;
    return RC_OK;
}

// Device build (k_build.hip): the tree and leaf order stay on the GPU; the nodes are read back once for the
// host-side statistics (leaf count, SAH cost), after the build time is taken.
static int build_device(rc_ctx* c, rc_scene* s, uint32_t max_leaf, bool sah = false, uint32_t bins = 32,
                        float node_cost = 4.0f)
{
    free_bvh(s);
    RC_HIP(hipStreamSynchronize(c->stream));
    auto t0 = std::chrono::steady_clock::now();
    HostBvh hb;
    int st = dev_alloc(&s->d_order, s->nt);
    if (st == RC_OK) st = dev_alloc(&s->d_tris, 3 * (size_t)s->nt);
    if (st != RC_OK) { free_bvh(s); return st; }
    Node4* d_nodes = nullptr;
    uint32_t n_nodes = 0;
    hipError_t e = sah ? rc_build_bvh_device_sah(s->d_pos, s->d_idx, s->nt, bins, max_leaf, node_cost, &d_nodes,
                                                 &n_nodes, s->d_order, hb.level_start, c->stream)
                       : rc_build_bvh_device(s->d_pos, s->d_idx, s->nt, max_leaf, nullptr, {}, {}, &d_nodes, &n_nodes,
                                             s->d_order, hb.level_start, c->stream);
    if (e != hipSuccess) { free_bvh(s); return hip_status(e); }
    s->d_nodes = d_nodes;
    rc_launch_pack(s->d_pos, s->d_idx, s->d_order, s->nt, s->d_tris, s->watertight, c->stream);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) { free_bvh(s); return RC_ERR_HIP; }
    s->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st = prepare_dirty_refit(c, s, n_nodes);
    if (st != RC_OK) { free_bvh(s); return st; }
    hb.nodes.resize(n_nodes);
    if (hipMemcpy(hb.nodes.data(), d_nodes, (size_t)n_nodes * sizeof(Node4), hipMemcpyDeviceToHost) != hipSuccess) {
        free_bvh(s);
        return RC_ERR_HIP;
    }
    hb.depth = (uint32_t)hb.level_start.size() - 1;
    hb.max_stack = 3 * hb.depth + 1;
    for (const Node4& nd : hb.nodes)
        for (int k = 0; k < 4; ++k) hb.n_leaves += rc_is_leaf(nd.child[k]) ? 1u : 0u;
    hb.sah_cost = rc_bvh_sah(hb.nodes);
    s->hb = std::move(hb);
    s->built = true;
    s->sah_stale = false;
    return ensure_overflow(c, s->hb.max_stack);
}

// Two-level build (k_build.hip): the bottom-level trees of all bodies in one pass over their rest positions,
// then the top level over the bodies' current maps.  Every triangle must belong to one body (all three
// vertices in its vertex range), and the bodies must own consecutive triangle ranges in body order.
static int build_two_level(rc_ctx* c, rc_scene* s, uint32_t max_leaf)
{
    if (s->nb == 0) return RC_ERR_INVALID_ARG;
    const uint32_t NONE = 0xFFFFFFFFu;
    std::vector<uint32_t> vb(s->nv, NONE);
    for (uint32_t b = 0; b < s->nb; ++b)
        for (uint32_t v = s->body_vr[2 * (size_t)b]; v < s->body_vr[2 * (size_t)b] + s->body_vr[2 * (size_t)b + 1]; ++v) {
            if (vb[v] != NONE) return RC_ERR_INVALID_VALUE;   // overlapping bodies
            vb[v] = b;
        }
    std::vector<uint32_t> seg(s->nt), first(s->nb, 0), count(s->nb, 0);
    for (uint32_t t = 0; t < s->nt; ++t) {
        const uint32_t b = vb[s->idx[3 * (size_t)t]];
        if (b == NONE || vb[s->idx[3 * (size_t)t + 1]] != b || vb[s->idx[3 * (size_t)t + 2]] != b) return RC_ERR_INVALID_VALUE;
        if (t > 0 && b < seg[t - 1]) return RC_ERR_INVALID_VALUE;   // triangle ranges out of body order
        seg[t] = b;
        ++count[b];
    }
    for (uint32_t b = 0, f = 0; b < s->nb; ++b) {
        if (count[b] == 0) return RC_ERR_INVALID_VALUE;
        first[b] = f;
        f += count[b];
    }
    free_bvh(s);
    RC_HIP(hipStreamSynchronize(c->stream));
    auto t0 = std::chrono::steady_clock::now();
    uint32_t* d_seg = nullptr;
    int st = dev_alloc(&d_seg, s->nt);
    if (st == RC_OK) st = dev_alloc(&s->d_order, s->nt);
    if (st == RC_OK) st = dev_alloc(&s->d_tris, 3 * (size_t)s->nt);
    if (st == RC_OK) st = dev_alloc(&s->d_inst, s->nb);
    if (st == RC_OK && hipMemcpyAsync(d_seg, seg.data(), seg.size() * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess)
        st = RC_ERR_HIP;
    HostBvh hb;
    Node4* d_blas = nullptr;
    uint32_t n_blas = 0;
    if (st == RC_OK) {
        hipError_t e = rc_build_bvh_device(s->d_rest, s->d_idx, s->nt, max_leaf, d_seg, first, count, &d_blas, &n_blas,
                                           s->d_order, hb.level_start, c->stream);
        if (e != hipSuccess) st = hip_status(e);
    }
    dev_free(d_seg);
    if (st == RC_OK && rc_tlas_alloc(s->tlas, s->nb) != hipSuccess) st = RC_ERR_OUT_OF_MEMORY;
    if (st == RC_OK) st = dev_alloc(&s->d_nodes, (size_t)n_blas + s->tlas.cap);
    if (st == RC_OK && hipMemcpyAsync(s->d_nodes, d_blas, (size_t)n_blas * sizeof(Node4), hipMemcpyDeviceToDevice,
                                      c->stream) != hipSuccess)
        st = RC_ERR_HIP;
    if (st == RC_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = RC_ERR_HIP;
    dev_free(d_blas);
    if (st != RC_OK) { free_bvh(s); return st; }
    s->blas_nodes = n_blas;
    s->blas_depth = (uint32_t)hb.level_start.size() - 1;
    rc_launch_pack(s->d_rest, s->d_idx, s->d_order, s->nt, s->d_tris, s->watertight, c->stream);
    if (hipGetLastError() != hipSuccess ||
        rc_tlas_build(s->tlas, s->d_o2w, s->d_nodes, n_blas, s->d_inst, RC_TLAS_MAX_LEVELS, c->d_counters + 8,
                      c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        free_bvh(s);
        return RC_ERR_HIP;
    }
    s->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    uint32_t info[3] = {0, 0, 0};
    if (hipMemcpy(info, s->tlas.info, sizeof(info), hipMemcpyDeviceToHost) != hipSuccess) { free_bvh(s); return RC_ERR_HIP; }
    if (info[2]) { free_bvh(s); return RC_ERR_QUEUE_OVERFLOW; }
    hb.nodes.resize((size_t)n_blas + info[0]);
    if (hipMemcpy(hb.nodes.data(), s->d_nodes, hb.nodes.size() * sizeof(Node4), hipMemcpyDeviceToHost) != hipSuccess) {
        free_bvh(s);
        return RC_ERR_HIP;
    }
    for (const Node4& nd : hb.nodes)
        for (int k = 0; k < 4; ++k) hb.n_leaves += rc_is_leaf(nd.child[k]) ? 1u : 0u;
    hb.depth = s->blas_depth + info[1];
    // a path crosses at most the top level's bound of levels and one bottom-level tree, plus the end marker
    hb.max_stack = 3 * (s->blas_depth + RC_TLAS_MAX_LEVELS) + 2;
    hb.sah_cost = 0.0;
    s->hb = std::move(hb);
    s->two_level = true;
    s->built = true;
    s->sah_stale = false;
    return ensure_overflow(c, s->hb.max_stack);
}

int rc_tlas_rebuild(rc_ctx* c, rc_scene* s, void* stream)
{
    if (!c || !s) return RC_ERR_INVALID_ARG;
    if (!s->built) return RC_ERR_NOT_BUILT;
    if (!s->two_level) return RC_ERR_UNSUPPORTED;
    RC_HIP(hipSetDevice(c->device));
    hipStream_t st = stream ? reinterpret_cast<hipStream_t>(stream) : c->stream;
    RC_HIP(rc_tlas_build(s->tlas, s->d_o2w, s->d_nodes, s->blas_nodes, s->d_inst, RC_TLAS_MAX_LEVELS,
                         c->d_counters + 8, st));
    return RC_OK;
}

int rc_bvh_build(rc_ctx* c, rc_scene* s, const rc_build_opts* o)
{
    if (!c || !s) return RC_ERR_INVALID_ARG;
    uint32_t bins = o && o->bins ? o->bins : 32u;
    uint32_t max_leaf = o && o->max_leaf ? o->max_leaf : 4u;
    float node_cost = o && o->node_cost != 0.0f ? o->node_cost : 4.0f;
    const uint32_t method = o ? o->method : RC_BUILD_HOST_SAH;
    if (bins < 2 || bins > 256 || max_leaf < 1 || max_leaf > 4 || !(node_cost > 0.0f && node_cost <= 64.0f) ||
        method > RC_BUILD_DEVICE_SAH || (o && (o->flags & ~(uint32_t)RC_BUILD_WATERTIGHT)))
        return RC_ERR_INVALID_ARG;
    RC_HIP(hipSetDevice(c->device));
    s->watertight = o && (o->flags & RC_BUILD_WATERTIGHT);
    if (method == RC_BUILD_DEVICE_LBVH) return build_device(c, s, max_leaf);
    if (method == RC_BUILD_DEVICE_SAH) {
        if (bins > 64) return RC_ERR_UNSUPPORTED;
        return build_device(c, s, max_leaf, true, bins, node_cost);
    }
    if (method == RC_BUILD_TWO_LEVEL) return build_two_level(c, s, max_leaf);
    if (s->host_pos_stale) {
        RC_HIP(hipMemcpyAsync(s->pos.data(), s->d_pos, s->pos.size() * 4, hipMemcpyDeviceToHost, c->stream));
        RC_HIP(hipStreamSynchronize(c->stream));
        s->host_pos_stale = false;
    }
    free_bvh(s);
    auto t0 = std::chrono::steady_clock::now();
    HostBvh hb;
    if (!rc_build_bvh_host(s->pos.data(), s->idx.data(), s->nt, bins, max_leaf, node_cost, hb))
        return RC_ERR_INVALID_VALUE;
    s->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int st = dev_alloc(&s->d_nodes, hb.nodes.size());
    if (st == RC_OK) st = dev_alloc(&s->d_order, hb.tri_order.size());
    if (st == RC_OK) st = dev_alloc(&s->d_tris, 3 * (size_t)s->nt);
    if (st == RC_OK && hipMemcpyAsync(s->d_nodes, hb.nodes.data(), hb.nodes.size() * sizeof(Node4),
                                      hipMemcpyHostToDevice, c->stream) != hipSuccess) st = RC_ERR_HIP;
    if (st == RC_OK && hipMemcpyAsync(s->d_order, hb.tri_order.data(), hb.tri_order.size() * 4,
                                      hipMemcpyHostToDevice, c->stream) != hipSuccess) st = RC_ERR_HIP;
    if (st != RC_OK) { free_bvh(s); return st; }
    rc_launch_pack(s->d_pos, s->d_idx, s->d_order, s->nt, s->d_tris, s->watertight, c->stream);
    st = prepare_dirty_refit(c, s, (uint32_t)hb.nodes.size());
    if (st != RC_OK) { free_bvh(s); return st; }
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
    rc_launch_transform(s->d_rest, s->d_pos, s->d_nrm_rest, s->d_nrm, s->d_body_vr, d_xforms, d_body_ids, n,
                        s->max_body_verts, s->nb, c->d_counters + 9, c->stream);
    rc_launch_record_o2w(d_xforms, d_body_ids, n, s->nb, s->d_o2w, c->stream);
    if (s->built && !s->two_level && s->d_dirty)
        rc_launch_mark_dirty(d_body_ids, n, s->nb, s->max_body_tris, s->d_body_tri_off, s->d_body_tris, s->d_tri_node,
                             s->d_dirty, s->refit_nodes, c->stream);
    RC_HIP(hipGetLastError());
    s->host_pos_stale = true;
    return RC_OK;
}

int rc_bvh_refit(rc_ctx* c, rc_scene* s)
{
    if (!c || !s) return RC_ERR_INVALID_ARG;
    if (!s->built) return RC_ERR_NOT_BUILT;
    RC_HIP(hipSetDevice(c->device));
    if (s->two_level) return rc_tlas_rebuild(c, s, nullptr);
    const auto& ls = s->hb.level_start;
    if (s->d_dirty) {
        // only the nodes holding moved triangles and their ancestors
        rc_launch_refit_dirty(s->d_nodes, s->d_pos, s->d_idx, s->d_order, s->d_tris, s->watertight, s->d_dirty, ls,
                              c->stream);
    } else {
        rc_launch_pack(s->d_pos, s->d_idx, s->d_order, s->nt, s->d_tris, s->watertight, c->stream);
        for (int lv = (int)s->hb.depth - 1; lv >= 0; --lv)
            rc_launch_refit_level(s->d_nodes, s->d_pos, s->d_idx, s->d_order, ls[lv], ls[lv + 1] - ls[lv], c->stream);
    }
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
    o->n_instances = s->two_level ? s->nb : 0u;
    o->tlas_levels = 0;
    o->tlas_root = s->two_level ? s->blas_nodes : 0u;
    o->reserved = 0;
    if (s->two_level) {
        uint32_t info[3] = {0, 0, 0};
        RC_HIP(hipSetDevice(c->device));
        RC_HIP(hipStreamSynchronize(c->stream));
        RC_HIP(hipMemcpy(info, s->tlas.info, sizeof(info), hipMemcpyDeviceToHost));
        o->n_nodes = (uint64_t)s->blas_nodes + info[0];
        o->n_leaves = s->hb.n_leaves;
        o->n_tris = s->nt;
        o->depth = s->blas_depth + info[1];
        o->max_stack = s->hb.max_stack;
        o->sah_cost = 0.0;
        o->build_ms = s->build_ms;
        o->tlas_levels = info[1];
        return RC_OK;
    }
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

int rc_tlas_export(rc_ctx* c, const rc_scene* s, float* inst_out)
{
    if (!c || !s || !inst_out) return RC_ERR_INVALID_ARG;
    if (!s->built) return RC_ERR_NOT_BUILT;
    if (!s->two_level) return RC_ERR_UNSUPPORTED;
    RC_HIP(hipSetDevice(c->device));
    RC_HIP(hipMemcpyAsync(inst_out, s->d_inst, (size_t)s->nb * sizeof(DevInst), hipMemcpyDeviceToHost, c->stream));
    RC_HIP(hipStreamSynchronize(c->stream));
    return RC_OK;
}

int rc_bvh_export(rc_ctx* c, const rc_scene* s, uint32_t* nodes_out, uint32_t* order_out)
{
    if (!c || !s) return RC_ERR_INVALID_ARG;
    if (!s->built) return RC_ERR_NOT_BUILT;
    RC_HIP(hipSetDevice(c->device));
    size_t n_nodes = s->hb.nodes.size();
    if (s->two_level) {
        uint32_t info[3] = {0, 0, 0};
        RC_HIP(hipStreamSynchronize(c->stream));
        RC_HIP(hipMemcpy(info, s->tlas.info, sizeof(info), hipMemcpyDeviceToHost));
        n_nodes = (size_t)s->blas_nodes + info[0];
    }
    if (nodes_out)
        RC_HIP(hipMemcpyAsync(nodes_out, s->d_nodes, n_nodes * sizeof(Node4), hipMemcpyDeviceToHost, c->stream));
    if (order_out)
        RC_HIP(hipMemcpyAsync(order_out, s->d_order, (size_t)s->nt * 4, hipMemcpyDeviceToHost, c->stream));
    RC_HIP(hipStreamSynchronize(c->stream));
    return RC_OK;
}

namespace {

// Camera checks shared by the entry points that take a camera: size, sample grid, finite pose, field of view.
int check_camera(const rc_camera* cam)
{
    if (cam->width <= 0 || cam->height <= 0 || (int64_t)cam->width * cam->height > (1ll << 28)) return RC_ERR_INVALID_ARG;
    if (cam->ssaa != 1 && cam->ssaa != 2) return RC_ERR_UNSUPPORTED;
    if (!(cam->vfov_deg > 0.0f && cam->vfov_deg < 180.0f) || !finite3(cam->eye) || !finite3(cam->target) ||
        !finite3(cam->up))
        return RC_ERR_INVALID_VALUE;
    return RC_OK;
}

// Light table of a render or shade call: finite positions, intensities and rect-light geometry.
int fill_lights(DevLights& L, const rc_point_light* lights, uint32_t n_lights, const rc_rect_light* rect)
{
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
    }
    return RC_OK;
}

}  // namespace

int rc_render(rc_ctx* c, rc_scene* s, const rc_camera* cam, const rc_point_light* lights, uint32_t n_lights,
              const rc_rect_light* rect, const rc_render_opts* opts, const rc_outputs* out)
{
    if (!c || !s || !cam || !out) return RC_ERR_INVALID_ARG;
    int st = check_camera(cam);
    if (st != RC_OK) return st;
    if (n_lights > 16 || (n_lights > 0 && !lights)) return RC_ERR_INVALID_ARG;
    if (!out->d_rgba || !out->d_hit) return RC_ERR_INVALID_ARG;
    if (n_lights > 0 && !out->d_shadow) return RC_ERR_INVALID_ARG;
    if (rect) {
        if (!out->d_visibility || !opts || opts->area_samples == 0 || opts->area_samples > 4096) return RC_ERR_INVALID_ARG;
        if (cam->ssaa != 1) return RC_ERR_UNSUPPORTED;
    }
    if ((reinterpret_cast<uintptr_t>(out->d_rgba) | reinterpret_cast<uintptr_t>(out->d_hit) |
         reinterpret_cast<uintptr_t>(out->d_sample_rgba)) & 15u)
        return RC_ERR_INVALID_ARG;
    if (opts && (opts->flags & RC_FLAG_PER_LANE) && (opts->flags & RC_FLAG_WAVE)) return RC_ERR_INVALID_ARG;
    if (!s->built) return RC_ERR_NOT_BUILT;
    RC_HIP(hipSetDevice(c->device));

    DevCamera dc = make_camera(cam);
    DevScene ds = dev_scene(s);
    DevLights L;
    st = fill_lights(L, lights, n_lights, rect);
    if (st != RC_OK) return st;
    if (rect) {
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
    st = ensure_overflow(c, s->hb.max_stack);
    if (st != RC_OK) return st;
    w.overflow = c->d_overflow;

    hipStream_t q = c->stream;
    rc_launch_fill_u32(c->d_counters, 0u, 8, q);
    rc_launch_fill_u32(c->d_counters + RC_QUEUE_BASE, 0u, RC_COUNTER_WORDS - RC_QUEUE_BASE, q);
    // ray, node and triangle counts are gathered on request only (RC_FLAG_COUNT: the wave kernels are compiled
    // without their counters otherwise)
    const bool counting = opts && (opts->flags & RC_FLAG_COUNT);
    if (counting) rc_launch_fill_u32(reinterpret_cast<uint32_t*>(c->d_rays), 0u, 16, q);
    uint4* gbuf = reinterpret_cast<uint4*>(out->d_hit);
    if (timing) RC_HIP(hipEventRecord(c->ev[0], q));
    w.ray_count = counting ? c->d_rays + 0 : nullptr;
    rc_launch_primary(ds, dc, gbuf, w, c->grid, opts && (opts->flags & RC_FLAG_PER_LANE), q);
    if (timing) RC_HIP(hipEventRecord(c->ev[1], q));
    if (n_lights > 0 || rect) {
        const size_t n_pix = (size_t)cam->width * cam->height, n_samples = n_pix * cam->ssaa * cam->ssaa;
        // per pixel one visible-sample counter of the rect light, then (16-byte aligned) per sample two float4
        // of shadow-ray setup (origin, normal) for the wave-uniform shadow kernels
        const size_t setup_off = (n_pix + 3) & ~(size_t)3, words = setup_off + 8 * n_samples;
        if (words > c->counts_cap) {
            RC_HIP(hipStreamSynchronize(q));
            dev_free(c->d_counts);
            c->counts_cap = 0;
            st = dev_alloc(&c->d_counts, words);
            if (st != RC_OK) return st;
            c->counts_cap = words;
        }
        w.ray_count = counting ? c->d_rays + 1 : nullptr;
        const RcKernels kern = !opts ? RC_KERNELS_AUTO
                               : (opts->flags & RC_FLAG_PER_LANE) ? RC_KERNELS_LANE
                               : (opts->flags & RC_FLAG_WAVE)     ? RC_KERNELS_WAVE
                                                                  : RC_KERNELS_AUTO;
        float4* setup = reinterpret_cast<float4*>(c->d_counts + setup_off);
        rc_launch_shadow(ds, dc, L, gbuf, out->d_shadow, out->d_visibility, c->d_counts, setup, w, c->grid, kern, q);
    }
    if (timing) RC_HIP(hipEventRecord(c->ev[2], q));
    if (!(opts && (opts->flags & RC_FLAG_NO_SHADE)))
        rc_launch_shade(ds, dc, L, gbuf, n_lights ? out->d_shadow : nullptr, out->d_visibility, out->d_rgba,
                        out->d_sample_rgba, c->d_counters + 9, q);
    if (timing) RC_HIP(hipEventRecord(c->ev[3], q));
    c->timed = timing;
    c->timed_batch = false;
    RC_HIP(hipGetLastError());
    return RC_OK;
}

int rc_shade(rc_ctx* c, rc_scene* s, const rc_camera* cam, const rc_point_light* lights, uint32_t n_lights,
             const rc_rect_light* rect, const uint32_t* d_hit, const uint32_t* d_shadow, const float* d_vis,
             float* d_rgba, float* d_sample_rgba)
{
    if (!c || !s || !cam || !d_hit || !d_rgba) return RC_ERR_INVALID_ARG;
    int st = check_camera(cam);
    if (st != RC_OK) return st;
    if (n_lights > 16 || (n_lights > 0 && (!lights || !d_shadow))) return RC_ERR_INVALID_ARG;
    if (rect && (!d_vis || cam->ssaa != 1)) return RC_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(d_rgba) | reinterpret_cast<uintptr_t>(d_hit) |
         reinterpret_cast<uintptr_t>(d_sample_rgba)) & 15u)
        return RC_ERR_INVALID_ARG;
    if (!s->built) return RC_ERR_NOT_BUILT;
    DevLights L;
    st = fill_lights(L, lights, n_lights, rect);
    if (st != RC_OK) return st;
    RC_HIP(hipSetDevice(c->device));
    DevCamera dc = make_camera(cam);
    DevScene ds = dev_scene(s);
    rc_launch_shade(ds, dc, L, reinterpret_cast<const uint4*>(d_hit), n_lights ? d_shadow : nullptr, d_vis, d_rgba,
                    d_sample_rgba, c->d_counters + 9, c->stream);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

int rc_postprocess(rc_ctx* c, const float* d_rgba, uint32_t width, uint32_t height, uint32_t flags, uint8_t* d_out)
{
    if (!c || !d_rgba || !d_out || width == 0 || height == 0) return RC_ERR_INVALID_ARG;
    if ((flags & ~(uint32_t)RC_POST_FXAA) != 0) return RC_ERR_INVALID_ARG;
    if ((uint64_t)width * height > (1ull << 30)) return RC_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(d_rgba) & 15u || reinterpret_cast<uintptr_t>(d_out) & 3u) return RC_ERR_INVALID_ARG;
    RC_HIP(hipSetDevice(c->device));
    const bool fxaa = (flags & RC_POST_FXAA) != 0;
    const size_t bytes = (size_t)width * height * 4;
    if (fxaa && bytes > c->post_cap) {
        RC_HIP(hipStreamSynchronize(c->stream));
        dev_free(c->d_post);
        c->post_cap = 0;
        int st = dev_alloc(&c->d_post, bytes);
        if (st != RC_OK) return st;
        c->post_cap = bytes;
    }
    rc_launch_postprocess(d_rgba, width, height, fxaa, c->d_post, d_out, c->stream);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

static_assert(RC_POST_SCRATCH_PIXELS == (uint32_t)RC_POST_NOALLOC_MAX_PIXELS, "scratch size of the ABI");

int rc_postprocess_noalloc(rc_ctx* c, const float* d_rgba, uint32_t width, uint32_t height, uint32_t flags,
                           uint8_t* d_out)
{
    if (!c || !d_rgba || !d_out || width == 0 || height == 0) return RC_ERR_INVALID_ARG;
    if ((flags & ~(uint32_t)RC_POST_FXAA) != 0) return RC_ERR_INVALID_ARG;
    if ((uint64_t)width * height > RC_POST_NOALLOC_MAX_PIXELS) return RC_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(d_rgba) & 15u || reinterpret_cast<uintptr_t>(d_out) & 3u) return RC_ERR_INVALID_ARG;
    uint8_t* scratch = rc_post_scratch(c->device);
    if (!scratch) return RC_ERR_HIP;
    RC_HIP(hipSetDevice(c->device));
    rc_launch_postprocess(d_rgba, width, height, (flags & RC_POST_FXAA) != 0, scratch, d_out, c->stream);
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

int rc_pack_features(rc_ctx* c, rc_scene* s, const rc_camera* cam, const uint32_t* d_hit, const float* d_vis,
                     float depth_norm, uint16_t* d_feat)
{
    if (!c || !s || !cam || !d_hit || !d_vis || !d_feat) return RC_ERR_INVALID_ARG;
    int st = check_camera(cam);
    if (st != RC_OK) return st;
    if (cam->ssaa != 1) return RC_ERR_UNSUPPORTED;
    if (!(depth_norm > 0.0f) || !isfinite(depth_norm)) return RC_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(d_hit) | reinterpret_cast<uintptr_t>(d_feat)) & 15u) return RC_ERR_INVALID_ARG;
    if (!s->built) return RC_ERR_NOT_BUILT;
    RC_HIP(hipSetDevice(c->device));
    DevCamera dc = make_camera(cam);
    DevScene ds = dev_scene(s);
    rc_launch_pack_features(ds, dc, reinterpret_cast<const uint4*>(d_hit), d_vis, (float)(1.0 / log1p((double)depth_norm)),
                            d_feat, c->d_counters + 9, c->stream);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

int rc_get_stage_times(rc_ctx* c, rc_stage_times* o)
{
    if (!c || !o) return RC_ERR_INVALID_ARG;
    memset(o, 0, sizeof(*o));
    RC_HIP(hipSetDevice(c->device));
    RC_HIP(hipStreamSynchronize(c->stream));
    if (c->timed && !c->timed_batch) {
        RC_HIP(hipEventElapsedTime(&o->ms[0], c->ev[0], c->ev[1]));
        RC_HIP(hipEventElapsedTime(&o->ms[1], c->ev[1], c->ev[2]));
        RC_HIP(hipEventElapsedTime(&o->ms[2], c->ev[2], c->ev[3]));
    }
    if (c->timed) RC_HIP(hipEventElapsedTime(&o->ms[3], c->ev[0], c->ev[3]));
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

// ------------------------------------------------------------------------- batch
namespace {

uint64_t fnv1a(uint64_t h, const void* p, size_t n)
{
    const uint8_t* b = static_cast<const uint8_t*>(p);
    for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    return h;
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

int check_tune(rc_tune* t, int max_wps)
{
    if (t->tile_w == 0) t->tile_w = 8;
    if (t->tile_h == 0) t->tile_h = 8;
    if (t->queue_depth == 0) t->queue_depth = 256;
    if (t->min_rays == 0) t->min_rays = 40;
    if (t->passes == 0) t->passes = 3;
    if (t->passes != 1 && t->passes != 3) return RC_ERR_INVALID_ARG;
    if (t->waves_per_simd == 0 || t->waves_per_simd > (uint32_t)max_wps) t->waves_per_simd = (uint32_t)max_wps;
    uint32_t tp = t->tile_w * t->tile_h;
    if (tp < 16 || tp > 1024 || t->queue_depth < 64 || t->queue_depth > 4096 || t->queue_depth % 64 ||
        t->min_rays > 64)
        return RC_ERR_INVALID_ARG;
    return RC_OK;
}

// resident waves per SIMD allowed by the occupancy of a batch kernel (pass 0: the one-kernel form)
int batch_wps_limit(int device, int pass)
{
    return std::max(1, rc_batch_max_blocks_per_cu(device, pass) * (RC_TRACE_BLOCK / 64) / 4);
}

// largest limit among the kernels of a form (1 pass: the one kernel; 3: camera, shadow and shading kernels)
int batch_form_wps(int device, uint32_t passes)
{
    if (passes == 1) return batch_wps_limit(device, 0);
    return std::max(batch_wps_limit(device, 1), std::max(batch_wps_limit(device, 2), batch_wps_limit(device, 3)));
}

struct BatchPlan {
    std::vector<DevScene> scenes;
    std::vector<DevView> views;
    uint32_t n_items = 0;
    uint32_t max_stack = 0;
    uint64_t n_samples = 0;    // samples of all views: entries of the three-kernel form's shadow-ray setup
    size_t bytes = 0, off_views = 0, off_lights = 0;
};

int plan_batch(rc_scene* const* scenes, uint32_t n_scenes, const rc_view* views, uint32_t n_views,
               const rc_point_light* lights, uint32_t n_lights_total, const rc_tune& t, BatchPlan& bp)
{
    if (!scenes || n_scenes == 0 || !views || n_views == 0) return RC_ERR_INVALID_ARG;
    if (n_lights_total > 0 && !lights) return RC_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < n_scenes; ++i) {
        if (!scenes[i]) return RC_ERR_INVALID_ARG;
        if (!scenes[i]->built) return RC_ERR_NOT_BUILT;
        if (scenes[i]->two_level || scenes[i]->watertight) return RC_ERR_UNSUPPORTED;
        bp.scenes.push_back(dev_scene(scenes[i]));
        bp.max_stack = std::max(bp.max_stack, scenes[i]->hb.max_stack);
    }
    uint64_t items = 0;
    for (uint32_t v = 0; v < n_views; ++v) {
        const rc_view& V = views[v];
        const rc_camera* cam = &V.camera;
        if (V.scene >= n_scenes) return RC_ERR_INVALID_ARG;
        if (cam->width <= 0 || cam->height <= 0 || (int64_t)cam->width * cam->height > (1ll << 28)) return RC_ERR_INVALID_ARG;
        if (cam->ssaa != 1 && cam->ssaa != 2) return RC_ERR_UNSUPPORTED;
        if (!(cam->vfov_deg > 0.0f && cam->vfov_deg < 180.0f) || !finite3(cam->eye) || !finite3(cam->target) ||
            !finite3(cam->up))
            return RC_ERR_INVALID_VALUE;
        if (V.n_lights > 16 || (uint64_t)V.light_first + V.n_lights > n_lights_total) return RC_ERR_INVALID_ARG;
        if (!V.d_rgba || !V.d_hit || (V.n_lights > 0 && !V.d_shadow)) return RC_ERR_INVALID_ARG;
        if ((reinterpret_cast<uintptr_t>(V.d_rgba) | reinterpret_cast<uintptr_t>(V.d_hit)) & 15u) return RC_ERR_INVALID_ARG;
        DevView d;
        memset(&d, 0, sizeof(d));
        d.cam = make_camera(cam);
        d.scene = V.scene;
        d.light_first = V.light_first;
        d.n_lights = V.n_lights;
        d.tiles_x = ((uint32_t)cam->width + t.tile_w - 1) / t.tile_w;
        uint32_t tiles_y = ((uint32_t)cam->height + t.tile_h - 1) / t.tile_h;
        d.item_first = (uint32_t)items;
        items += (uint64_t)d.tiles_x * tiles_y * t.tile_w * t.tile_h;
        d.setup_first = (uint32_t)bp.n_samples;
        bp.n_samples += (uint64_t)cam->width * cam->height * cam->ssaa * cam->ssaa;
        if (bp.n_samples >= (1ull << 32)) return RC_ERR_UNSUPPORTED;
        d.rgba = V.d_rgba;
        d.hit = reinterpret_cast<uint4*>(V.d_hit);
        d.shadow = V.n_lights > 0 ? V.d_shadow : nullptr;
        bp.views.push_back(d);
    }
    if (items >= (1ull << 32) - 8192) return RC_ERR_UNSUPPORTED;
    for (uint32_t l = 0; l < n_lights_total; ++l)
        if (!finite3(lights[l].position) || !finite3(lights[l].intensity)) return RC_ERR_INVALID_VALUE;
    bp.n_items = (uint32_t)items;
    bp.off_views = align16(sizeof(DevScene) * n_scenes);
    bp.off_lights = bp.off_views + align16(sizeof(DevView) * n_views);
    bp.bytes = bp.off_lights + align16(sizeof(float) * 6 * std::max<uint32_t>(n_lights_total, 1));
    return RC_OK;
}

int batch_launch(rc_ctx* c, rc_scene* const* scenes, uint32_t n_scenes, const rc_view* views, uint32_t n_views,
                 const rc_point_light* lights, uint32_t n_lights_total, const rc_tune* tune_in, uint32_t flags)
{
    if (!c) return RC_ERR_INVALID_ARG;
    RC_HIP(hipSetDevice(c->device));
    int n_cu = 0;
    RC_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
    rc_tune t = tune_in ? *tune_in : rc_tune{0, 0, 0, 0, 0, 0};
    const uint32_t passes_in = t.passes == 0 ? 3u : t.passes;
    if (passes_in != 1 && passes_in != 3) return RC_ERR_INVALID_ARG;
    int st = check_tune(&t, batch_form_wps(c->device, passes_in));
    if (st != RC_OK) return st;
    BatchPlan bp;
    st = plan_batch(scenes, n_scenes, views, n_views, lights, n_lights_total, t, bp);
    if (st != RC_OK) return st;
    // persistent grid of each launch: the requested waves per SIMD, capped at that kernel's own occupancy
    const int blocks_req = std::max(1, (int)(t.waves_per_simd * 4) / (RC_TRACE_BLOCK / 64));
    int grids[4] = {0, 0, 0, 0};
    for (int p = 0; p < 4; ++p)
        if ((p == 0) == (t.passes == 1))
            grids[p] = n_cu * std::min(blocks_req, rc_batch_max_blocks_per_cu(c->device, p));
    const int grid = std::max(std::max(grids[0], grids[1]), std::max(grids[2], grids[3]));

    // overflow stack area for this grid
    uint32_t depth = bp.max_stack > RC_STACK_LDS ? bp.max_stack - RC_STACK_LDS : 0;
    size_t words = (size_t)grid * RC_TRACE_BLOCK * depth * 2;
    if (words > c->overflow_words || !c->d_overflow) {
        RC_HIP(hipStreamSynchronize(c->stream));
        dev_free(c->d_overflow);
        c->overflow_words = 0;
        st = dev_alloc(&c->d_overflow, words);
        if (st != RC_OK) return st;
        c->overflow_words = words;
        c->graph_key = 0;   // the captured graph points at the old buffer
    }
    // table: device copy of scenes, views and lights, staged through pinned host memory
    if (bp.bytes > c->table_cap) {
        RC_HIP(hipStreamSynchronize(c->stream));
        if (c->h_table) hipHostFree(c->h_table);
        dev_free(c->d_table);
        c->h_table = nullptr;
        c->table_cap = 0;
        RC_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_table), bp.bytes, hipHostMallocDefault));
        st = dev_alloc(&c->d_table, bp.bytes);
        if (st != RC_OK) return st;
        c->table_cap = bp.bytes;
        c->graph_key = 0;
    }
    if (!c->ev_staging) RC_HIP(hipEventCreateWithFlags(&c->ev_staging, hipEventDisableTiming));
    if (c->staging_pending) RC_HIP(hipEventSynchronize(c->ev_staging));
    memcpy(c->h_table, bp.scenes.data(), sizeof(DevScene) * n_scenes);
    memcpy(c->h_table + bp.off_views, bp.views.data(), sizeof(DevView) * n_views);
    for (uint32_t l = 0; l < n_lights_total; ++l) {
        float* L = reinterpret_cast<float*>(c->h_table + bp.off_lights) + 6 * l;
        for (int k = 0; k < 3; ++k) { L[k] = lights[l].position[k]; L[3 + k] = lights[l].intensity[k]; }
    }
    RC_HIP(hipMemcpyAsync(c->d_table, c->h_table, bp.bytes, hipMemcpyHostToDevice, c->stream));
    RC_HIP(hipEventRecord(c->ev_staging, c->stream));
    c->staging_pending = true;

    // shadow-ray setup entries of the three-kernel form (2 float4 per sample)
    if (t.passes == 3 && 2 * bp.n_samples > c->bsetup_cap) {
        RC_HIP(hipStreamSynchronize(c->stream));
        dev_free(c->d_bsetup);
        c->bsetup_cap = 0;
        st = dev_alloc(&c->d_bsetup, 2 * bp.n_samples);
        if (st != RC_OK) return st;
        c->bsetup_cap = 2 * bp.n_samples;
        c->graph_key = 0;   // the captured graph points at the old buffer
    }

    BatchParams P;
    memset(&P, 0, sizeof(P));
    P.setup = t.passes == 3 ? c->d_bsetup : nullptr;
    P.scenes = reinterpret_cast<const DevScene*>(c->d_table);
    P.views = reinterpret_cast<const DevView*>(c->d_table + bp.off_views);
    P.lights = reinterpret_cast<const float*>(c->d_table + bp.off_lights);
    P.n_views = n_views;
    P.n_items = bp.n_items;
    P.tune = BatchTune{t.tile_w, t.tile_h, t.queue_depth, t.min_rays, t.waves_per_simd, t.passes};
    P.w.counters = c->d_counters;
    P.w.overflow = c->d_overflow;
    P.w.overflow_depth = depth;
    P.w.n_lanes = (uint32_t)grid * RC_TRACE_BLOCK;
    P.w.error_flag = c->d_counters + 8;
    P.w.ray_count = (flags & RC_FLAG_COUNT) ? c->d_rays : nullptr;   // counts on request only

    bool timing = (flags & RC_FLAG_TIMING) != 0;
    if (timing) RC_HIP(hipEventRecord(c->ev[0], c->stream));
    if (flags & RC_FLAG_GRAPH) {
        uint64_t key = fnv1a(1469598103934665603ull, &P, sizeof(P));
        key = fnv1a(key, grids, sizeof(grids));
        if (key != c->graph_key || !c->graph_exec) {
            if (c->graph_exec) { hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
            if (c->graph) { hipGraphDestroy(c->graph); c->graph = nullptr; }
            if (!c->capture_stream) RC_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
            RC_HIP(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeRelaxed));
            rc_launch_fill_u32(c->d_counters, 0u, 8, c->capture_stream);   // not word 8: the sticky error flag
            rc_launch_fill_u32(c->d_counters + RC_QUEUE_BASE, 0u, RC_COUNTER_WORDS - RC_QUEUE_BASE, c->capture_stream);
            rc_launch_fill_u32(reinterpret_cast<uint32_t*>(c->d_rays), 0u, 16, c->capture_stream);
            for (int p = 0; p < 4; ++p)
                if (grids[p]) rc_launch_batch(P, p, grids[p], c->capture_stream);
            hipError_t e = hipStreamEndCapture(c->capture_stream, &c->graph);
            if (e != hipSuccess) return RC_ERR_HIP;
            RC_HIP(hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
            c->graph_key = key;
        }
        RC_HIP(hipGraphLaunch(c->graph_exec, c->stream));
    } else {
        rc_launch_fill_u32(c->d_counters, 0u, 8, c->stream);   // not word 8: the sticky error flag
        rc_launch_fill_u32(c->d_counters + RC_QUEUE_BASE, 0u, RC_COUNTER_WORDS - RC_QUEUE_BASE, c->stream);
        rc_launch_fill_u32(reinterpret_cast<uint32_t*>(c->d_rays), 0u, 16, c->stream);
        if (t.passes == 1) {
            rc_launch_batch(P, 0, grids[0], c->stream);
        } else {
            // events between the stages: per-pass times in rc_get_stage_times ms[0..2]
            rc_launch_batch(P, 1, grids[1], c->stream);
            if (timing) RC_HIP(hipEventRecord(c->ev[1], c->stream));
            rc_launch_batch(P, 2, grids[2], c->stream);
            if (timing) RC_HIP(hipEventRecord(c->ev[2], c->stream));
            rc_launch_batch(P, 3, grids[3], c->stream);
        }
    }
    if (timing) RC_HIP(hipEventRecord(c->ev[3], c->stream));
    c->timed = timing;
    c->timed_batch = !(t.passes == 3 && !(flags & RC_FLAG_GRAPH));
    RC_HIP(hipGetLastError());
    return RC_OK;
}

std::string tune_key(rc_ctx* c, rc_scene* const* scenes, uint32_t n_scenes, const rc_view* views, uint32_t n_views)
{
    hipDeviceProp_t prop;
    memset(&prop, 0, sizeof(prop));
    hipGetDeviceProperties(&prop, c->device);
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, &n_scenes, sizeof(n_scenes));
    for (uint32_t i = 0; i < n_scenes; ++i) {
        uint64_t sz[2] = {scenes[i]->nt, scenes[i]->hb.nodes.size()};
        h = fnv1a(h, sz, sizeof(sz));
    }
    h = fnv1a(h, &n_views, sizeof(n_views));
    for (uint32_t v = 0; v < n_views; ++v) {
        int32_t f[5] = {(int32_t)views[v].scene, views[v].camera.width, views[v].camera.height, views[v].camera.ssaa,
                        (int32_t)views[v].n_lights};
        h = fnv1a(h, f, sizeof(f));
    }
    char arch[64];
    snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
    for (char* p = arch; *p; ++p)
        if (*p == ':' || *p == '"') { *p = 0; break; }
    char buf[160];
    snprintf(buf, sizeof(buf), "%s:%d:%016llx", arch, prop.multiProcessorCount, (unsigned long long)h);
    return buf;
}

bool read_field(const char* line, const char* name, double* out)
{
    char pat[64];
    snprintf(pat, sizeof(pat), "\"%s\":", name);
    const char* p = strstr(line, pat);
    if (!p) return false;
    return sscanf(p + strlen(pat), "%lf", out) == 1;
}

bool cache_lookup(const char* path, const std::string& key, rc_tune* t, float* ms)
{
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    std::string pat = "\"key\":\"" + key + "\"";
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        if (!strstr(line, pat.c_str())) continue;
        double a, b, q, m, w, x = 0;
        if (read_field(line, "tile_w", &a) && read_field(line, "tile_h", &b) && read_field(line, "queue_depth", &q) &&
            read_field(line, "min_rays", &m) && read_field(line, "waves_per_simd", &w)) {
            read_field(line, "ms", &x);
            double ps = 1;   // entries written before the three-kernel form existed were one-kernel tunings
            read_field(line, "passes", &ps);
            *t = rc_tune{(uint32_t)a, (uint32_t)b, (uint32_t)q, (uint32_t)m, (uint32_t)w, (uint32_t)ps};
            *ms = (float)x;
            found = true;
        }
    }
    fclose(f);
    return found;
}

}  // namespace

extern "C" {

int rc_render_batch(rc_ctx* c, rc_scene* const* scenes, uint32_t n_scenes, const rc_view* views, uint32_t n_views,
                    const rc_point_light* lights, uint32_t n_lights_total, const rc_tune* tune, uint32_t flags)
{
    return batch_launch(c, scenes, n_scenes, views, n_views, lights, n_lights_total, tune, flags);
}

int rc_autotune(rc_ctx* c, rc_scene* const* scenes, uint32_t n_scenes, const rc_view* views, uint32_t n_views,
                const rc_point_light* lights, uint32_t n_lights_total, const rc_tune* candidates, uint32_t n_candidates,
                uint32_t reps, const char* cache_path, rc_tune* best, float* best_ms)
{
    if (!c || !best) return RC_ERR_INVALID_ARG;
    if (reps == 0) reps = 3;
    RC_HIP(hipSetDevice(c->device));
    std::string key;
    if (cache_path) {
        BatchPlan probe;
        rc_tune d = {8, 8, 256, 40, 1, 3};
        int st = plan_batch(scenes, n_scenes, views, n_views, lights, n_lights_total, d, probe);
        if (st != RC_OK) return st;
        key = tune_key(c, scenes, n_scenes, views, n_views);
        float ms = 0.0f;
        if (cache_lookup(cache_path, key, best, &ms)) {
            if (best_ms) *best_ms = ms;
            return RC_OK;
        }
    }
    std::vector<rc_tune> cand;
    if (candidates && n_candidates) {
        cand.assign(candidates, candidates + n_candidates);
    } else {
        const uint32_t tiles[3][2] = {{8, 8}, {16, 8}, {16, 16}};
        const uint32_t depths[3] = {64, 256, 1024};
        const uint32_t mins[3] = {16, 32, 48};
        for (uint32_t passes : {1u, 3u}) {
            const uint32_t max_wps = (uint32_t)batch_form_wps(c->device, passes);
            for (auto& tl : tiles)
                for (uint32_t q : depths)
                    for (uint32_t m : mins)
                        for (uint32_t w = max_wps; w + 1 >= max_wps && w >= 1; --w)
                            cand.push_back(rc_tune{tl[0], tl[1], q, m, w, passes});
        }
    }
    hipEvent_t e0, e1;
    RC_HIP(hipEventCreate(&e0));
    RC_HIP(hipEventCreate(&e1));
    float best_t = INFINITY;
    int st = RC_OK;
    for (const rc_tune& t : cand) {
        std::vector<float> times;
        for (uint32_t r = 0; r <= reps && st == RC_OK; ++r) {
            if (hipEventRecord(e0, c->stream) != hipSuccess) { st = RC_ERR_HIP; break; }
            st = batch_launch(c, scenes, n_scenes, views, n_views, lights, n_lights_total, &t, 0);
            if (st != RC_OK) break;
            if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { st = RC_ERR_HIP; break; }
            float ms = 0;
            hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) times.push_back(ms);
        }
        if (st != RC_OK) break;
        std::sort(times.begin(), times.end());
        float med = times[times.size() / 2];
        if (med < best_t) { best_t = med; *best = t; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != RC_OK) return st;
    if (best_ms) *best_ms = best_t;
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "{\"key\":\"%s\",\"tile_w\":%u,\"tile_h\":%u,\"queue_depth\":%u,\"min_rays\":%u,"
                       "\"waves_per_simd\":%u,\"passes\":%u,\"ms\":%.4f}\n",
                    key.c_str(), best->tile_w, best->tile_h, best->queue_depth, best->min_rays, best->waves_per_simd,
                    best->passes, best_t);
            fclose(f);
        }
    }
    return RC_OK;
}

}  // extern "C"
