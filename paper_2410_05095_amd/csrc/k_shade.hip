// Shading + supersampling resolve, triangle packing, rigid-body transforms and BVH refit.
#include "rc_trav.h"

namespace {

// One thread per pixel: every sample is shaded in FP64 from the FP32 hit (the hit point is
// reconstructed from the camera ray and the triangle), rounded to FP32, and the samples are
// box-averaged in the fixed order ((s0 + s1) + (s2 + s3)) * 0.25.
// A hit id at or beyond the scene's triangle count (a G-buffer from another scene) is shaded as a miss and
// sets the context's invalid-value flag.
__global__ __launch_bounds__(256) void k_shade(DevScene sc, DevCamera cam, DevLights L, const uint4* gbuf,
                                               const uint32_t* mask, const float* vis, float* rgba,
                                               float* sample_rgba, uint32_t* bad_value)
{
    const uint32_t n_pix = (uint32_t)cam.width * (uint32_t)cam.height;
    const uint32_t pixel = blockIdx.x * blockDim.x + threadIdx.x;
    if (pixel >= n_pix) return;
    const uint32_t spp = (uint32_t)(cam.ssaa * cam.ssaa);
    float4 smp[4];
    for (uint32_t k = 0; k < spp; ++k) {
        size_t s = (size_t)pixel * spp + k;
        uint4 h = gbuf[s];
        float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
        if (h.x != RC_NO_HIT && h.x >= sc.n_tris) {
            *bad_value = 1u;
        } else if (h.x != RC_NO_HIT) {
            out = rc_shade_sample(sc, cam, &L.point[0][0], L.n_point, L.has_rect ? L.rect : nullptr,
                                  L.has_rect ? (double)vis[pixel] : 0.0, pixel, k, h.x, mask ? mask[s] : 0u);
        }
        smp[k] = out;
        if (sample_rgba) reinterpret_cast<float4*>(sample_rgba)[s] = out;
    }
    float4 r;
    if (spp == 4) {
        float4 a, b;
        a.x = smp[0].x + smp[1].x; a.y = smp[0].y + smp[1].y; a.z = smp[0].z + smp[1].z; a.w = smp[0].w + smp[1].w;
        b.x = smp[2].x + smp[3].x; b.y = smp[2].y + smp[3].y; b.z = smp[2].z + smp[3].z; b.w = smp[2].w + smp[3].w;
        r.x = (a.x + b.x) * 0.25f; r.y = (a.y + b.y) * 0.25f; r.z = (a.z + b.z) * 0.25f; r.w = (a.w + b.w) * 0.25f;
    } else {
        r = smp[0];
    }
    reinterpret_cast<float4*>(rgba)[pixel] = r;
}

// slot i of the leaf order: (v0, id), (v1 - v0, 0), (v2 - v0, 0)
// Triangle records in leaf order: (v0, id), then the FP32 edges (v1 - v0), (v2 - v0) for Moller-Trumbore, or
// the vertices v1, v2 themselves for the watertight test (raw), whose shared edges must see identical values.
__global__ __launch_bounds__(256) void k_pack(const float* pos, const uint32_t* idx, const uint32_t* order,
                                              uint32_t n, uint32_t raw, float4* tris)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t t = order[i];
    const uint32_t* ix = idx + 3 * (size_t)t;
    const float* a = pos + 3 * (size_t)ix[0];
    const float* b = pos + 3 * (size_t)ix[1];
    const float* c = pos + 3 * (size_t)ix[2];
    tris[3 * (size_t)i + 0] = make_float4(a[0], a[1], a[2], __uint_as_float(t));
    if (raw) {
        tris[3 * (size_t)i + 1] = make_float4(b[0], b[1], b[2], 0.0f);
        tris[3 * (size_t)i + 2] = make_float4(c[0], c[1], c[2], 0.0f);
    } else {
        tris[3 * (size_t)i + 1] = make_float4(b[0] - a[0], b[1] - a[1], b[2] - a[2], 0.0f);
        tris[3 * (size_t)i + 2] = make_float4(c[0] - a[0], c[1] - a[1], c[2] - a[2], 0.0f);
    }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// x' = ((R00 x + R01 y) + R02 z) + t0 per row, from the rest positions of body body_ids[blockIdx.y]
// vertex normals (when present) are rotated the same way, without the translation
__global__ __launch_bounds__(256) void k_transform(const float* rest, float* pos, const float* nrm_rest, float* nrm,
                                                   const uint32_t* body_vrange, const float* xf,
                                                   const uint32_t* body_ids, uint32_t n_bodies, uint32_t* bad_value)
{
    uint32_t b = blockIdx.y;
    uint32_t body = body_ids[b];
    if (body >= n_bodies) {   // not a body of the scene: nothing moves, the invalid-value flag is set
        if (blockIdx.x == 0 && threadIdx.x == 0) *bad_value = 1u;
        return;
    }
    uint32_t first = body_vrange[2 * (size_t)body], count = body_vrange[2 * (size_t)body + 1];
    const float* M = xf + 12 * (size_t)b;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const float* p = rest + 3 * (size_t)(first + i);
        float x = p[0], y = p[1], z = p[2];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            float a = M[4 * r + 0] * x;
            float bb = M[4 * r + 1] * y;
            float cc = M[4 * r + 2] * z;
            pos[3 * (size_t)(first + i) + r] = ((a + bb) + cc) + M[4 * r + 3];
        }
        if (nrm) {
            const float* q = nrm_rest + 3 * (size_t)(first + i);
            float nx = q[0], ny = q[1], nz = q[2];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                float a = M[4 * r + 0] * nx;
                float bb = M[4 * r + 1] * ny;
                float cc = M[4 * r + 2] * nz;
                nrm[3 * (size_t)(first + i) + r] = (a + bb) + cc;
            }
        }
    }
}

// The current rigid map of each moved body (read by the top level of two-level structures).
__global__ __launch_bounds__(256) void k_record_o2w(const float* xf, const uint32_t* body_ids, uint32_t n,
                                                    uint32_t scene_bodies, float* o2w)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 12 * n) return;
    const uint32_t body = body_ids[q / 12];
    if (body < scene_bodies) o2w[12 * (size_t)body + q % 12] = xf[q];
}

// Refit of a flat BVH touching only moved bodies.  tri_node[t] = the node whose leaf child holds triangle t;
// rc_scene_set_transforms marks (dirty = 1) the nodes holding triangles of the moved bodies; the refit then
// goes through the levels from the deepest, recomputing only marked nodes (exact FP32 min/max of their leaf
// triangles' current vertices, whose packed records are rewritten on the way, and of their already refit child
// nodes), each marking its parent.  Untouched nodes keep boxes that are exact for their unmoved triangles, so
// the result equals a full refit bit for bit.
__global__ __launch_bounds__(256) void k_tri_nodes(const Node4* nodes, uint32_t n_nodes, const uint32_t* order,
                                                   uint32_t* tri_node)
{
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint32_t w = nodes[n].child[c];
        if (!rc_is_leaf(w)) continue;
        for (uint32_t i = 0; i < rc_leaf_count(w); ++i) tri_node[order[rc_leaf_first(w) + i]] = n;
    }
}

// grid (x: triangle blocks of the largest body, y: moved bodies): mark the nodes holding moved triangles
__global__ __launch_bounds__(256) void k_mark_dirty(const uint32_t* body_ids, uint32_t n_bodies, const uint32_t* tri_off,
                                                    const uint32_t* body_tris, const uint32_t* tri_node,
                                                    uint32_t* dirty, uint32_t n_nodes)
{
    const uint32_t b = body_ids[blockIdx.y];
    if (b >= n_bodies) return;   // reported by k_transform
    const uint32_t i = tri_off[b] + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tri_off[b + 1]) return;
    const uint32_t n = tri_node[body_tris[i]];
    if (n < n_nodes) dirty[n] = 1u;
}

// The marked nodes of one level (first .. first + count - 1), four threads per node: thread c recomputes child
// slot c; thread 0 then clears the node's mark and marks its parent (read by the next launch).
__global__ __launch_bounds__(256) void k_refit_level_dirty(Node4* nodes, const float* pos, const uint32_t* idx,
                                                           const uint32_t* order, float4* tris, uint32_t raw,
                                                           uint32_t* dirty, uint32_t first, uint32_t count,
                                                           uint32_t n_nodes)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q / 4 >= count) return;
    const uint32_t n = first + q / 4, c = q & 3u;
    if (dirty[n] == 0u) return;
    Node4* nd = nodes + n;
    const uint32_t w = nd->child[c];
    if (w != RC_EMPTY_CHILD) {
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        if (rc_is_leaf(w)) {
            // independent loads first (slots, then vertex indices, then vertices), then the packed records
            const uint32_t f = rc_leaf_first(w), cnt = rc_leaf_count(w);
            uint32_t t[4], ix[4][3];
            float v[4][9];
#pragma unroll
            for (int i = 0; i < 4; ++i) t[i] = (uint32_t)i < cnt ? order[f + i] : 0u;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) ix[i][k] = (uint32_t)i < cnt ? idx[3 * (size_t)t[i] + k] : 0u;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int k = 0; k < 9; ++k) v[i][k] = (uint32_t)i < cnt ? pos[3 * (size_t)ix[i][k / 3] + k % 3] : 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if ((uint32_t)i >= cnt) continue;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    lo[k] = fminf(fminf(fminf(lo[k], v[i][k]), v[i][3 + k]), v[i][6 + k]);
                    hi[k] = fmaxf(fmaxf(fmaxf(hi[k], v[i][k]), v[i][3 + k]), v[i][6 + k]);
                }
                float4* tp = tris + 3 * (size_t)(f + i);
                tp[0] = make_float4(v[i][0], v[i][1], v[i][2], __uint_as_float(t[i]));
                if (raw) {
                    tp[1] = make_float4(v[i][3], v[i][4], v[i][5], 0.0f);
                    tp[2] = make_float4(v[i][6], v[i][7], v[i][8], 0.0f);
                } else {
                    tp[1] = make_float4(v[i][3] - v[i][0], v[i][4] - v[i][1], v[i][5] - v[i][2], 0.0f);
                    tp[2] = make_float4(v[i][6] - v[i][0], v[i][7] - v[i][1], v[i][8] - v[i][2], 0.0f);
                }
            }
        } else {
            const Node4* ch = nodes + w;
            const float4 lx = *reinterpret_cast<const float4*>(ch->lo_x), hx = *reinterpret_cast<const float4*>(ch->hi_x);
            const float4 ly = *reinterpret_cast<const float4*>(ch->lo_y), hy = *reinterpret_cast<const float4*>(ch->hi_y);
            const float4 lz = *reinterpret_cast<const float4*>(ch->lo_z), hz = *reinterpret_cast<const float4*>(ch->hi_z);
            lo[0] = fminf(fminf(lx.x, lx.y), fminf(lx.z, lx.w)); hi[0] = fmaxf(fmaxf(hx.x, hx.y), fmaxf(hx.z, hx.w));
            lo[1] = fminf(fminf(ly.x, ly.y), fminf(ly.z, ly.w)); hi[1] = fmaxf(fmaxf(hy.x, hy.y), fmaxf(hy.z, hy.w));
            lo[2] = fminf(fminf(lz.x, lz.y), fminf(lz.z, lz.w)); hi[2] = fmaxf(fmaxf(hz.x, hz.y), fmaxf(hz.z, hz.w));
        }
        nd->lo_x[c] = lo[0]; nd->hi_x[c] = hi[0];
        nd->lo_y[c] = lo[1]; nd->hi_y[c] = hi[1];
        nd->lo_z[c] = lo[2]; nd->hi_z[c] = hi[2];
    }
    if (c == 0u) {   // every lane of the node read the mark above, in the same instruction
        dirty[n] = 0u;
        const uint32_t p = nd->parent;
        if (p < n_nodes) dirty[p] = 1u;   // the root's parent is 0xFFFFFFFF
    }
}

// One thread per node of one BVH level: child boxes from the triangles of leaf children and
// from the (already refit) boxes of internal children.  Exact FP32 min/max.
__global__ __launch_bounds__(256) void k_refit(Node4* nodes, const float* pos, const uint32_t* idx,
                                               const uint32_t* order, uint32_t first, uint32_t count)
{
    uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    Node4* n = nodes + first + q;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        uint32_t w = n->child[c];
        if (w == RC_EMPTY_CHILD) continue;
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        if (rc_is_leaf(w)) {
            uint32_t f = rc_leaf_first(w), cnt = rc_leaf_count(w);
            for (uint32_t i = 0; i < cnt; ++i) {
                const uint32_t* ix = idx + 3 * (size_t)order[f + i];
                for (int v = 0; v < 3; ++v) {
                    const float* p = pos + 3 * (size_t)ix[v];
                    for (int a = 0; a < 3; ++a) { lo[a] = fminf(lo[a], p[a]); hi[a] = fmaxf(hi[a], p[a]); }
                }
            }
        } else {
            const Node4* ch = nodes + w;
            for (int k = 0; k < 4; ++k) {
                lo[0] = fminf(lo[0], ch->lo_x[k]); hi[0] = fmaxf(hi[0], ch->hi_x[k]);
                lo[1] = fminf(lo[1], ch->lo_y[k]); hi[1] = fmaxf(hi[1], ch->hi_y[k]);
                lo[2] = fminf(lo[2], ch->lo_z[k]); hi[2] = fmaxf(hi[2], ch->hi_z[k]);
            }
        }
        n->lo_x[c] = lo[0]; n->hi_x[c] = hi[0];
        n->lo_y[c] = lo[1]; n->hi_y[c] = hi[1];
        n->lo_z[c] = lo[2]; n->hi_z[c] = hi[2];
    }
}

__global__ __launch_bounds__(256) void k_camera_rays(DevCamera cam, float* o, float* d, uint32_t n)
{
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t spp = (uint32_t)(cam.ssaa * cam.ssaa);
    float of[3], df[3];
    rc_camera_ray(cam, s / spp, s % spp, of, df);
    for (int a = 0; a < 3; ++a) { o[3 * (size_t)s + a] = of[a]; d[3 * (size_t)s + a] = df[a]; }
}

__device__ inline uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}

// denoiser features per pixel: 1-spp visibility, log depth, normal, albedo (background: 1, 1, 0...); a hit id
// beyond the scene's triangles is packed as background and sets the invalid-value flag
__global__ __launch_bounds__(256) void k_pack_features(DevScene sc, DevCamera cam, const uint4* gbuf, const float* vis,
                                                       float inv_log_norm, uint16_t* feat, uint32_t* bad_value)
{
    uint32_t pixel = blockIdx.x * blockDim.x + threadIdx.x;
    if (pixel >= (uint32_t)(cam.width * cam.height)) return;
    uint4 h = gbuf[pixel];
    float f[8] = {1.0f, 1.0f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (h.x != RC_NO_HIT && h.x >= sc.n_tris) {
        *bad_value = 1u;
    } else if (h.x != RC_NO_HIT) {
        Surface S = rc_surface(sc, cam, pixel, 0, h.x);
        const float* mat = sc.mats + 5 * (size_t)sc.tri_mat[h.x];
        f[0] = vis[pixel];
        f[1] = log1pf(__uint_as_float(h.y)) * inv_log_norm;
        f[2] = (float)S.n.x; f[3] = (float)S.n.y; f[4] = (float)S.n.z;
        f[5] = mat[0]; f[6] = mat[1]; f[7] = mat[2];
    }
    uint4 o;
    o.x = (uint32_t)f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16);
    o.y = (uint32_t)f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16);
    o.z = (uint32_t)f2bf(f[4]) | ((uint32_t)f2bf(f[5]) << 16);
    o.w = (uint32_t)f2bf(f[6]) | ((uint32_t)f2bf(f[7]) << 16);
    reinterpret_cast<uint4*>(feat)[pixel] = o;
}

inline unsigned blocks(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void rc_launch_shade(const DevScene& sc, const DevCamera& cam, const DevLights& L, const uint4* gbuf,
                     const uint32_t* mask, const float* visibility, float* rgba, float* sample_rgba,
                     uint32_t* bad_value, hipStream_t st)
{
    size_t n = (size_t)cam.width * cam.height;
    hipLaunchKernelGGL(k_shade, dim3(blocks(n, 256)), dim3(256), 0, st, sc, cam, L, gbuf, mask, visibility, rgba,
                       sample_rgba, bad_value);
}

void rc_launch_camera_rays(const DevCamera& cam, float* o, float* d, uint32_t n, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_camera_rays, dim3(blocks(n, 256)), dim3(256), 0, st, cam, o, d, n);
}

void rc_launch_pack_features(const DevScene& sc, const DevCamera& cam, const uint4* gbuf, const float* vis,
                             float inv_log_norm, uint16_t* feat, uint32_t* bad_value, hipStream_t st)
{
    size_t n = (size_t)cam.width * cam.height;
    hipLaunchKernelGGL(k_pack_features, dim3(blocks(n, 256)), dim3(256), 0, st, sc, cam, gbuf, vis, inv_log_norm, feat,
                       bad_value);
}

void rc_launch_pack(const float* pos, const uint32_t* idx, const uint32_t* order, uint32_t n_tris, float4* tris,
                    bool raw, hipStream_t st)
{
    if (n_tris == 0) return;
    hipLaunchKernelGGL(k_pack, dim3(blocks(n_tris, 256)), dim3(256), 0, st, pos, idx, order, n_tris, raw ? 1u : 0u, tris);
}

void rc_launch_fill_u32(uint32_t* p, uint32_t value, uint32_t n, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks(n, 256)), dim3(256), 0, st, p, value, n);
}

void rc_launch_transform(const float* rest, float* pos, const float* nrm_rest, float* nrm,
                         const uint32_t* body_vrange, const float* xf, const uint32_t* body_ids, uint32_t n_bodies,
                         uint32_t max_count, uint32_t scene_bodies, uint32_t* bad_value, hipStream_t st)
{
    if (n_bodies == 0 || max_count == 0) return;
    unsigned gx = std::min(blocks(max_count, 256), 64u);
    hipLaunchKernelGGL(k_transform, dim3(gx, n_bodies), dim3(256), 0, st, rest, pos, nrm_rest, nrm, body_vrange, xf,
                       body_ids, scene_bodies, bad_value);
}

void rc_launch_record_o2w(const float* xf, const uint32_t* body_ids, uint32_t n, uint32_t scene_bodies, float* o2w,
                          hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_record_o2w, dim3(blocks(12 * n, 256)), dim3(256), 0, st, xf, body_ids, n, scene_bodies, o2w);
}

void rc_launch_refit_level(Node4* nodes, const float* pos, const uint32_t* idx, const uint32_t* order,
                           uint32_t first, uint32_t count, hipStream_t st)
{
    if (count == 0) return;
    hipLaunchKernelGGL(k_refit, dim3(blocks(count, 256)), dim3(256), 0, st, nodes, pos, idx, order, first, count);
}

void rc_launch_tri_nodes(const Node4* nodes, uint32_t n_nodes, const uint32_t* order, uint32_t* tri_node,
                         hipStream_t st)
{
    if (n_nodes == 0) return;
    hipLaunchKernelGGL(k_tri_nodes, dim3(blocks(n_nodes, 256)), dim3(256), 0, st, nodes, n_nodes, order, tri_node);
}

void rc_launch_mark_dirty(const uint32_t* body_ids, uint32_t n, uint32_t n_bodies, uint32_t max_body_tris,
                          const uint32_t* tri_off, const uint32_t* body_tris, const uint32_t* tri_node, uint32_t* dirty,
                          uint32_t n_nodes, hipStream_t st)
{
    if (n == 0 || max_body_tris == 0) return;
    hipLaunchKernelGGL(k_mark_dirty, dim3(blocks(max_body_tris, 256), n), dim3(256), 0, st, body_ids, n_bodies, tri_off,
                       body_tris, tri_node, dirty, n_nodes);
}

void rc_launch_refit_dirty(Node4* nodes, const float* pos, const uint32_t* idx, const uint32_t* order, float4* tris,
                           bool raw, uint32_t* dirty, const std::vector<uint32_t>& level_start, hipStream_t st)
{
    const int depth = (int)level_start.size() - 1;
    const uint32_t n_nodes = level_start[depth];
    for (int lv = depth - 1; lv >= 0; --lv) {
        const uint32_t first = level_start[lv], count = level_start[lv + 1] - level_start[lv];
        if (count == 0) continue;
        hipLaunchKernelGGL(k_refit_level_dirty, dim3(blocks(4 * (size_t)count, 256)), dim3(256), 0, st, nodes, pos, idx,
                           order, tris, raw ? 1u : 0u, dirty, first, count, n_nodes);
    }
}

