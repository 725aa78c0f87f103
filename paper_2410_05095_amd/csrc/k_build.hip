// BVH builds on the GPU: linear BVHs (Morton order of primitive centroids, the binary radix tree of Karras,
// 2012), boxes computed bottom-up with exact FP32 min/max, then collapsed level by level into the 4-wide,
// breadth-first node layout of the host builder (every subtree of at most max_leaf primitives becomes one
// leaf), so that traversal and refit use the trees unchanged.
//
//  * Flat build: one tree over all triangles.
//  * Bottom levels of a two-level structure: the triangles are sorted by (body, Morton code), so the
//    triangles of each body form one subtree of the radix tree; collapsing from the body subtrees' roots
//    gives one 4-wide tree per body (body b's root is node b), in one pass over all bodies.
//  * Top level: one leaf per instance over the instances' world boxes, rebuilt every frame on a stream
//    without host synchronisation or allocation (the collapse runs in one workgroup).
//
// Binary tree indexing: internal nodes 0 .. n-2, leaves n-1 .. 2n-2 (leaf n-1+i holds the primitive at
// sorted position i).
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "rc_internal.h"

namespace {

struct Box6 {
    float lo[3], hi[3];
};
static_assert(sizeof(Box6) == 24, "box record");

__device__ inline float4 box_centroid(const Box6& b)
{
    return make_float4(0.5f * b.lo[0] + 0.5f * b.hi[0], 0.5f * b.lo[1] + 0.5f * b.hi[1],
                       0.5f * b.lo[2] + 0.5f * b.hi[2], 0.0f);
}

__global__ __launch_bounds__(256) void k_tri_boxes(const float* pos, const uint32_t* idx, uint32_t n, Box6* box,
                                                   float4* cen)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    Box6 b;
#pragma unroll
    for (int k = 0; k < 3; ++k) { b.lo[k] = INFINITY; b.hi[k] = -INFINITY; }
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const float* p = pos + 3 * (size_t)idx[3 * (size_t)t + v];
#pragma unroll
        for (int k = 0; k < 3; ++k) { b.lo[k] = fminf(b.lo[k], p[k]); b.hi[k] = fmaxf(b.hi[k], p[k]); }
    }
    box[t] = b;
    cen[t] = box_centroid(b);
}

// Instance records of the top level: world-to-object map (M = R^T, m = -(R^T t), each component of R^T t as
// ((R0k t0 + R1k t1) + R2k t2) in FP32), the bottom-level root (node i for body i), and the world box: the
// eight corners of the body's rest box mapped by [R | t] in FP32, padded by 2^-18 of the largest coordinate
// magnitude (at least 1) to cover the rounding of the corners and of the rays mapped into the body.
__global__ __launch_bounds__(256) void k_instances(const float* o2w, const Node4* blas, uint32_t n, DevInst* inst,
                                                   Box6* box, float4* cen)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float X[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) X[k] = o2w[12 * (size_t)i + k];
    DevInst d;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int j = 0; j < 3; ++j) d.w2o[4 * k + j] = X[4 * j + k];
        const float a = X[k] * X[3];
        const float b = X[4 + k] * X[7];
        const float c = X[8 + k] * X[11];
        d.w2o[4 * k + 3] = -((a + b) + c);
    }
    d.root = i;
    d.pad[0] = d.pad[1] = d.pad[2] = 0u;
    inst[i] = d;
    const Node4& r = blas[i];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int c = 0; c < 4; ++c) {
        if (r.child[c] == RC_EMPTY_CHILD) continue;
        lo[0] = fminf(lo[0], r.lo_x[c]); hi[0] = fmaxf(hi[0], r.hi_x[c]);
        lo[1] = fminf(lo[1], r.lo_y[c]); hi[1] = fmaxf(hi[1], r.hi_y[c]);
        lo[2] = fminf(lo[2], r.lo_z[c]); hi[2] = fmaxf(hi[2], r.hi_z[c]);
    }
    Box6 w;
#pragma unroll
    for (int k = 0; k < 3; ++k) { w.lo[k] = INFINITY; w.hi[k] = -INFINITY; }
    for (int corner = 0; corner < 8; ++corner) {
        const float p[3] = {(corner & 1) ? hi[0] : lo[0], (corner & 2) ? hi[1] : lo[1], (corner & 4) ? hi[2] : lo[2]};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float a = X[4 * k] * p[0];
            const float b = X[4 * k + 1] * p[1];
            const float c = X[4 * k + 2] * p[2];
            const float v = ((a + b) + c) + X[4 * k + 3];
            w.lo[k] = fminf(w.lo[k], v);
            w.hi[k] = fmaxf(w.hi[k], v);
        }
    }
    float mag = 1.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) mag = fmaxf(mag, fmaxf(fabsf(w.lo[k]), fabsf(w.hi[k])));
    const float pad = mag * 0x1p-18f;
#pragma unroll
    for (int k = 0; k < 3; ++k) { w.lo[k] -= pad; w.hi[k] += pad; }
    box[i] = w;
    cen[i] = box_centroid(w);
}

// centroid bounds: per-block min/max, then one block over the partials
__global__ __launch_bounds__(256) void k_cen_bounds(const float4* cen, uint32_t n, float* out)
{
    __shared__ float sm[6][256];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float4 c = cen[i];
        v[0] = fminf(v[0], c.x); v[1] = fminf(v[1], c.y); v[2] = fminf(v[2], c.z);
        v[3] = fmaxf(v[3], c.x); v[4] = fmaxf(v[4], c.y); v[5] = fmaxf(v[5], c.z);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) sm[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] = fminf(sm[k][threadIdx.x], sm[k][threadIdx.x + h]);
#pragma unroll
            for (int k = 3; k < 6; ++k) sm[k][threadIdx.x] = fmaxf(sm[k][threadIdx.x], sm[k][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[blockIdx.x * 6 + threadIdx.x] = sm[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_cen_bounds_final(const float* partial, int nb, float* out)
{
    __shared__ float sm[6][256];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += 256) {
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] = fminf(v[k], partial[b * 6 + k]);
#pragma unroll
        for (int k = 3; k < 6; ++k) v[k] = fmaxf(v[k], partial[b * 6 + k]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) sm[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] = fminf(sm[k][threadIdx.x], sm[k][threadIdx.x + h]);
#pragma unroll
            for (int k = 3; k < 6; ++k) sm[k][threadIdx.x] = fmaxf(sm[k][threadIdx.x], sm[k][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = sm[threadIdx.x][0];
}

// spread the low 21 bits of x to every third bit of a 64-bit word
__device__ inline uint64_t spread21(uint64_t x)
{
    x &= 0x1FFFFFull;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// 63-bit Morton code of the centroid in the centroid bounds (21 bits per axis, x most significant)
__global__ __launch_bounds__(256) void k_morton(const float4* cen, uint32_t n, const float* bounds, uint64_t* keys,
                                                uint32_t* vals)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float4 c = cen[t];
    const float cc[3] = {c.x, c.y, c.z};
    uint64_t q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float ext = bounds[3 + k] - bounds[k];
        float u = ext > 0.0f ? (cc[k] - bounds[k]) / ext : 0.0f;
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        q[k] = (uint64_t)fminf(u * 2097152.0f, 2097151.0f);
    }
    keys[t] = (spread21(q[0]) << 2) | (spread21(q[1]) << 1) | spread21(q[2]);
    vals[t] = t;
}

// segment (body) of each primitive in Morton order, with its position
__global__ __launch_bounds__(256) void k_seg_gather(const uint32_t* seg, const uint32_t* order, uint32_t n,
                                                    uint32_t* seg_g, uint32_t* pos)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    seg_g[i] = seg[order[i]];
    pos[i] = i;
}

// apply the stable sort by segment: (segment, Morton) order
__global__ __launch_bounds__(256) void k_seg_apply(const uint32_t* perm, const uint64_t* keys_m, const uint32_t* order_m,
                                                   uint32_t n, uint64_t* keys, uint32_t* order)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = keys_m[perm[i]];
    order[i] = order_m[perm[i]];
}

// common prefix length of the sorted keys (segment, Morton code, position) at i and j; -1 outside
__device__ inline int delta(const uint32_t* seg, const uint64_t* k, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    if (seg) {
        const uint32_t sa = seg[i], sb = seg[j];
        if (sa != sb) return __clz(sa ^ sb);
    }
    const uint64_t a = k[i], b = k[j];
    if (a != b) return 32 + __clzll(a ^ b);
    return 96 + __clz((uint32_t)i ^ (uint32_t)j);
}

// internal node i of the radix tree: children (unified index) and the range of sorted positions it covers
__global__ __launch_bounds__(256) void k_radix_tree(const uint32_t* seg, const uint64_t* keys, int n, int2* child,
                                                    int2* range, int* parent)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (delta(seg, keys, n, i, i + 1) - delta(seg, keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta(seg, keys, n, i, i - d);
    int lmax = 2;
    while (delta(seg, keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(seg, keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = delta(seg, keys, n, i, j);
    int s = 0;
    for (int t = (l + 1) >> 1;; t = (t + 1) >> 1) {
        if (delta(seg, keys, n, i, i + (s + t) * d) > dnode) s += t;
        if (t == 1) break;
    }
    const int gamma = i + s * d + min(d, 0);
    const int first = min(i, j), last = max(i, j);
    const int left = first == gamma ? (n - 1 + gamma) : gamma;
    const int right = last == gamma + 1 ? (n - 1 + gamma + 1) : gamma + 1;
    child[i] = make_int2(left, right);
    range[i] = make_int2(first, last);
    parent[left] = i;
    parent[right] = i;
}

// root of each segment's subtree: the internal node whose range is the segment, or the segment's only leaf
__global__ __launch_bounds__(256) void k_seg_roots_internal(const int2* range, const uint32_t* seg_s, int n,
                                                            const uint32_t* seg_first, const uint32_t* seg_count,
                                                            int* roots)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int2 r = range[i];
    const uint32_t b = seg_s[r.x];
    if ((uint32_t)r.x == seg_first[b] && (uint32_t)r.y == seg_first[b] + seg_count[b] - 1u) roots[b] = i;
}

__global__ __launch_bounds__(256) void k_seg_roots_single(int n, const uint32_t* seg_first, const uint32_t* seg_count,
                                                          uint32_t n_seg, int* roots)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_seg) return;
    if (seg_count[b] == 1u) roots[b] = n - 1 + (int)seg_first[b];
}

// Box records shared between threads of different workgroups (and XCDs) during the bottom-up pass are
// written and read only with device-scope atomic stores and loads, which are coherent without cache
// maintenance; the writer waits for its stores to complete before it increments the arrival counter,
// and the reader loads only after its increment returned, so no device-wide fence is needed.
__device__ inline void box_store(Box6* p, const Box6& b)
{
    float* f = reinterpret_cast<float*>(p);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        __hip_atomic_store(f + k, b.lo[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(f + 3 + k, b.hi[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ inline Box6 box_load(const Box6* p)
{
    const float* f = reinterpret_cast<const float*>(p);
    Box6 b;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        b.lo[k] = __hip_atomic_load(f + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        b.hi[k] = __hip_atomic_load(f + 3 + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return b;
}

// boxes of all binary nodes: each leaf walks up; the second thread to reach a node computes its box
__global__ __launch_bounds__(256) void k_bottom_up(const Box6* prim_box, const uint32_t* vals, int n, const int2* child,
                                                   const int* parent, uint32_t* flags, Box6* box)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int node = n - 1 + i;
    Box6 u = prim_box[vals[i]];
    box_store(box + node, u);
    for (;;) {
        const int p = parent[node];
        if (p < 0) break;
        __builtin_amdgcn_s_waitcnt(0);   // this thread's box stores have completed
        if (__hip_atomic_fetch_add(&flags[p], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
            break;                       // the sibling's box is not ready: its thread continues
        const int2 c = child[p];
        const Box6 o = box_load(box + (c.x == node ? c.y : c.x));
#pragma unroll
        for (int k = 0; k < 3; ++k) { u.lo[k] = fminf(u.lo[k], o.lo[k]); u.hi[k] = fmaxf(u.hi[k], o.hi[k]); }
        box_store(box + p, u);
        node = p;
    }
}

struct TreeView {
    int n, max_leaf;
    const int2* child;
    const int2* range;
    const Box6* box;
    const uint32_t* leaf_id;   // when set (leaves of one primitive): leaf word holds leaf_id[position]
};

__device__ inline int node_size(const TreeView& T, int b) { return b >= T.n - 1 ? 1 : T.range[b].y - T.range[b].x + 1; }
__device__ inline bool openable(const TreeView& T, int b) { return b < T.n - 1 && node_size(T, b) > T.max_leaf; }
__device__ inline float box_area(const Box6& b)
{
    const float dx = b.hi[0] - b.lo[0], dy = b.hi[1] - b.lo[1], dz = b.hi[2] - b.lo[2];
    return dx * dy + dy * dz + dz * dx;
}

// children of the 4-wide node over binary node b: open the largest openable child until there are 4; a
// root that holds at most max_leaf primitives is the single leaf child of its node
__device__ inline int gather_kids(const TreeView& T, int b, int kids[4])
{
    if (!openable(T, b)) {
        kids[0] = b;
        return 1;
    }
    int cnt = 2;
    kids[0] = T.child[b].x;
    kids[1] = T.child[b].y;
    while (cnt < 4) {
        int pick = -1;
        float best = -1.0f;
        for (int k = 0; k < cnt; ++k) {
            if (!openable(T, kids[k])) continue;
            const float a = box_area(T.box[kids[k]]);
            if (a > best) { best = a; pick = k; }
        }
        if (pick < 0) break;
        const int2 c = T.child[kids[pick]];
        for (int k = cnt; k > pick + 1; --k) kids[k] = kids[k - 1];
        kids[pick] = c.x;
        kids[pick + 1] = c.y;
        ++cnt;
    }
    return cnt;
}

__device__ inline uint32_t leaf_word(const TreeView& T, int b)
{
    const int first = b >= T.n - 1 ? b - (T.n - 1) : T.range[b].x;
    if (T.leaf_id) return rc_make_leaf(T.leaf_id[first], 1u);
    return rc_make_leaf((uint32_t)first, (uint32_t)node_size(T, b));
}

__device__ inline int n_open_kids(const TreeView& T, int b, const int kids[4], int cnt)
{
    int ni = 0;
    for (int s = 0; s < cnt; ++s) ni += (kids[s] != b && openable(T, kids[s])) ? 1 : 0;
    return ni;
}

// One 4-wide node (index self) over binary node b; its internal children get the next level's slots
// slot0, slot0 + 1, ... (node index next_base + slot); slots at or beyond cap_next set *overflow.
__device__ inline void write_node(const TreeView& T, int b, const int kids[4], int cnt, uint32_t parent,
                                  uint32_t depth, uint32_t next_base, uint32_t slot0, uint32_t cap_next,
                                  int* next_level, uint32_t* next_parent, uint32_t self, Node4* out,
                                  uint32_t* overflow)
{
    Node4 nd;
    uint32_t j = 0;
    for (int s = 0; s < 4; ++s) {
        if (s >= cnt) {
            nd.lo_x[s] = nd.lo_y[s] = nd.lo_z[s] = INFINITY;
            nd.hi_x[s] = nd.hi_y[s] = nd.hi_z[s] = -INFINITY;
            nd.child[s] = RC_EMPTY_CHILD;
            continue;
        }
        const int c = kids[s];
        const Box6 bx = T.box[c];
        nd.lo_x[s] = bx.lo[0]; nd.hi_x[s] = bx.hi[0];
        nd.lo_y[s] = bx.lo[1]; nd.hi_y[s] = bx.hi[1];
        nd.lo_z[s] = bx.lo[2]; nd.hi_z[s] = bx.hi[2];
        if (c != b && openable(T, c)) {
            const uint32_t slot = slot0 + j++;
            nd.child[s] = next_base + slot;
            if (slot < cap_next) {
                next_level[slot] = c;
                next_parent[slot] = self;
            } else {
                atomicOr(overflow, 1u);
            }
        } else {
            nd.child[s] = leaf_word(T, c);
        }
    }
    nd.parent = parent;
    nd.level = depth;
    nd.pad[0] = nd.pad[1] = 0u;
    out[self] = nd;
}

__global__ __launch_bounds__(256) void k_collapse_count(TreeView T, const int* level, int m, int* n_internal)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    int kids[4];
    const int b = level[k];
    const int cnt = gather_kids(T, b, kids);
    n_internal[k] = n_open_kids(T, b, kids, cnt);
}

__global__ __launch_bounds__(256) void k_collapse_write(TreeView T, const int* level, const uint32_t* level_parent,
                                                        int m, const int* offs, uint32_t level_base, uint32_t next_base,
                                                        uint32_t depth, uint32_t cap, Node4* nodes,
                                                        int* next_level, uint32_t* next_parent, uint32_t* overflow)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    int kids[4];
    const int b = level[k];
    const int cnt = gather_kids(T, b, kids);
    const uint32_t cap_next = next_base < cap ? cap - next_base : 0u;
    write_node(T, b, kids, cnt, level_parent[k], depth, next_base, (uint32_t)offs[k], cap_next, next_level,
               next_parent, level_base + (uint32_t)k, nodes, overflow);
}

// The whole collapse from one root in one workgroup, level by level (small trees: no host round trip).
// Writes nodes base .. base + count - 1 with absolute child indices; info = {count, levels, error}.
constexpr int CB_THREADS = 1024;
__global__ __launch_bounds__(CB_THREADS) void k_collapse_block(TreeView T, int root, Node4* nodes, uint32_t base,
                                                               uint32_t cap, uint32_t max_levels, int* lvl_a,
                                                               int* lvl_b, uint32_t* par_a, uint32_t* par_b,
                                                               uint32_t* info, uint32_t* error_flag)
{
    __shared__ int s_wave[CB_THREADS / 64 + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        lvl_a[0] = root;
        par_a[0] = 0xFFFFFFFFu;
        info[2] = 0u;
    }
    __syncthreads();
    uint32_t m = 1, level_base = 0, depth = 0;
    int* cur = lvl_a;
    int* nxt = lvl_b;
    uint32_t* pc = par_a;
    uint32_t* pn = par_b;
    bool failed = false;
    while (m > 0) {
        if (depth >= max_levels || level_base + m > cap) { failed = true; break; }
        const uint32_t next_base = level_base + m;
        const uint32_t cap_next = cap - next_base;
        uint32_t next_m = 0;
        for (uint32_t c0 = 0; c0 < m; c0 += CB_THREADS) {
            const uint32_t k = c0 + (uint32_t)tid;
            int kids[4] = {0, 0, 0, 0}, cnt = 0, ni = 0, b = 0;
            if (k < m) {
                b = cur[k];
                cnt = gather_kids(T, b, kids);
                ni = n_open_kids(T, b, kids, cnt);
            }
            int x = ni;   // inclusive scan over the wave, then over the wave totals
            for (int off = 1; off < 64; off <<= 1) {
                const int y = __shfl_up(x, off);
                if (lane >= off) x += y;
            }
            if (lane == 63) s_wave[wave] = x;
            __syncthreads();
            if (tid == 0) {
                int acc = 0;
                for (int w = 0; w < CB_THREADS / 64; ++w) { const int t = s_wave[w]; s_wave[w] = acc; acc += t; }
                s_wave[CB_THREADS / 64] = acc;
            }
            __syncthreads();
            const uint32_t off = next_m + (uint32_t)(s_wave[wave] + x - ni);
            if (k < m)
                write_node(T, b, kids, cnt, pc[k], depth, base + next_base, off, cap_next, nxt, pn,
                           base + level_base + k, nodes, info + 2);
            next_m += (uint32_t)s_wave[CB_THREADS / 64];
            __syncthreads();
        }
        if (__hip_atomic_load(info + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) { failed = true; break; }
        level_base = next_base;
        ++depth;
        m = next_m;
        int* t = cur; cur = nxt; nxt = t;
        uint32_t* tp = pc; pc = pn; pn = tp;
    }
    __syncthreads();
    if (tid == 0) {
        info[0] = failed ? 1u : level_base;
        info[1] = depth;
        if (failed) {
            info[2] = 1u;
            *error_flag = 1u;
            // an empty root, so that traversal finds nothing
            Node4 nd;
            for (int s = 0; s < 4; ++s) {
                nd.lo_x[s] = nd.lo_y[s] = nd.lo_z[s] = INFINITY;
                nd.hi_x[s] = nd.hi_y[s] = nd.hi_z[s] = -INFINITY;
                nd.child[s] = RC_EMPTY_CHILD;
            }
            nd.parent = 0xFFFFFFFFu;
            nd.level = 0;
            nd.pad[0] = nd.pad[1] = 0u;
            nodes[base] = nd;
        }
    }
}

__global__ void k_fill_i32(int* p, int v, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned nb(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

template <class T>
struct DevBuf {
    T* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    hipError_t alloc(size_t n) { return hipMalloc(reinterpret_cast<void**>(&p), (n ? n : 1) * sizeof(T)); }
};

#define BH(call)                                  \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) return e_;          \
    } while (0)

}  // namespace

// Build the 4-wide BVH(s) of n triangles (n >= 1) on the device.  Without segments: one tree (root node 0).
// With segments (d_seg[t] = segment of triangle t; segment b = the triangles seg_first[b] .. seg_first[b] +
// seg_count[b] - 1, consecutive and covering 0 .. n-1 in order): one tree per segment, roots 0 .. n_seg-1,
// leaves only over the segment's own triangles.  On success *d_nodes_out (device, allocated here with
// hipMalloc, owned by the caller afterwards) holds *n_nodes_out nodes in breadth-first level order, d_order
// (device, n entries, caller-allocated) maps leaf slots to original triangle ids, and level_start receives
// the first node of every level followed by the node count.  Synchronises the stream before returning.
hipError_t rc_build_bvh_device(const float* d_pos, const uint32_t* d_idx, uint32_t n, uint32_t max_leaf,
                               const uint32_t* d_seg, const std::vector<uint32_t>& seg_first,
                               const std::vector<uint32_t>& seg_count, Node4** d_nodes_out, uint32_t* n_nodes_out,
                               uint32_t* d_order, std::vector<uint32_t>& level_start, hipStream_t st)
{
    *d_nodes_out = nullptr;
    *n_nodes_out = 0;
    level_start.clear();
    if (n == 0 || n > (1u << 28) || max_leaf < 1 || max_leaf > 4) return hipErrorInvalidValue;
    const bool segmented = d_seg != nullptr;
    const uint32_t n_seg = segmented ? (uint32_t)seg_first.size() : 1u;
    if (segmented && (n_seg == 0 || seg_count.size() != n_seg)) return hipErrorInvalidValue;
    const int N = (int)n;
    // 4-wide nodes: each non-root node consumes at least one binary node of more than max_leaf triangles,
    // and those that consume only one have two leaf children over disjoint triangle ranges of size >= 2, so
    // there are at most (n - 1 + n / 2) / 2 < 3n / 4 of them, plus one root per segment.
    const size_t cap = 3 * (size_t)n / 4 + n_seg + 2;
    const int red_blocks = 1024;
    DevBuf<Box6> tri_box, box;
    DevBuf<float4> cen;
    DevBuf<float> partial, bounds;
    DevBuf<uint64_t> keys, keys_s, keys_m;
    DevBuf<uint32_t> vals, flags, par_a, par_b, overflow, order_m, seg_g, seg_s, pos, perm, seg_first_d,
        seg_count_d;
    DevBuf<int2> child, range;
    DevBuf<int> parent, lvl_a, lvl_b, nint, offs;
    DevBuf<Node4> nodes;
    DevBuf<uint8_t> temp;
    BH(tri_box.alloc(n));
    BH(cen.alloc(n));
    BH(partial.alloc((size_t)red_blocks * 6));
    BH(bounds.alloc(6));
    BH(keys.alloc(n));
    BH(keys_s.alloc(n));
    BH(vals.alloc(n));
    BH(box.alloc(2 * (size_t)n));
    BH(child.alloc(n));
    BH(range.alloc(n));
    BH(parent.alloc(2 * (size_t)n));
    BH(flags.alloc(n));
    BH(nodes.alloc(cap));
    BH(lvl_a.alloc(cap));
    BH(lvl_b.alloc(cap));
    BH(par_a.alloc(cap));
    BH(par_b.alloc(cap));
    BH(nint.alloc(cap));
    BH(offs.alloc(cap));
    BH(overflow.alloc(1));
    if (segmented) {
        BH(keys_m.alloc(n));
        BH(order_m.alloc(n));
        BH(seg_g.alloc(n));
        BH(seg_s.alloc(n));
        BH(pos.alloc(n));
        BH(perm.alloc(n));
        BH(seg_first_d.alloc(n_seg));
        BH(seg_count_d.alloc(n_seg));
    }
    size_t sort_bytes = 0, seg_sort_bytes = 0, scan_bytes = 0;
    BH(rocprim::radix_sort_pairs(nullptr, sort_bytes, keys.p, keys_s.p, vals.p, d_order, n, 0, 63, st));
    if (segmented)
        BH(rocprim::radix_sort_pairs(nullptr, seg_sort_bytes, seg_g.p, seg_s.p, pos.p, perm.p, n, 0, 32, st));
    BH(rocprim::exclusive_scan(nullptr, scan_bytes, nint.p, offs.p, 0, cap, rocprim::plus<int>(), st));
    BH(temp.alloc(std::max(std::max(sort_bytes, seg_sort_bytes), scan_bytes)));

    hipLaunchKernelGGL(k_tri_boxes, dim3(nb(n, 256)), dim3(256), 0, st, d_pos, d_idx, n, tri_box.p, cen.p);
    hipLaunchKernelGGL(k_cen_bounds, dim3(red_blocks), dim3(256), 0, st, cen.p, n, partial.p);
    hipLaunchKernelGGL(k_cen_bounds_final, dim3(1), dim3(256), 0, st, partial.p, red_blocks, bounds.p);
    hipLaunchKernelGGL(k_morton, dim3(nb(n, 256)), dim3(256), 0, st, cen.p, n, bounds.p, keys.p, vals.p);
    BH(hipGetLastError());
    if (!segmented) {
        BH(rocprim::radix_sort_pairs(temp.p, sort_bytes, keys.p, keys_s.p, vals.p, d_order, n, 0, 63, st));
    } else {
        BH(rocprim::radix_sort_pairs(temp.p, sort_bytes, keys.p, keys_m.p, vals.p, order_m.p, n, 0, 63, st));
        hipLaunchKernelGGL(k_seg_gather, dim3(nb(n, 256)), dim3(256), 0, st, d_seg, order_m.p, n, seg_g.p, pos.p);
        BH(rocprim::radix_sort_pairs(temp.p, seg_sort_bytes, seg_g.p, seg_s.p, pos.p, perm.p, n, 0, 32, st));
        hipLaunchKernelGGL(k_seg_apply, dim3(nb(n, 256)), dim3(256), 0, st, perm.p, keys_m.p, order_m.p, n, keys_s.p,
                           d_order);
        BH(hipMemcpyAsync(seg_first_d.p, seg_first.data(), n_seg * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        BH(hipMemcpyAsync(seg_count_d.p, seg_count.data(), n_seg * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    }
    hipLaunchKernelGGL(k_fill_i32, dim3(nb(2 * (size_t)n, 256)), dim3(256), 0, st, parent.p, -1, 2 * n);
    hipLaunchKernelGGL(k_fill_i32, dim3(nb(n, 256)), dim3(256), 0, st, reinterpret_cast<int*>(flags.p), 0, n);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, reinterpret_cast<int*>(overflow.p), 0, 1u);
    if (N > 1)
        hipLaunchKernelGGL(k_radix_tree, dim3(nb(n - 1, 256)), dim3(256), 0, st, segmented ? seg_s.p : nullptr,
                           keys_s.p, N, child.p, range.p, parent.p);
    hipLaunchKernelGGL(k_bottom_up, dim3(nb(n, 256)), dim3(256), 0, st, tri_box.p, d_order, N, child.p, parent.p,
                       flags.p, box.p);
    // level 0: the roots (one tree: internal node 0, or for n = 1 the only leaf, whose index n - 1 is also 0)
    hipLaunchKernelGGL(k_fill_i32, dim3(nb(n_seg, 256)), dim3(256), 0, st, lvl_a.p, 0, n_seg);
    hipLaunchKernelGGL(k_fill_i32, dim3(nb(n_seg, 256)), dim3(256), 0, st, reinterpret_cast<int*>(par_a.p), -1,
                       n_seg);
    if (segmented) {
        if (N > 1)
            hipLaunchKernelGGL(k_seg_roots_internal, dim3(nb(n - 1, 256)), dim3(256), 0, st, range.p, seg_s.p, N,
                               seg_first_d.p, seg_count_d.p, lvl_a.p);
        hipLaunchKernelGGL(k_seg_roots_single, dim3(nb(n_seg, 256)), dim3(256), 0, st, N, seg_first_d.p,
                           seg_count_d.p, n_seg, lvl_a.p);
    }
    BH(hipGetLastError());
    const TreeView T{N, (int)max_leaf, child.p, range.p, box.p, nullptr};
    uint32_t m = n_seg, base = 0, depth = 0;
    while (m > 0) {
        if ((size_t)base + m > cap) return hipErrorUnknown;   // excluded by the bound on cap
        hipLaunchKernelGGL(k_collapse_count, dim3(nb(m, 256)), dim3(256), 0, st, T, lvl_a.p, (int)m, nint.p);
        size_t sb = scan_bytes;
        BH(rocprim::exclusive_scan(temp.p, sb, nint.p, offs.p, 0, (size_t)m, rocprim::plus<int>(), st));
        hipLaunchKernelGGL(k_collapse_write, dim3(nb(m, 256)), dim3(256), 0, st, T, lvl_a.p, par_a.p, (int)m, offs.p,
                           base, base + m, depth, (uint32_t)cap, nodes.p, lvl_b.p, par_b.p, overflow.p);
        BH(hipGetLastError());
        int tail[2] = {0, 0};
        uint32_t ovf = 0;
        BH(hipMemcpyAsync(&tail[0], offs.p + (m - 1), sizeof(int), hipMemcpyDeviceToHost, st));
        BH(hipMemcpyAsync(&tail[1], nint.p + (m - 1), sizeof(int), hipMemcpyDeviceToHost, st));
        BH(hipMemcpyAsync(&ovf, overflow.p, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        BH(hipStreamSynchronize(st));
        if (ovf) return hipErrorUnknown;
        level_start.push_back(base);
        base += m;
        ++depth;
        m = (uint32_t)(tail[0] + tail[1]);
        std::swap(lvl_a.p, lvl_b.p);
        std::swap(par_a.p, par_b.p);
    }
    level_start.push_back(base);
    const uint32_t total = level_start.back();
    Node4* out = nullptr;
    BH(hipMalloc(reinterpret_cast<void**>(&out), (size_t)total * sizeof(Node4)));
    hipError_t e = hipMemcpyAsync(out, nodes.p, (size_t)total * sizeof(Node4), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(out);
        return e;
    }
    *d_nodes_out = out;
    *n_nodes_out = total;
    return hipSuccess;
}

// ---------------------------------------------------------------- top level --------
hipError_t rc_tlas_alloc(TlasWork& w, uint32_t n)
{
    rc_tlas_free(w);
    if (n == 0) return hipErrorInvalidValue;
    w.n = n;
    w.cap = 3 * n / 4 + 3;
    auto A = [](void** p, size_t bytes) { return hipMalloc(p, bytes ? bytes : 1); };
    BH(A(&w.box, (size_t)n * sizeof(Box6)));
    BH(A(&w.cen, (size_t)n * sizeof(float4)));
    BH(A(&w.partial, (size_t)64 * 6 * sizeof(float)));
    BH(A(&w.bounds, 6 * sizeof(float)));
    BH(A(&w.keys, (size_t)n * 8));
    BH(A(&w.keys_s, (size_t)n * 8));
    BH(A(&w.vals, (size_t)n * 4));
    BH(A(&w.order, (size_t)n * 4));
    BH(A(&w.flags, (size_t)n * 4));
    BH(A(&w.child, (size_t)n * sizeof(int2)));
    BH(A(&w.range, (size_t)n * sizeof(int2)));
    BH(A(&w.parent, (size_t)2 * n * 4));
    BH(A(&w.nbox, (size_t)2 * n * sizeof(Box6)));
    BH(A(&w.lvl, (size_t)4 * w.cap * 4));
    BH(A(&w.info, 4 * sizeof(uint32_t)));
    size_t bytes = 0;
    BH(rocprim::radix_sort_pairs(nullptr, bytes, (uint64_t*)w.keys, (uint64_t*)w.keys_s, (uint32_t*)w.vals,
                                 (uint32_t*)w.order, n, 0, 63, (hipStream_t)0));
    w.temp_bytes = bytes;
    BH(A(&w.temp, bytes));
    return hipSuccess;
}

void rc_tlas_free(TlasWork& w)
{
    void** ptrs[] = {&w.box, &w.cen, &w.partial, &w.bounds, &w.keys, &w.keys_s, &w.vals, &w.order, &w.flags,
                     &w.child, &w.range, &w.parent, &w.nbox, &w.lvl, &w.info, &w.temp};
    for (void** p : ptrs) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    w.n = w.cap = 0;
    w.temp_bytes = 0;
}

// Rebuild the top level over w.n instances on stream st from their object-to-world maps o2w (12 floats per
// instance) and the bottom-level roots (nodes 0 .. w.n - 1): instance records (inst), then the top-level
// nodes tlas_base .. tlas_base + count - 1 of `nodes` (root at tlas_base; leaf words hold instance ids).
// No allocation and no host synchronisation.  A top level deeper than max_levels (or larger than the
// workspace) leaves an empty root and sets *error_flag.
hipError_t rc_tlas_build(TlasWork& w, const float* o2w, Node4* nodes, uint32_t tlas_base, DevInst* inst,
                         uint32_t max_levels, uint32_t* error_flag, hipStream_t st)
{
    const uint32_t n = w.n;
    if (n == 0) return hipErrorInvalidValue;
    Box6* box = (Box6*)w.box;
    float4* cen = (float4*)w.cen;
    const int red_blocks = (int)std::min<uint32_t>(64, nb(n, 256));
    hipLaunchKernelGGL(k_instances, dim3(nb(n, 256)), dim3(256), 0, st, o2w, nodes, n, inst, box, cen);
    hipLaunchKernelGGL(k_cen_bounds, dim3(red_blocks), dim3(256), 0, st, cen, n, (float*)w.partial);
    hipLaunchKernelGGL(k_cen_bounds_final, dim3(1), dim3(256), 0, st, (const float*)w.partial, red_blocks,
                       (float*)w.bounds);
    hipLaunchKernelGGL(k_morton, dim3(nb(n, 256)), dim3(256), 0, st, cen, n, (const float*)w.bounds,
                       (uint64_t*)w.keys, (uint32_t*)w.vals);
    size_t bytes = w.temp_bytes;
    BH(rocprim::radix_sort_pairs(w.temp, bytes, (uint64_t*)w.keys, (uint64_t*)w.keys_s, (uint32_t*)w.vals,
                                 (uint32_t*)w.order, n, 0, 63, st));
    hipLaunchKernelGGL(k_fill_i32, dim3(nb(2 * (size_t)n, 256)), dim3(256), 0, st, (int*)w.parent, -1, 2 * n);
    hipLaunchKernelGGL(k_fill_i32, dim3(nb(n, 256)), dim3(256), 0, st, (int*)w.flags, 0, n);
    const int N = (int)n;
    if (N > 1)
        hipLaunchKernelGGL(k_radix_tree, dim3(nb(n - 1, 256)), dim3(256), 0, st, nullptr, (const uint64_t*)w.keys_s,
                           N, (int2*)w.child, (int2*)w.range, (int*)w.parent);
    hipLaunchKernelGGL(k_bottom_up, dim3(nb(n, 256)), dim3(256), 0, st, box, (const uint32_t*)w.order, N,
                       (const int2*)w.child, (const int*)w.parent, (uint32_t*)w.flags, (Box6*)w.nbox);
    const TreeView T{N, 1, (const int2*)w.child, (const int2*)w.range, (const Box6*)w.nbox,
                     (const uint32_t*)w.order};
    int* lvl = (int*)w.lvl;
    hipLaunchKernelGGL(k_collapse_block, dim3(1), dim3(CB_THREADS), 0, st, T, 0, nodes, tlas_base, w.cap, max_levels,
                       lvl, lvl + w.cap, (uint32_t*)(lvl + 2 * w.cap), (uint32_t*)(lvl + 3 * w.cap),
                       (uint32_t*)w.info, error_flag);
    return hipGetLastError();
}
