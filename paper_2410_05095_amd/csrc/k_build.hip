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

// A binary tree to collapse.  Radix trees (explicit = 0): internal nodes 0 .. n-2 with inclusive primitive ranges,
// leaves n-1 .. 2n-2 of one primitive each; a subtree of at most max_leaf primitives becomes one leaf.  Explicit
// trees (explicit = 1, the binned-SAH build): node b is a leaf when child[b].x < 0, with range[b] = (first slot,
// count); every other node is opened.
struct TreeView {
    int n, max_leaf;
    const int2* child;
    const int2* range;
    const Box6* box;
    const uint32_t* leaf_id;   // when set (leaves of one primitive): leaf word holds leaf_id[position]
    int explicit_leaves = 0;
};

__device__ inline int node_size(const TreeView& T, int b) { return b >= T.n - 1 ? 1 : T.range[b].y - T.range[b].x + 1; }
__device__ inline bool openable(const TreeView& T, int b)
{
    if (T.explicit_leaves) return T.child[b].x >= 0;
    return b < T.n - 1 && node_size(T, b) > T.max_leaf;
}
// half the surface area, in FP64 from the FP32 box (as the host builder's collapse compares it)
__device__ inline double box_area(const Box6& b)
{
    const double dx = (double)b.hi[0] - b.lo[0], dy = (double)b.hi[1] - b.lo[1], dz = (double)b.hi[2] - b.lo[2];
    if (!(dx >= 0.0) || !(dy >= 0.0) || !(dz >= 0.0)) return 0.0;
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
        double best = -1.0;
        for (int k = 0; k < cnt; ++k) {
            if (!openable(T, kids[k])) continue;
            const double a = box_area(T.box[kids[k]]);
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
    if (T.explicit_leaves) return rc_make_leaf((uint32_t)T.range[b].x, (uint32_t)T.range[b].y);
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

// Sort of up to SORT_BLOCK_MAX (key, value) pairs in one workgroup, bitonic in LDS, by (key, value): with
// distinct values given in increasing order (instance ids) this is the order a stable sort by key gives.  The
// per-frame top level sorts its ~1500 instance keys with it in one launch.
constexpr uint32_t SORT_BLOCK_MAX = 4096;
constexpr int SORT_THREADS = 1024;

__global__ __launch_bounds__(SORT_THREADS) void k_sort_block(const uint64_t* keys, const uint32_t* vals, uint32_t n,
                                                             uint64_t* keys_out, uint32_t* vals_out)
{
    __shared__ uint64_t K[SORT_BLOCK_MAX];
    __shared__ uint32_t V[SORT_BLOCK_MAX];
    uint32_t m = 64;
    while (m < n) m <<= 1;
    for (uint32_t i = threadIdx.x; i < m; i += SORT_THREADS) {
        K[i] = i < n ? keys[i] : ~0ull;
        V[i] = i < n ? vals[i] : ~0u;
    }
    __syncthreads();
    // Each step compares the m / 2 pairs (i, i + j), i with bit j clear, one pair per thread and iteration: pair
    // t has i = t with a zero bit inserted at j's position.  For j < 64 the 64 pairs of a wave lie in one block
    // of 128 elements that no other wave touches, so such steps need no workgroup barrier between them: the
    // wave's own LDS accesses complete in order.
    for (uint32_t k = 2; k <= m; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t t = threadIdx.x; t < m / 2; t += SORT_THREADS) {
                const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const uint32_t l = i | j;
                const uint64_t ka = K[i], kb = K[l];
                const uint32_t va = V[i], vb = V[l];
                const bool greater = ka > kb || (ka == kb && va > vb);
                if (greater == ((i & k) == 0)) {   // ascending runs where bit k of i is clear
                    K[i] = kb; K[l] = ka;
                    V[i] = vb; V[l] = va;
                }
            }
            const bool next_in_wave = (j >> 1) > 0 ? (j >> 1) < 64 : (k << 1) <= 64;
            if (next_in_wave && j < 64) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else {
                __syncthreads();
            }
        }
    }
    for (uint32_t i = threadIdx.x; i < n; i += SORT_THREADS) {
        keys_out[i] = K[i];
        vals_out[i] = V[i];
    }
}

__global__ void k_iota(uint32_t* p, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
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

// ---------------------------------------------------------------- binned SAH on the GPU --------
// The host builder's algorithm (binned SAH over triangle centroids, `bins` bins per axis, node cost relative to
// a triangle test, leaves of at most max_leaf triangles) with the same arithmetic, so that it chooses the same
// splits: bin k = (int)(((double)c - lo) * (bins / (double)(hi - lo))) clamped to [0, bins - 1] per axis with a
// positive centroid extent; cost of a split before bin k = area(left) n_left + area(right) n_right in FP64 from
// the exact FP32 union boxes, the first minimum over (axis, k) in order; a range of n <= max_leaf triangles
// stays a leaf when no split exists or n <= node_cost + best / area(node); a range whose centroids coincide is
// halved.  Ranges above SAH_SMALL triangles are split level by level, every workgroup binning a chunk of one
// range; each smaller range is then built to the leaves by one wave.  Partitions are stable, so the build is
// deterministic.  The binary tree is collapsed to 4-wide like the radix trees (explicit leaves).
namespace {

constexpr int SAH_NB_MAX = 64;
constexpr uint32_t SAH_SMALL = 1024;
constexpr uint32_t SAH_CHUNK = 8192;
constexpr int SAH_BIN_WORDS = 8;   // ordered lo[3], hi[3], count, pad

__device__ inline uint32_t f2o(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float o2f(uint32_t o) { return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o); }
constexpr uint32_t O_POS_INF = 0xFF800000u;   // f2o(+inf)
constexpr uint32_t O_NEG_INF = 0x007FFFFFu;   // f2o(-inf)

// surface area 2 (dx dy + dy dz + dz dx) in FP64, 0 for an empty or inverted box (the host builder's)
__device__ inline double sah_area(const float lo[3], const float hi[3])
{
    const double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
    if (!(dx >= 0.0) || !(dy >= 0.0) || !(dz >= 0.0)) return 0.0;
    return 2.0 * (dx * dy + dy * dz + dz * dx);
}

__device__ inline int sah_bin(float c, float lo, double scale, int NB)
{
    int k = (int)(((double)c - (double)lo) * scale);
    return min(max(k, 0), NB - 1);
}

struct SahTask {
    uint32_t node, first, count, pad;
};

struct SahTree {
    int2* child;     // (left, right), or (-1, -1) for a leaf
    int2* range;     // (first slot, count)
    Box6* box;
    uint32_t* node_ctr;
};

// The split decision of one range, by one wave: from the bins of the three axes (box as ordered words, count)
// and the node box; returns best axis (-1: none), the first bin of the right side, and the left count.  Lanes
// k < NB hold bin k of the axis being swept.
__device__ inline void sah_decide(const uint32_t* bins /* [3][NB][SAH_BIN_WORDS] */, int NB, const float clo[3],
                                  const float chi[3], int& best_axis, int& best_split, uint32_t& best_nl,
                                  double& best_cost)
{
    const int lane = (int)__lane_id();
    double bc = INFINITY;
    int bidx = 0x7FFFFFFF;
    uint32_t bnl = 0;
    for (int axis = 0; axis < 3; ++axis) {
        const float ext = chi[axis] - clo[axis];
        if (!(ext > 0.0f)) continue;
        float lo[3], hi[3];
        uint32_t cnt = 0;
        if (lane < NB) {
            const uint32_t* b = bins + ((size_t)axis * NB + lane) * SAH_BIN_WORDS;
            for (int k = 0; k < 3; ++k) { lo[k] = o2f(b[k]); hi[k] = o2f(b[3 + k]); }
            cnt = b[6];
        } else {
            for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
        }
        // inclusive prefix (lanes 0..k) and suffix (lanes k..NB-1) unions and counts
        float plo[3], phi[3], slo[3], shi[3];
        uint32_t pc = cnt, sc = cnt;
        for (int k = 0; k < 3; ++k) { plo[k] = slo[k] = lo[k]; phi[k] = shi[k] = hi[k]; }
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t pcu = __shfl_up(pc, off), scd = __shfl_down(sc, off);
            float u[6], d[6];
            for (int k = 0; k < 3; ++k) {
                u[k] = __shfl_up(plo[k], off); u[3 + k] = __shfl_up(phi[k], off);
                d[k] = __shfl_down(slo[k], off); d[3 + k] = __shfl_down(shi[k], off);
            }
            if (lane >= off) {
                pc += pcu;
                for (int k = 0; k < 3; ++k) { plo[k] = fminf(plo[k], u[k]); phi[k] = fmaxf(phi[k], u[3 + k]); }
            }
            if (lane + off < 64) {
                sc += scd;
                for (int k = 0; k < 3; ++k) { slo[k] = fminf(slo[k], d[k]); shi[k] = fmaxf(shi[k], d[3 + k]); }
            }
        }
        // split before bin lane + 1: left = prefix of lane, right = suffix of lane + 1
        float rlo[3], rhi[3];
        for (int k = 0; k < 3; ++k) { rlo[k] = __shfl_down(slo[k], 1); rhi[k] = __shfl_down(shi[k], 1); }
        const uint32_t rc = __shfl_down(sc, 1);
        if (lane < NB - 1 && pc > 0 && rc > 0) {
            const double cost = sah_area(plo, phi) * (double)pc + sah_area(rlo, rhi) * (double)rc;
            const int idx = axis * NB + lane + 1;
            if (cost < bc) { bc = cost; bidx = idx; bnl = pc; }
        }
    }
    // first minimum over (axis, split) in order
    for (int off = 32; off > 0; off >>= 1) {
        const double oc = __shfl_xor(bc, off);
        const int oi = __shfl_xor(bidx, off);
        const uint32_t on = __shfl_xor(bnl, off);
        if (oc < bc || (oc == bc && oi < bidx)) { bc = oc; bidx = oi; bnl = on; }
    }
    best_cost = bc;
    if (bidx == 0x7FFFFFFF) {
        best_axis = -1;
        best_split = 0;
        best_nl = 0;
    } else {
        best_axis = bidx / NB;
        best_split = bidx % NB;
        best_nl = bnl;
    }
}

__device__ inline void write_sah_node(const SahTree& T, uint32_t node, const float lo[3], const float hi[3], int left,
                                      int right, uint32_t first, uint32_t count)
{
    Box6 b;
    for (int k = 0; k < 3; ++k) { b.lo[k] = lo[k]; b.hi[k] = hi[k]; }
    T.box[node] = b;
    T.child[node] = make_int2(left, right);
    T.range[node] = make_int2((int)first, (int)count);
}

// ---- large ranges, level by level (chunk c of the level: elements chunk_begin[c] .. chunk_end[c] - 1 of task
// chunk_task[c]) ----
__global__ __launch_bounds__(256) void k_sah_reset(uint32_t* acc, uint32_t* bins, uint32_t n_tasks, int NB)
{
    const size_t per_task = 12 + (size_t)3 * NB * SAH_BIN_WORDS;
    const size_t total = per_task * n_tasks;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
        const size_t t = i / per_task, w = i % per_task;
        uint32_t v;
        if (w < 12) {
            v = (w % 6) < 3 ? O_POS_INF : O_NEG_INF;   // box lo, box hi, centroid lo, centroid hi
            acc[t * 12 + w] = v;
        } else {
            const size_t q = w - 12, word = q % SAH_BIN_WORDS;
            v = word < 3 ? O_POS_INF : (word < 6 ? O_NEG_INF : 0u);
            bins[t * (per_task - 12) + q] = v;
        }
    }
}

__device__ inline void block_reduce_minmax(float v[12], float* sm /* [12][4] */)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1)
        for (int k = 0; k < 12; ++k) {
            const float o = __shfl_xor(v[k], off);
            v[k] = (k % 6) < 3 ? fminf(v[k], o) : fmaxf(v[k], o);
        }
    if (lane == 0)
        for (int k = 0; k < 12; ++k) sm[k * 4 + wave] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 12; ++k)
            for (int w = 1; w < 4; ++w) v[k] = (k % 6) < 3 ? fminf(v[k], sm[k * 4 + w]) : fmaxf(v[k], sm[k * 4 + w]);
}

__global__ __launch_bounds__(256) void k_sah_bounds(const uint32_t* ids, const Box6* tri_box, const float4* cen,
                                                    const uint32_t* chunk_task, const uint32_t* chunk_begin,
                                                    const uint32_t* chunk_end, uint32_t* acc)
{
    __shared__ float sm[48];
    const uint32_t c = blockIdx.x;
    float v[12];
    for (int k = 0; k < 12; ++k) v[k] = (k % 6) < 3 ? INFINITY : -INFINITY;
    for (uint32_t i = chunk_begin[c] + threadIdx.x; i < chunk_end[c]; i += 256) {
        const uint32_t t = ids[i];
        const Box6 b = tri_box[t];
        const float4 q = cen[t];
        const float cc[3] = {q.x, q.y, q.z};
        for (int k = 0; k < 3; ++k) {
            v[k] = fminf(v[k], b.lo[k]); v[3 + k] = fmaxf(v[3 + k], b.hi[k]);
            v[6 + k] = fminf(v[6 + k], cc[k]); v[9 + k] = fmaxf(v[9 + k], cc[k]);
        }
    }
    block_reduce_minmax(v, sm);
    if (threadIdx.x == 0) {
        uint32_t* a = acc + 12 * (size_t)chunk_task[c];
        for (int k = 0; k < 12; ++k) {
            if ((k % 6) < 3) atomicMin(a + k, f2o(v[k]));
            else atomicMax(a + k, f2o(v[k]));
        }
    }
}

__global__ __launch_bounds__(256) void k_sah_bins(const uint32_t* ids, const Box6* tri_box, const float4* cen,
                                                  const uint32_t* chunk_task, const uint32_t* chunk_begin,
                                                  const uint32_t* chunk_end, const uint32_t* acc, uint32_t* bins,
                                                  int NB)
{
    __shared__ uint32_t lb[3 * SAH_NB_MAX * SAH_BIN_WORDS];
    const uint32_t c = blockIdx.x, task = chunk_task[c];
    const int words = 3 * NB * SAH_BIN_WORDS;
    for (int i = threadIdx.x; i < words; i += 256) {
        const int w = i % SAH_BIN_WORDS;
        lb[i] = w < 3 ? O_POS_INF : (w < 6 ? O_NEG_INF : 0u);
    }
    const uint32_t* a = acc + 12 * (size_t)task;
    float clo[3], chi[3];
    for (int k = 0; k < 3; ++k) { clo[k] = o2f(a[6 + k]); chi[k] = o2f(a[9 + k]); }
    __syncthreads();
    for (uint32_t i = chunk_begin[c] + threadIdx.x; i < chunk_end[c]; i += 256) {
        const uint32_t t = ids[i];
        const Box6 b = tri_box[t];
        const float4 q = cen[t];
        const float cc[3] = {q.x, q.y, q.z};
        for (int axis = 0; axis < 3; ++axis) {
            const float ext = chi[axis] - clo[axis];
            if (!(ext > 0.0f)) continue;
            const int k = sah_bin(cc[axis], clo[axis], (double)NB / (double)ext, NB);
            uint32_t* w = lb + ((size_t)axis * NB + k) * SAH_BIN_WORDS;
            for (int j = 0; j < 3; ++j) { atomicMin(w + j, f2o(b.lo[j])); atomicMax(w + 3 + j, f2o(b.hi[j])); }
            atomicAdd(w + 6, 1u);
        }
    }
    __syncthreads();
    uint32_t* g = bins + (size_t)task * 3 * NB * SAH_BIN_WORDS;
    for (int i = threadIdx.x; i < words; i += 256) {
        const int w = i % SAH_BIN_WORDS;
        if (lb[i - w + 6] == 0u || w == 7) continue;   // empty bin
        if (w < 3) atomicMin(g + i, lb[i]);
        else if (w < 6) atomicMax(g + i, lb[i]);
        else atomicAdd(g + i, lb[i]);
    }
}

// One wave per large range: split it (it holds more than SAH_SMALL >= max_leaf triangles, so it is never a
// leaf), write its node, and queue its halves as large or small ranges.  decision[t] = (axis or -1, split bin,
// left count).
__global__ __launch_bounds__(64) void k_sah_split(const SahTask* tasks, const uint32_t* acc, const uint32_t* bins,
                                                  int NB, SahTree T, SahTask* big_next, uint32_t* big_next_n,
                                                  SahTask* small, uint32_t* small_n, int4* decision)
{
    const uint32_t t = blockIdx.x;
    const SahTask task = tasks[t];
    const uint32_t* a = acc + 12 * (size_t)t;
    float blo[3], bhi[3], clo[3], chi[3];
    for (int k = 0; k < 3; ++k) {
        blo[k] = o2f(a[k]); bhi[k] = o2f(a[3 + k]); clo[k] = o2f(a[6 + k]); chi[k] = o2f(a[9 + k]);
    }
    int axis, split;
    uint32_t nl;
    double cost;
    sah_decide(bins + (size_t)t * 3 * NB * SAH_BIN_WORDS, NB, clo, chi, axis, split, nl, cost);
    if (axis < 0) nl = task.count / 2;
    if (__lane_id() == 0) {
        const uint32_t l = atomicAdd(T.node_ctr, 2u), r = l + 1;
        write_sah_node(T, task.node, blo, bhi, (int)l, (int)r, task.first, task.count);
        const SahTask kids[2] = {{l, task.first, nl, 0u}, {r, task.first + nl, task.count - nl, 0u}};
        for (int s = 0; s < 2; ++s) {
            if (kids[s].count > SAH_SMALL) big_next[atomicAdd(big_next_n, 1u)] = kids[s];
            else small[atomicAdd(small_n, 1u)] = kids[s];
        }
        decision[t] = make_int4(axis, split, (int)nl, 0);
    }
}

// stable partition of the large ranges: per chunk the left count, per task the chunks' offsets, then the scatter
__device__ inline bool sah_goes_left(const float4* cen, uint32_t tri, int axis, int split, const uint32_t* a, int NB)
{
    const float lo = o2f(a[6 + axis]), hi = o2f(a[9 + axis]);
    const float4 q = cen[tri];
    const float c = axis == 0 ? q.x : (axis == 1 ? q.y : q.z);
    return sah_bin(c, lo, (double)NB / (double)(hi - lo), NB) < split;
}

__global__ __launch_bounds__(256) void k_sah_count(const uint32_t* ids, const float4* cen, const SahTask* tasks,
                                                   const uint32_t* chunk_task,
                                                   const uint32_t* chunk_begin, const uint32_t* chunk_end,
                                                   const uint32_t* acc, const int4* decision, int NB,
                                                   uint32_t* chunk_left)
{
    __shared__ uint32_t s;
    const uint32_t c = blockIdx.x, task = chunk_task[c];
    const int4 d = decision[task];
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    uint32_t mine = 0;
    for (uint32_t i = chunk_begin[c] + threadIdx.x; i < chunk_end[c]; i += 256) {
        const bool left = d.x >= 0 ? sah_goes_left(cen, ids[i], d.x, d.y, acc + 12 * (size_t)task, NB)
                                   : (i - tasks[task].first) < (uint32_t)d.z;   // halved range: order kept
        mine += left ? 1u : 0u;
    }
    atomicAdd(&s, mine);
    __syncthreads();
    if (threadIdx.x == 0) chunk_left[c] = s;
}

// one thread per large range: exclusive offsets of its chunks' left counts (its chunks are consecutive)
__global__ __launch_bounds__(256) void k_sah_offsets(const uint32_t* task_chunk0, const uint32_t* task_nchunks,
                                                     uint32_t n_tasks, const uint32_t* chunk_left, uint32_t* chunk_off)
{
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n_tasks) return;
    uint32_t acc = 0;
    for (uint32_t c = task_chunk0[t]; c < task_chunk0[t] + task_nchunks[t]; ++c) {
        chunk_off[c] = acc;
        acc += chunk_left[c];
    }
}

__global__ __launch_bounds__(256) void k_sah_scatter(const uint32_t* ids, const float4* cen, const SahTask* tasks,
                                                     const uint32_t* chunk_task, const uint32_t* chunk_begin,
                                                     const uint32_t* chunk_end, const uint32_t* acc,
                                                     const int4* decision, int NB, const uint32_t* chunk_off,
                                                     uint32_t* ids_out)
{
    __shared__ uint32_t s_wave[4];
    const uint32_t c = blockIdx.x, task = chunk_task[c];
    const int4 d = decision[task];
    const SahTask tk = tasks[task];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // left slots: first + chunk_off + rank; right slots: first + nl + (elements before this chunk that go right)
    uint32_t left_base = tk.first + chunk_off[c];
    uint32_t right_base = tk.first + (uint32_t)d.z + (chunk_begin[c] - tk.first - chunk_off[c]);
    for (uint32_t i0 = chunk_begin[c]; i0 < chunk_end[c]; i0 += 256) {
        const uint32_t i = i0 + threadIdx.x;
        const bool valid = i < chunk_end[c];
        const uint32_t tri = valid ? ids[i] : 0u;
        bool left;
        if (d.x >= 0) left = valid && sah_goes_left(cen, tri, d.x, d.y, acc + 12 * (size_t)task, NB);
        else left = valid && (i - tk.first) < (uint32_t)d.z;   // halved range: order kept
        const uint64_t m = __ballot(left);
        const uint32_t below = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) s_wave[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (uint32_t w = 0; w < 4; ++w) {
            if (w < wave) before += s_wave[w];
            total += s_wave[w];
        }
        const uint32_t rank_l = before + below;
        const uint32_t n_valid = min(256u, chunk_end[c] - i0);
        const uint32_t dst = left ? left_base + rank_l : right_base + (threadIdx.x - rank_l);
        if (valid && dst < tk.first + tk.count) ids_out[dst] = tri;   // always in range (same decisions as the bins)
        left_base += total;
        right_base += n_valid - total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_sah_copy(const uint32_t* src, const uint32_t* chunk_begin,
                                                  const uint32_t* chunk_end, uint32_t* dst)
{
    const uint32_t c = blockIdx.x;
    for (uint32_t i = chunk_begin[c] + threadIdx.x; i < chunk_end[c]; i += 256) dst[i] = src[i];
}

// ---- small ranges: one wave builds the whole subtree (depth first, its pending ranges in stack[first ..]) ----
__global__ __launch_bounds__(256) void k_sah_small(const SahTask* small, uint32_t n_small, uint32_t* ids,
                                                   uint32_t* tmp, const Box6* tri_box, const float4* cen, int NB,
                                                   uint32_t max_leaf, double node_cost, SahTree T, uint4* stack)
{
    __shared__ uint32_t lbins[4][3 * SAH_NB_MAX * SAH_BIN_WORDS];
    const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
    const uint32_t ti = blockIdx.x * 4 + wave;
    if (ti >= n_small) return;   // whole waves only: no workgroup barrier below
    uint32_t* lb = lbins[wave];
    const SahTask root = small[ti];
    uint4* stk = stack + root.first;
    uint32_t sp = 0;
    uint32_t node = root.node, f = root.first, n = root.count;
    const int words = 3 * NB * SAH_BIN_WORDS;
    for (;;) {
        // bounds of the range
        float v[12];
        for (int k = 0; k < 12; ++k) v[k] = (k % 6) < 3 ? INFINITY : -INFINITY;
        for (uint32_t i = f + lane; i < f + n; i += 64) {
            const uint32_t t = ids[i];
            const Box6 b = tri_box[t];
            const float4 q = cen[t];
            const float cc[3] = {q.x, q.y, q.z};
            for (int k = 0; k < 3; ++k) {
                v[k] = fminf(v[k], b.lo[k]); v[3 + k] = fmaxf(v[3 + k], b.hi[k]);
                v[6 + k] = fminf(v[6 + k], cc[k]); v[9 + k] = fmaxf(v[9 + k], cc[k]);
            }
        }
        for (int off = 32; off > 0; off >>= 1)
            for (int k = 0; k < 12; ++k) {
                const float o = __shfl_xor(v[k], off);
                v[k] = (k % 6) < 3 ? fminf(v[k], o) : fmaxf(v[k], o);
            }
        const float blo[3] = {v[0], v[1], v[2]}, bhi[3] = {v[3], v[4], v[5]};
        const float clo[3] = {v[6], v[7], v[8]}, chi[3] = {v[9], v[10], v[11]};
        bool leaf = n == 1;
        int axis = -1, split = 0;
        uint32_t nl = 0;
        if (!leaf) {
            for (int i = lane; i < words; i += 64) {
                const int w = i % SAH_BIN_WORDS;
                lb[i] = w < 3 ? O_POS_INF : (w < 6 ? O_NEG_INF : 0u);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (uint32_t i = f + lane; i < f + n; i += 64) {
                const uint32_t t = ids[i];
                const Box6 b = tri_box[t];
                const float4 q = cen[t];
                const float cc[3] = {q.x, q.y, q.z};
                for (int ax = 0; ax < 3; ++ax) {
                    const float ext = chi[ax] - clo[ax];
                    if (!(ext > 0.0f)) continue;
                    const int k = sah_bin(cc[ax], clo[ax], (double)NB / (double)ext, NB);
                    uint32_t* w = lb + ((size_t)ax * NB + k) * SAH_BIN_WORDS;
                    for (int j = 0; j < 3; ++j) { atomicMin(w + j, f2o(b.lo[j])); atomicMax(w + 3 + j, f2o(b.hi[j])); }
                    atomicAdd(w + 6, 1u);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            double best;
            sah_decide(lb, NB, clo, chi, axis, split, nl, best);
            const double parea = sah_area(blo, bhi);
            const double split_cost = parea > 0.0 ? node_cost + best / parea : (double)n;
            leaf = n <= max_leaf && (axis < 0 || (double)n <= split_cost);
            __builtin_amdgcn_wave_barrier();
        }
        if (leaf) {
            if (lane == 0) write_sah_node(T, node, blo, bhi, -1, -1, f, n);
            if (sp == 0) break;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            const uint4 e = stk[--sp];
            node = e.x; f = e.y; n = e.z;
            continue;
        }
        if (axis < 0) {
            nl = n / 2;   // coinciding centroids: halve the range, order kept
        } else {
            // stable partition into tmp, then back
            const float lo = clo[axis];
            const double scale = (double)NB / (double)(chi[axis] - clo[axis]);
            uint32_t lpos = f, rpos = f + nl;
            for (uint32_t i0 = f; i0 < f + n; i0 += 64) {
                const uint32_t i = i0 + lane;
                const bool valid = i < f + n;
                const uint32_t t = valid ? ids[i] : 0u;
                float c = 0.0f;
                if (valid) {
                    const float4 q = cen[t];
                    c = axis == 0 ? q.x : (axis == 1 ? q.y : q.z);
                }
                const bool left = valid && sah_bin(c, lo, scale, NB) < split;
                const uint64_t m = __ballot(left), mv = __ballot(valid);
                const uint64_t below = (1ull << lane) - 1ull;
                const uint32_t rl = (uint32_t)__popcll(m & below), rr = (uint32_t)__popcll(mv & ~m & below);
                const uint32_t dst = left ? lpos + rl : rpos + rr;
                if (valid && dst < f + n) tmp[dst] = t;   // always in range: the bins counted the same decisions
                lpos += (uint32_t)__popcll(m);
                rpos += (uint32_t)__popcll(mv & ~m);
            }
            // the lanes exchange ids through global memory: order the stores before the other lanes' loads
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            for (uint32_t i = f + lane; i < f + n; i += 64) ids[i] = tmp[i];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        uint32_t l = 0;
        if (lane == 0) l = atomicAdd(T.node_ctr, 2u);
        l = (uint32_t)__builtin_amdgcn_readfirstlane((int)l);
        if (lane == 0) write_sah_node(T, node, blo, bhi, (int)l, (int)(l + 1), f, n);
        stk[sp] = make_uint4(l + 1, f + nl, n - nl, 0u);   // every lane writes (and later reads) the same entry
        ++sp;
        node = l;
        n = nl;
    }
}

}  // namespace

// Binned-SAH build of n triangles on the device (see above); outputs as rc_build_bvh_device.
hipError_t rc_build_bvh_device_sah(const float* d_pos, const uint32_t* d_idx, uint32_t n, uint32_t bins,
                                   uint32_t max_leaf, float node_cost, Node4** d_nodes_out, uint32_t* n_nodes_out,
                                   uint32_t* d_order, std::vector<uint32_t>& level_start, hipStream_t st)
{
    *d_nodes_out = nullptr;
    *n_nodes_out = 0;
    level_start.clear();
    if (n == 0 || n > (1u << 28) || max_leaf < 1 || max_leaf > 4 || bins < 2 || bins > (uint32_t)SAH_NB_MAX)
        return hipErrorInvalidValue;
    const int NB = (int)bins;
    const size_t n2 = 2 * (size_t)n;                 // binary nodes
    const uint32_t max_big = n / SAH_SMALL + 2;      // large ranges of one level are disjoint
    const uint32_t max_chunks = n / SAH_CHUNK + max_big + 2;
    const size_t cap = (size_t)n + 2;                 // 4-wide nodes: at most one per internal binary node, plus root
    DevBuf<Box6> tri_box, box;
    DevBuf<float4> cen;
    DevBuf<int2> child, range;
    DevBuf<uint32_t> tmp, ctr, acc, binbuf, chunk_task, chunk_begin, chunk_end, chunk_left, chunk_off, task_chunk0,
        task_nchunks, par_a, par_b, overflow;
    DevBuf<SahTask> big_a, big_b, small;
    DevBuf<int4> decision;
    DevBuf<uint4> stack;
    DevBuf<int> lvl_a, lvl_b, nint, offs;
    DevBuf<Node4> nodes;
    DevBuf<uint8_t> temp;
    BH(tri_box.alloc(n));
    BH(cen.alloc(n));
    BH(box.alloc(n2));
    BH(child.alloc(n2));
    BH(range.alloc(n2));
    BH(tmp.alloc(n));
    BH(ctr.alloc(4));
    BH(acc.alloc((size_t)max_big * 12));
    BH(binbuf.alloc((size_t)max_big * 3 * NB * SAH_BIN_WORDS));
    BH(chunk_task.alloc(max_chunks));
    BH(chunk_begin.alloc(max_chunks));
    BH(chunk_end.alloc(max_chunks));
    BH(chunk_left.alloc(max_chunks));
    BH(chunk_off.alloc(max_chunks));
    BH(task_chunk0.alloc(max_big));
    BH(task_nchunks.alloc(max_big));
    BH(big_a.alloc(max_big));
    BH(big_b.alloc(max_big));
    BH(small.alloc(n));
    BH(decision.alloc(max_big));
    BH(stack.alloc(n));
    BH(nodes.alloc(cap));
    BH(lvl_a.alloc(cap));
    BH(lvl_b.alloc(cap));
    BH(par_a.alloc(cap));
    BH(par_b.alloc(cap));
    BH(nint.alloc(cap));
    BH(offs.alloc(cap));
    BH(overflow.alloc(1));
    size_t scan_bytes = 0;
    BH(rocprim::exclusive_scan(nullptr, scan_bytes, nint.p, offs.p, 0, cap, rocprim::plus<int>(), st));
    BH(temp.alloc(scan_bytes));

    hipLaunchKernelGGL(k_tri_boxes, dim3(nb(n, 256)), dim3(256), 0, st, d_pos, d_idx, n, tri_box.p, cen.p);
    hipLaunchKernelGGL(k_iota, dim3(nb(n, 256)), dim3(256), 0, st, d_order, n);
    // counters: [0] binary nodes allocated (the root is node 0), [1] large ranges of the next level, [2] small ranges
    const uint32_t ctr0[4] = {1u, 0u, 0u, 0u};
    BH(hipMemcpyAsync(ctr.p, ctr0, sizeof(ctr0), hipMemcpyHostToDevice, st));
    const SahTree T{child.p, range.p, box.p, ctr.p};
    std::vector<SahTask> big_h;
    if (n > SAH_SMALL) {
        big_h.push_back({0u, 0u, n, 0u});
    } else {
        const SahTask root{0u, 0u, n, 0u};
        BH(hipMemcpyAsync(small.p, &root, sizeof(root), hipMemcpyHostToDevice, st));
        const uint32_t one = 1u;
        BH(hipMemcpyAsync(ctr.p + 2, &one, sizeof(one), hipMemcpyHostToDevice, st));
    }
    if (!big_h.empty()) BH(hipMemcpyAsync(big_a.p, big_h.data(), sizeof(SahTask), hipMemcpyHostToDevice, st));
    std::vector<uint32_t> ct, cb, ce, t0, tn;
    while (!big_h.empty()) {
        const uint32_t nt = (uint32_t)big_h.size();
        ct.clear(); cb.clear(); ce.clear(); t0.clear(); tn.clear();
        for (uint32_t t = 0; t < nt; ++t) {
            t0.push_back((uint32_t)ct.size());
            for (uint32_t b = big_h[t].first; b < big_h[t].first + big_h[t].count; b += SAH_CHUNK) {
                ct.push_back(t);
                cb.push_back(b);
                ce.push_back(std::min(b + SAH_CHUNK, big_h[t].first + big_h[t].count));
            }
            tn.push_back((uint32_t)ct.size() - t0.back());
        }
        const uint32_t nc = (uint32_t)ct.size();
        if (nc > max_chunks || nt > max_big) return hipErrorUnknown;
        BH(hipMemcpyAsync(chunk_task.p, ct.data(), nc * 4, hipMemcpyHostToDevice, st));
        BH(hipMemcpyAsync(chunk_begin.p, cb.data(), nc * 4, hipMemcpyHostToDevice, st));
        BH(hipMemcpyAsync(chunk_end.p, ce.data(), nc * 4, hipMemcpyHostToDevice, st));
        BH(hipMemcpyAsync(task_chunk0.p, t0.data(), nt * 4, hipMemcpyHostToDevice, st));
        BH(hipMemcpyAsync(task_nchunks.p, tn.data(), nt * 4, hipMemcpyHostToDevice, st));
        const uint32_t zero = 0u;
        BH(hipMemcpyAsync(ctr.p + 1, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_sah_reset, dim3(std::min<unsigned>(1024, nb((size_t)nt * (12 + 3 * NB * SAH_BIN_WORDS), 256))),
                           dim3(256), 0, st, acc.p, binbuf.p, nt, NB);
        hipLaunchKernelGGL(k_sah_bounds, dim3(nc), dim3(256), 0, st, d_order, tri_box.p, cen.p, chunk_task.p,
                           chunk_begin.p, chunk_end.p, acc.p);
        hipLaunchKernelGGL(k_sah_bins, dim3(nc), dim3(256), 0, st, d_order, tri_box.p, cen.p, chunk_task.p,
                           chunk_begin.p, chunk_end.p, acc.p, binbuf.p, NB);
        hipLaunchKernelGGL(k_sah_split, dim3(nt), dim3(64), 0, st, big_a.p, acc.p, binbuf.p, NB, T, big_b.p, ctr.p + 1,
                           small.p, ctr.p + 2, decision.p);
        hipLaunchKernelGGL(k_sah_count, dim3(nc), dim3(256), 0, st, d_order, cen.p, big_a.p, chunk_task.p,
                           chunk_begin.p, chunk_end.p, acc.p, decision.p, NB, chunk_left.p);
        hipLaunchKernelGGL(k_sah_offsets, dim3(nb(nt, 256)), dim3(256), 0, st, task_chunk0.p, task_nchunks.p, nt,
                           chunk_left.p, chunk_off.p);
        hipLaunchKernelGGL(k_sah_scatter, dim3(nc), dim3(256), 0, st, d_order, cen.p, big_a.p, chunk_task.p,
                           chunk_begin.p, chunk_end.p, acc.p, decision.p, NB, chunk_off.p, tmp.p);
        hipLaunchKernelGGL(k_sah_copy, dim3(nc), dim3(256), 0, st, tmp.p, chunk_begin.p, chunk_end.p, d_order);
        BH(hipGetLastError());
        uint32_t next = 0;
        BH(hipMemcpyAsync(&next, ctr.p + 1, sizeof(next), hipMemcpyDeviceToHost, st));
        BH(hipStreamSynchronize(st));
        if (next > max_big) return hipErrorUnknown;
        big_h.resize(next);
        if (next) BH(hipMemcpyAsync(big_h.data(), big_b.p, next * sizeof(SahTask), hipMemcpyDeviceToHost, st));
        BH(hipStreamSynchronize(st));
        std::swap(big_a.p, big_b.p);
        if (next) BH(hipMemcpyAsync(big_a.p, big_h.data(), next * sizeof(SahTask), hipMemcpyHostToDevice, st));
    }
    uint32_t n_small = 0;
    BH(hipMemcpyAsync(&n_small, ctr.p + 2, sizeof(n_small), hipMemcpyDeviceToHost, st));
    BH(hipStreamSynchronize(st));
    if (n_small > n) return hipErrorUnknown;
    if (n_small)
        hipLaunchKernelGGL(k_sah_small, dim3(nb(n_small, 4)), dim3(256), 0, st, small.p, n_small, d_order, tmp.p,
                           tri_box.p, cen.p, NB, max_leaf, (double)node_cost, T, stack.p);
    BH(hipGetLastError());

    // 4-wide collapse from the root (binary node 0), level by level
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, lvl_a.p, 0, 1u);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, reinterpret_cast<int*>(par_a.p), -1, 1u);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, reinterpret_cast<int*>(overflow.p), 0, 1u);
    TreeView TV{(int)n, (int)max_leaf, child.p, range.p, box.p, nullptr};
    TV.explicit_leaves = 1;
    uint32_t m = 1, base = 0, depth = 0;
    while (m > 0) {
        if ((size_t)base + m > cap) return hipErrorUnknown;
        hipLaunchKernelGGL(k_collapse_count, dim3(nb(m, 256)), dim3(256), 0, st, TV, lvl_a.p, (int)m, nint.p);
        size_t sb = scan_bytes;
        BH(rocprim::exclusive_scan(temp.p, sb, nint.p, offs.p, 0, (size_t)m, rocprim::plus<int>(), st));
        hipLaunchKernelGGL(k_collapse_write, dim3(nb(m, 256)), dim3(256), 0, st, TV, lvl_a.p, par_a.p, (int)m, offs.p,
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
    if (n <= SORT_BLOCK_MAX) {
        hipLaunchKernelGGL(k_sort_block, dim3(1), dim3(SORT_THREADS), 0, st, (const uint64_t*)w.keys,
                           (const uint32_t*)w.vals, n, (uint64_t*)w.keys_s, (uint32_t*)w.order);
    } else {
        size_t bytes = w.temp_bytes;
        BH(rocprim::radix_sort_pairs(w.temp, bytes, (uint64_t*)w.keys, (uint64_t*)w.keys_s, (uint32_t*)w.vals,
                                     (uint32_t*)w.order, n, 0, 63, st));
    }
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
