// BVH build on the GPU: a linear BVH (Morton order of triangle centroids, radix tree of Karras, 2012),
// boxes computed bottom-up with exact FP32 min/max, then collapsed level by level into the same 4-wide,
// breadth-first node layout as the host builder (ranges of at most max_leaf consecutive triangles in
// Morton order become leaves), so that traversal and refit use it unchanged.
//
// Binary tree indexing: internal nodes 0 .. n-2 (root 0), leaves n-1 .. 2n-2 (leaf n-1+i holds the
// triangle at sorted position i).
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "rc_internal.h"

namespace {

struct Box6 {
    float lo[3], hi[3];
};

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
    cen[t] = make_float4(0.5f * b.lo[0] + 0.5f * b.hi[0], 0.5f * b.lo[1] + 0.5f * b.hi[1],
                         0.5f * b.lo[2] + 0.5f * b.hi[2], 0.0f);
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

__global__ void k_cen_bounds_final(const float* partial, int nb, float* out)
{
    if (threadIdx.x >= 6) return;
    const int k = threadIdx.x;
    float v = k < 3 ? INFINITY : -INFINITY;
    for (int b = 0; b < nb; ++b) v = k < 3 ? fminf(v, partial[b * 6 + k]) : fmaxf(v, partial[b * 6 + k]);
    out[k] = v;
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

// common prefix length of sorted keys i and j, with the position as a tie-break for equal keys; -1 outside
__device__ inline int delta(const uint64_t* k, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    const uint64_t a = k[i], b = k[j];
    if (a == b) return 64 + __clz((uint32_t)i ^ (uint32_t)j);
    return __clzll(a ^ b);
}

// internal node i of the radix tree: children (unified index) and the range of sorted positions it covers
__global__ __launch_bounds__(256) void k_radix_tree(const uint64_t* keys, int n, int2* child, int2* range, int* parent)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta(keys, n, i, i - d);
    int lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = delta(keys, n, i, j);
    int s = 0;
    for (int t = (l + 1) >> 1;; t = (t + 1) >> 1) {
        if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
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
__global__ __launch_bounds__(256) void k_bottom_up(const Box6* tri_box, const uint32_t* vals, int n, const int2* child,
                                                   const int* parent, uint32_t* flags, Box6* box)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int node = n - 1 + i;
    Box6 u = tri_box[vals[i]];
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
};

__device__ inline int node_size(const TreeView& T, int b) { return b >= T.n - 1 ? 1 : T.range[b].y - T.range[b].x + 1; }
__device__ inline bool openable(const TreeView& T, int b) { return b < T.n - 1 && node_size(T, b) > T.max_leaf; }
__device__ inline float box_area(const Box6& b)
{
    const float dx = b.hi[0] - b.lo[0], dy = b.hi[1] - b.lo[1], dz = b.hi[2] - b.lo[2];
    return dx * dy + dy * dz + dz * dx;
}

// children of the 4-wide node over binary node b: open the largest openable child until there are 4
__device__ inline int gather_kids(const TreeView& T, int b, int kids[4])
{
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

__global__ __launch_bounds__(256) void k_collapse_count(TreeView T, const int* level, int m, int* n_internal)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    int kids[4];
    const int cnt = gather_kids(T, level[k], kids);
    int ni = 0;
    for (int s = 0; s < cnt; ++s) ni += openable(T, kids[s]) ? 1 : 0;
    n_internal[k] = ni;
}

__global__ __launch_bounds__(256) void k_collapse_write(TreeView T, const int* level, const uint32_t* level_parent,
                                                        int m, const int* offs, uint32_t level_base, uint32_t next_base,
                                                        uint32_t depth, uint32_t cap, Node4* nodes,
                                                        int* next_level, uint32_t* next_parent, uint32_t* overflow)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    int kids[4];
    const int cnt = gather_kids(T, level[k], kids);
    Node4 nd;
    int j = 0;
    for (int s = 0; s < 4; ++s) {
        if (s >= cnt) {
            nd.lo_x[s] = nd.lo_y[s] = nd.lo_z[s] = INFINITY;
            nd.hi_x[s] = nd.hi_y[s] = nd.hi_z[s] = -INFINITY;
            nd.child[s] = RC_EMPTY_CHILD;
            continue;
        }
        const int b = kids[s];
        const Box6 bx = T.box[b];
        nd.lo_x[s] = bx.lo[0]; nd.hi_x[s] = bx.hi[0];
        nd.lo_y[s] = bx.lo[1]; nd.hi_y[s] = bx.hi[1];
        nd.lo_z[s] = bx.lo[2]; nd.hi_z[s] = bx.hi[2];
        if (openable(T, b)) {
            const int slot = offs[k] + j++;
            nd.child[s] = next_base + (uint32_t)slot;
            if (next_base + (uint32_t)slot < cap) {
                next_level[slot] = b;
                next_parent[slot] = level_base + (uint32_t)k;
            } else {
                atomicOr(overflow, 1u);
            }
        } else {
            const int first = b >= T.n - 1 ? b - (T.n - 1) : T.range[b].x;
            nd.child[s] = rc_make_leaf((uint32_t)first, (uint32_t)node_size(T, b));
        }
    }
    nd.parent = level_parent[k];
    nd.level = depth;
    nd.pad[0] = nd.pad[1] = 0u;
    nodes[level_base + k] = nd;
}

// root node over all triangles as one leaf (n <= max_leaf)
__global__ void k_single_leaf_root(const Box6* box, uint32_t n, Node4* nodes)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    Node4 nd;
    for (int s = 0; s < 4; ++s) {
        nd.lo_x[s] = nd.lo_y[s] = nd.lo_z[s] = INFINITY;
        nd.hi_x[s] = nd.hi_y[s] = nd.hi_z[s] = -INFINITY;
        nd.child[s] = RC_EMPTY_CHILD;
    }
    const Box6 b = box[0];
    nd.lo_x[0] = b.lo[0]; nd.hi_x[0] = b.hi[0];
    nd.lo_y[0] = b.lo[1]; nd.hi_y[0] = b.hi[1];
    nd.lo_z[0] = b.lo[2]; nd.hi_z[0] = b.hi[2];
    nd.child[0] = rc_make_leaf(0u, n);
    nd.parent = 0xFFFFFFFFu;
    nd.level = 0;
    nd.pad[0] = nd.pad[1] = 0u;
    nodes[0] = nd;
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

// Build the BVH of n triangles (n >= 1) on the device.  On success *d_nodes_out (device, allocated here with
// hipMalloc, owned by the caller afterwards) holds *n_nodes_out nodes in breadth-first level order, d_order
// (device, n entries, caller-allocated) maps leaf slots to original triangle ids, and level_start receives
// the first node of every level followed by the node count.  Synchronises the stream before returning.
hipError_t rc_build_bvh_device(const float* d_pos, const uint32_t* d_idx, uint32_t n, uint32_t max_leaf,
                               Node4** d_nodes_out, uint32_t* n_nodes_out, uint32_t* d_order,
                               std::vector<uint32_t>& level_start, hipStream_t st)
{
    *d_nodes_out = nullptr;
    *n_nodes_out = 0;
    level_start.clear();
    if (n == 0 || n > (1u << 28) || max_leaf < 1 || max_leaf > 4) return hipErrorInvalidValue;
    const int N = (int)n;
    // 4-wide nodes: each consumes at least one binary node of more than max_leaf triangles, and those that
    // consume only one have two children that are leaves over disjoint triangle ranges of size >= 2, so
    // there are at most (n - 1 + n / 2) / 2 < 3n / 4 of them.
    const size_t cap = 3 * (size_t)n / 4 + 2;
    const int red_blocks = 1024;
    DevBuf<Box6> tri_box, box;
    DevBuf<float4> cen;
    DevBuf<float> partial, bounds;
    DevBuf<uint64_t> keys, keys_s;
    DevBuf<uint32_t> vals, flags, par_a, par_b, overflow;
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
    size_t sort_bytes = 0, scan_bytes = 0;
    BH(rocprim::radix_sort_pairs(nullptr, sort_bytes, keys.p, keys_s.p, vals.p, d_order, n, 0, 63, st));
    BH(rocprim::exclusive_scan(nullptr, scan_bytes, nint.p, offs.p, 0, cap, rocprim::plus<int>(), st));
    BH(temp.alloc(std::max(sort_bytes, scan_bytes)));

    hipLaunchKernelGGL(k_tri_boxes, dim3(nb(n, 256)), dim3(256), 0, st, d_pos, d_idx, n, tri_box.p, cen.p);
    hipLaunchKernelGGL(k_cen_bounds, dim3(red_blocks), dim3(256), 0, st, cen.p, n, partial.p);
    hipLaunchKernelGGL(k_cen_bounds_final, dim3(1), dim3(64), 0, st, partial.p, red_blocks, bounds.p);
    hipLaunchKernelGGL(k_morton, dim3(nb(n, 256)), dim3(256), 0, st, cen.p, n, bounds.p, keys.p, vals.p);
    BH(hipGetLastError());
    BH(rocprim::radix_sort_pairs(temp.p, sort_bytes, keys.p, keys_s.p, vals.p, d_order, n, 0, 63, st));
    hipLaunchKernelGGL(k_fill_i32, dim3(nb(2 * (size_t)n, 256)), dim3(256), 0, st, parent.p, -1, 2 * n);
    hipLaunchKernelGGL(k_fill_i32, dim3(nb(n, 256)), dim3(256), 0, st, reinterpret_cast<int*>(flags.p), 0, n);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, reinterpret_cast<int*>(overflow.p), 0, 1u);
    if (N > 1)
        hipLaunchKernelGGL(k_radix_tree, dim3(nb(n - 1, 256)), dim3(256), 0, st, keys_s.p, N, child.p, range.p,
                           parent.p);
    // binary root: internal node 0, or for n = 1 the only leaf, whose unified index n - 1 is also 0
    hipLaunchKernelGGL(k_bottom_up, dim3(nb(n, 256)), dim3(256), 0, st, tri_box.p, d_order, N, child.p, parent.p,
                       flags.p, box.p);
    BH(hipGetLastError());
    if (N <= (int)max_leaf) {
        hipLaunchKernelGGL(k_single_leaf_root, dim3(1), dim3(64), 0, st, box.p, n, nodes.p);
        BH(hipGetLastError());
        level_start = {0u, 1u};
    } else {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, lvl_a.p, 0, 1u);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, reinterpret_cast<int*>(par_a.p), -1, 1u);
        const TreeView T{N, (int)max_leaf, child.p, range.p, box.p};
        uint32_t m = 1, base = 0, depth = 0;
        while (m > 0) {
            if ((size_t)base + m > cap) return hipErrorUnknown;   // excluded by the bound on cap
            hipLaunchKernelGGL(k_collapse_count, dim3(nb(m, 256)), dim3(256), 0, st, T, lvl_a.p, (int)m, nint.p);
            size_t sb = scan_bytes;
            BH(rocprim::exclusive_scan(temp.p, sb, nint.p, offs.p, 0, (size_t)m, rocprim::plus<int>(), st));
            hipLaunchKernelGGL(k_collapse_write, dim3(nb(m, 256)), dim3(256), 0, st, T, lvl_a.p, par_a.p, (int)m,
                               offs.p, base, base + m, depth, (uint32_t)cap, nodes.p, lvl_b.p, par_b.p, overflow.p);
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
    }
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
