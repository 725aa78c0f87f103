// One traversal step of the 4-wide BVH, shared by the single-view kernels and the batched
// megakernel so that both run exactly the same sequence of tests for a given ray.
#pragma once

#include "rc_device.h"

#define RC_STACK_EMPTY 0xFFFFFFFEu
// stack entry that ends a bottom-level traversal (two-level structures): the ray returns to world space
#define RC_INST_RETURN 0xFFFFFFFDu

// growth of the far-plane reciprocals (1 + 2^-20): the far slab distances round outward
#define RC_FAR_GROW 1.000001f

struct TravRay {
    float o[3], d[3], inv[3];
    float invf[3], cn[3], cf[3];   // slab test constants (set with inv by rc_ray_inv)
    float sx, sy, sz;         // watertight test: shear constants (set with inv by rc_ray_inv)
    uint32_t kx, ky, kz;      // watertight test: axes
};

__device__ inline float rc_axis(const float v[3], uint32_t k) { return k == 0u ? v[0] : (k == 1u ? v[1] : v[2]); }

// a, b or c for k = 0, 1, 2, as two selects (a nested conditional or an indexed array compiled into per-lane
// branches or scratch memory in the triangle tests)
__device__ inline float rc_pick(float a, float b, float c, uint32_t k)
{
    const float ab = k == 0u ? a : b;
    return k == 2u ? c : ab;
}

struct TravState {
    uint32_t cur;       // child word being processed (node index or leaf), or RC_STACK_EMPTY
    int sp;
    uint32_t best_id;
    float best_t, best_u, best_v;
};

// World-space ray of a two-level traversal while the working ray is mapped into an instance.  The flag is
// a 32-bit word: per-lane bool state carried through the divergent traversal loops has been mishandled
// by the compiler (lanes losing their value), 32-bit words have not.
struct TravWorld {
    float o[3], d[3];
    uint32_t in_blas;
};

// Per-ray constants of the traversal.
// Slab tests: with dd the direction clamped away from zero (|dd| >= 1e-20), a plane at coordinate p lies at
// distance (p - o) / dd along the ray, which the tests evaluate as one FMA, p * inv + c:
//   near planes  inv  = 1 / dd (correctly rounded),      cn = -o * inv  moved down by 2^-21 |.| + 2^-120,
//   far planes   invf = inv * (1 + 2^-20),               cf = -o * invf moved up   by 2^-21 |.| + 2^-120.
// The margins exceed the rounding of the products -o * inv (and of the margin additions), so cn <= -o * inv
// and cf >= -o * invf hold in exact arithmetic.  A computed near distance is then at most (1 + 2u) times the
// exact one and a computed far distance, where the exact one is >= 0, at least (1 + 12u) times it
// (u = 2^-24), so a box that the exact segment enters always passes max(near, 0) <= min(far, bound).
// Watertight triangle test: the axis kz of the largest |d| (first on ties), kx and ky the next axes
// cyclically (swapped when d[kz] < 0), Sx = d[kx] / d[kz], Sy = d[ky] / d[kz], Sz = 1 / d[kz] (correctly
// rounded).  Kernels that test triangles with Moller-Trumbore never read the shear constants, so their
// computation is dropped.
__device__ inline void rc_ray_inv(TravRay& r)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float dd = fabsf(r.d[a]) < 1e-20f ? copysignf(1e-20f, r.d[a]) : r.d[a];
        r.inv[a] = 1.0f / dd;
        r.invf[a] = r.inv[a] * RC_FAR_GROW;
        const float c = -(r.o[a] * r.inv[a]);
        r.cn[a] = c - (fabsf(c) * 0x1p-21f + 0x1p-120f);
        const float e = -(r.o[a] * r.invf[a]);
        r.cf[a] = e + (fabsf(e) * 0x1p-21f + 0x1p-120f);
    }
    uint32_t kz = 0u;
    if (fabsf(r.d[1]) > fabsf(r.d[0])) kz = 1u;
    if (fabsf(r.d[2]) > fabsf(rc_axis(r.d, kz))) kz = 2u;
    uint32_t kx = kz == 2u ? 0u : kz + 1u;
    uint32_t ky = kx == 2u ? 0u : kx + 1u;
    const float dz = rc_axis(r.d, kz);
    if (dz < 0.0f) { const uint32_t t = kx; kx = ky; ky = t; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.sx = rc_axis(r.d, kx) / dz;
    r.sy = rc_axis(r.d, ky) / dz;
    r.sz = 1.0f / dz;
}

// Slab test of one box, its near (nx, ny, nz) and far (fx, fy, fz) plane coordinates picked by the signs
// of the ray's direction: whether the segment [0, bound] enters the box, and the entry distance t0 >= 0.
__device__ inline bool rc_slab(const TravRay& r, float nx, float ny, float nz, float fx, float fy, float fz,
                               float bound, float& t0)
{
    t0 = fmaxf(fmaxf(fmaf(nx, r.inv[0], r.cn[0]), fmaf(ny, r.inv[1], r.cn[1])),
               fmaxf(fmaf(nz, r.inv[2], r.cn[2]), 0.0f));
    const float t1 = fminf(fminf(fmaf(fx, r.invf[0], r.cf[0]), fmaf(fy, r.invf[1], r.cf[1])),
                           fminf(fmaf(fz, r.invf[2], r.cf[2]), bound));
    return t0 <= t1;
}

// The world ray (o, d) mapped into an instance by its world-to-object map W = [M | m] (row-major 3x4):
// o' = M o + m, d' = M d, each component as ((M0 a0 + M1 a1) + M2 a2) [+ m] in FP32.
__device__ inline void rc_map_ray(const float* W, const float o[3], const float d[3], TravRay& r)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float a = W[4 * k] * o[0];
        const float b = W[4 * k + 1] * o[1];
        const float c = W[4 * k + 2] * o[2];
        r.o[k] = ((a + b) + c) + W[4 * k + 3];
        const float e = W[4 * k] * d[0];
        const float f = W[4 * k + 1] * d[1];
        const float g = W[4 * k + 2] * d[2];
        r.d[k] = (e + f) + g;
    }
    rc_ray_inv(r);
}

// Work queue split over the XCDs.  Workgroups are dispatched to the XCDs round-robin, so workgroup b runs
// on XCD g = b % RC_XCDS.  The work sequence (items, or 64-ray packets) is cut into chunks of CHUNK that
// are dealt to the XCDs in turn; the waves of XCD g claim positions j = 0, 1, 2, ... of that XCD's share
// from their own counter (one atomic per claim of several positions).  The waves of one XCD thus work
// on neighbouring pixels and share its L2, the eight counters split the atomic traffic, and the fine
// interleave of chunks keeps the XCDs' shares balanced.
template <uint32_t CHUNK>
struct XcdQueue {
    uint32_t* ctr;
    uint32_t g;
    uint64_t n;
    __device__ XcdQueue(uint32_t* counters, uint32_t slot, uint64_t n_work)
        : ctr(counters + RC_QUEUE_BASE + (slot * RC_XCDS + blockIdx.x % RC_XCDS) * 64),
          g(blockIdx.x % RC_XCDS), n(n_work) {}
    __device__ uint64_t chunk_of(uint64_t j) const { return g + (uint64_t)RC_XCDS * (j / CHUNK); }
    // work index at position j of this XCD's share (may be >= n inside the last chunk)
    __device__ uint64_t at(uint64_t j) const { return chunk_of(j) * CHUNK + j % CHUNK; }
    // no work at position j or beyond
    __device__ bool exhausted(uint64_t j) const { return chunk_of(j) * CHUNK >= n; }
    // wave-uniform claim of `count` positions (called by all lanes; lane 0 does the atomic)
    __device__ uint32_t claim(uint32_t count) const
    {
        uint32_t b = 0;
        if (__lane_id() == 0) b = atomicAdd(ctr, count);
        return __builtin_amdgcn_readfirstlane(b);
    }
};

// Dynamic LDS of the traversal kernels: the per-lane stacks.
extern __shared__ uint32_t rc_lds[];

// Per-lane stack: LDS part [depth][block] (lane-interleaved, conflict free; node words, then the entry
// distances when HAS_T) + global overflow.  LDS bytes per block: rc_stack_lds_bytes<...>().
template <int SL, int BLOCK, bool HAS_T>
struct TravStack {
    int tid;
    uint2* overflow;
    uint32_t overflow_depth, n_lanes, glane;
    uint32_t* error_flag;

    static constexpr size_t lds_bytes() { return (size_t)SL * BLOCK * 4 * (HAS_T ? 2 : 1); }

    __device__ inline void push(int& sp, uint32_t w, float tn)
    {
        if (sp < SL) {
            rc_lds[sp * BLOCK + tid] = w;
            if (HAS_T) rc_lds[(SL + sp) * BLOCK + tid] = __float_as_uint(tn);
        } else if ((uint32_t)(sp - SL) < overflow_depth) {
            overflow[(size_t)(sp - SL) * n_lanes + glane] = make_uint2(w, __float_as_uint(tn));
        } else {
            *error_flag = 1u;   // bound exceeded: the entry is dropped and the error is reported
            return;
        }
        ++sp;
    }

    // pop the next entry; closest-hit rays skip entries that start beyond the current hit
    __device__ inline uint32_t pop(int& sp, bool cull, float best_t)
    {
        for (;;) {
            if (sp == 0) return RC_STACK_EMPTY;
            --sp;
            uint32_t w;
            float tn;
            if (sp < SL) {
                w = rc_lds[sp * BLOCK + tid];
                tn = HAS_T ? __uint_as_float(rc_lds[(SL + sp) * BLOCK + tid]) : 0.0f;
            } else {
                uint2 g = overflow[(size_t)(sp - SL) * n_lanes + glane];
                w = g.x;
                tn = __uint_as_float(g.y);
            }
            if (!cull || tn <= best_t) return w;
        }
    }
};

// Start a ray at node `root` (0 for a flat BVH, the top-level root of a two-level structure); w (two-level
// traversals only) keeps the world ray.
__device__ inline void trav_begin(TravRay& r, TravState& s, uint32_t root = 0u, TravWorld* w = nullptr)
{
    rc_ray_inv(r);
    s.cur = root;
    s.sp = 0;
    s.best_id = RC_NO_HIT;
    s.best_t = INFINITY;
    s.best_u = s.best_v = 0.0f;
    if (w) {
#pragma unroll
        for (int a = 0; a < 3; ++a) { w->o[a] = r.o[a]; w->d[a] = r.d[a]; }
        w->in_blas = 0u;
    }
}

// Next stack entry; in a two-level traversal an instance's end marker restores the world ray.
template <bool TWO, class Stack>
__device__ inline uint32_t trav_pop(TravRay& r, TravState& s, Stack& st, bool any, TravWorld* w)
{
    for (;;) {
        const uint32_t c = st.pop(s.sp, !any, s.best_t);
        if (!TWO || c != RC_INST_RETURN) return c;
#pragma unroll
        for (int a = 0; a < 3; ++a) { r.o[a] = w->o[a]; r.d[a] = w->d[a]; }
        rc_ray_inv(r);
        w->in_blas = 0u;
    }
}

// Visit the internal node s.cur: test the four child boxes, continue with the nearest hit child and
// push the others (farthest first), or pop.  `any`: any-hit ray on the segment 0 < t < 1, otherwise
// closest hit (boxes beyond the current hit are culled).
template <bool TWO = false, class Stack>
__device__ inline void trav_visit_node(const DevScene& sc, TravRay& r, TravState& s, Stack& st, bool any,
                                       TravWorld* w = nullptr)
{
    const float4* np = reinterpret_cast<const float4*>(sc.nodes + s.cur);
    float4 lx = np[0], hx = np[1], ly = np[2], hy = np[3], lz = np[4], hz = np[5];
    uint4 ch = reinterpret_cast<const uint4*>(np)[6];
    const float bound = any ? 1.0f : s.best_t;
    float lxs[4] = {lx.x, lx.y, lx.z, lx.w}, hxs[4] = {hx.x, hx.y, hx.z, hx.w};
    float lys[4] = {ly.x, ly.y, ly.z, ly.w}, hys[4] = {hy.x, hy.y, hy.z, hy.w};
    float lzs[4] = {lz.x, lz.y, lz.z, lz.w}, hzs[4] = {hz.x, hz.y, hz.z, hz.w};
    uint32_t cw[4] = {ch.x, ch.y, ch.z, ch.w};
    float tn[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float nx = r.inv[0] >= 0.0f ? lxs[c] : hxs[c], fx = r.inv[0] >= 0.0f ? hxs[c] : lxs[c];
        float ny = r.inv[1] >= 0.0f ? lys[c] : hys[c], fy = r.inv[1] >= 0.0f ? hys[c] : lys[c];
        float nz = r.inv[2] >= 0.0f ? lzs[c] : hzs[c], fz = r.inv[2] >= 0.0f ? hzs[c] : lzs[c];
        float t0;
        const bool hit = rc_slab(r, nx, ny, nz, fx, fy, fz, bound, t0);
        tn[c] = hit ? t0 : INFINITY;
    }
    // sort (distance, child) ascending with five comparators: misses (inf) sink to the end
#define RC_CS(a, b)                                                                   \
    {                                                                                 \
        bool sw = tn[b] < tn[a];                                                      \
        float ta = sw ? tn[b] : tn[a], tb = sw ? tn[a] : tn[b];                       \
        uint32_t ca = sw ? cw[b] : cw[a], cb = sw ? cw[a] : cw[b];                    \
        tn[a] = ta; tn[b] = tb; cw[a] = ca; cw[b] = cb;                               \
    }
    RC_CS(0, 1) RC_CS(2, 3) RC_CS(0, 2) RC_CS(1, 3) RC_CS(1, 2)
#undef RC_CS
    if (tn[3] < INFINITY) st.push(s.sp, cw[3], tn[3]);
    if (tn[2] < INFINITY) st.push(s.sp, cw[2], tn[2]);
    if (tn[1] < INFINITY) st.push(s.sp, cw[1], tn[1]);
    s.cur = tn[0] < INFINITY ? cw[0] : trav_pop<TWO>(r, s, st, any, w);
}

// Moller-Trumbore in FP32 on a packed triangle (v0, e1, e2): the fixed operation order every traversal
// kernel uses.  Each cross-product component is fma(a, b, -(c d)) and each dot product
// fma(z, z', fma(y, y', x x')): one rounding per FMA, so every result stays within the running forward-error
// bound of the unfused evaluation (product roundings and sum roundings counted separately).  Returns whether
// the ray's line crosses the triangle at t > 0 (edges inclusive).
__device__ inline bool rc_mt(const TravRay& r, float ax, float ay, float az, float bx, float by, float bz, float cx,
                             float cy, float cz, float& t, float& u, float& v)
{
    const float px_ = fmaf(r.d[1], cz, -(r.d[2] * cy));
    const float py_ = fmaf(r.d[2], cx, -(r.d[0] * cz));
    const float pz_ = fmaf(r.d[0], cy, -(r.d[1] * cx));
    const float det = fmaf(bz, pz_, fmaf(by, py_, bx * px_));
    const float idet = __builtin_amdgcn_rcpf(det);
    const float sx = r.o[0] - ax, sy = r.o[1] - ay, sz = r.o[2] - az;
    const float su = fmaf(sz, pz_, fmaf(sy, py_, sx * px_));
    u = su * idet;
    t = 0.0f;
    v = 0.0f;
    // staged so that a wave skips the rest once no lane can still hit; u > 1 fails as u + v <= 1 would
    // (v >= 0 makes the rounded u + v at least u), so every decision is the unstaged test's
    if (!(u >= 0.0f && u <= 1.0f)) return false;
    const float qx = fmaf(sy, bz, -(sz * by));
    const float qy = fmaf(sz, bx, -(sx * bz));
    const float qz = fmaf(sx, by, -(sy * bx));
    const float sv = fmaf(r.d[2], qz, fmaf(r.d[1], qy, r.d[0] * qx));
    v = sv * idet;
    if (!(v >= 0.0f && u + v <= 1.0f)) return false;
    const float stq = fmaf(cz, qz, fmaf(cy, qy, cx * qx));
    t = stq * idet;
    return t > 0.0f;
}

// rc_mt's arithmetic with its conditions decided without branches, for a segment: whether the ray crosses
// the triangle at 0 < t < 1.  min(u, v, 1 - (u + v)) >= 0 holds exactly when u >= 0, v >= 0 and u + v <= 1
// (1 - s, for an FP32 s > 1, is at most -2^-23, so its sign is exact) as long as rcp(det) is finite (m is
// then never NaN); when it is not, t is infinite or NaN and fails the range test, as it fails rc_mt.
// 0 < t < 1 is one unsigned compare of t's bit pattern minus one against that of the largest float below 1.
// Called by whole waves (uniform control flow): once u is known, the wave skips the rest when no lane has
// 0 <= u <= 1 (u > 1 fails as u + v <= 1 would, since v >= 0 makes the rounded u + v at least u).
__device__ inline bool rc_mt_segment(const TravRay& r, float ax, float ay, float az, float bx, float by, float bz,
                                     float cx, float cy, float cz)
{
    const float px_ = fmaf(r.d[1], cz, -(r.d[2] * cy));
    const float py_ = fmaf(r.d[2], cx, -(r.d[0] * cz));
    const float pz_ = fmaf(r.d[0], cy, -(r.d[1] * cx));
    const float det = fmaf(bz, pz_, fmaf(by, py_, bx * px_));
    const float idet = __builtin_amdgcn_rcpf(det);
    const float sx = r.o[0] - ax, sy = r.o[1] - ay, sz = r.o[2] - az;
    const float su = fmaf(sz, pz_, fmaf(sy, py_, sx * px_));
    const float u = su * idet;
    if (__ballot(u >= 0.0f && u <= 1.0f) == 0) return false;
    const float qx = fmaf(sy, bz, -(sz * by));
    const float qy = fmaf(sz, bx, -(sx * bz));
    const float qz = fmaf(sx, by, -(sy * bx));
    const float sv = fmaf(r.d[2], qz, fmaf(r.d[1], qy, r.d[0] * qx));
    const float v = sv * idet;
    const float stq = fmaf(cz, qz, fmaf(cy, qy, cx * qx));
    const float t = stq * idet;
    const float m = fminf(fminf(u, v), 1.0f - (u + v));
    // all ones when m < 0 (m + 0 turns -0 into +0, which passes like u >= 0 does for u = -0)
    const uint32_t neg = (uint32_t)((int32_t)__float_as_uint(m + 0.0f) >> 31);
    return ((__float_as_uint(t) - 1u) | neg) < 0x3F7FFFFFu;
}

// Watertight ray/triangle test (Woop, Benthin and Wald, JCGT 2013) in FP32 on a triangle given by its three
// vertices: vertices relative to the origin, sheared so the ray runs along +z, 2D edge functions (recomputed
// in FP64 when one is exactly zero, so shared edges are decided consistently), a crossing when all three have
// one sign; det = (U + V) + W, T = (U Az + V Bz) + W Cz, t = T rcp(det), u = V rcp(det), v = W rcp(det).
// Returns whether the ray's line crosses the triangle at t > 0.
__device__ inline bool rc_wt(const TravRay& r, float ax, float ay, float az, float bx, float by, float bz, float cx,
                             float cy, float cz, float& t, float& u, float& v)
{
    const float A0 = ax - r.o[0], A1 = ay - r.o[1], A2 = az - r.o[2];
    const float B0 = bx - r.o[0], B1 = by - r.o[1], B2 = bz - r.o[2];
    const float C0 = cx - r.o[0], C1 = cy - r.o[1], C2 = cz - r.o[2];
    const float Akz = rc_pick(A0, A1, A2, r.kz), Bkz = rc_pick(B0, B1, B2, r.kz), Ckz = rc_pick(C0, C1, C2, r.kz);
    float p, q;
    p = r.sx * Akz; const float Ax = rc_pick(A0, A1, A2, r.kx) - p;
    p = r.sy * Akz; const float Ay = rc_pick(A0, A1, A2, r.ky) - p;
    p = r.sx * Bkz; const float Bx = rc_pick(B0, B1, B2, r.kx) - p;
    p = r.sy * Bkz; const float By = rc_pick(B0, B1, B2, r.ky) - p;
    p = r.sx * Ckz; const float Cx = rc_pick(C0, C1, C2, r.kx) - p;
    p = r.sy * Ckz; const float Cy = rc_pick(C0, C1, C2, r.ky) - p;
    p = Cx * By; q = Cy * Bx; float U = p - q;
    p = Ax * Cy; q = Ay * Cx; float V = p - q;
    p = Bx * Ay; q = By * Ax; float W = p - q;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = U + V;
    det = det + W;
    if (det == 0.0f) return false;
    const float Az = r.sz * Akz, Bz = r.sz * Bkz, Cz = r.sz * Ckz;
    p = U * Az;
    q = V * Bz;
    float T = p + q;
    p = W * Cz;
    T = T + p;
    const float rcp = __builtin_amdgcn_rcpf(det);
    t = T * rcp;
    u = V * rcp;
    v = W * rcp;
    return t > 0.0f;
}

// rc_wt's arithmetic for the wave kernels (called by whole waves), for a segment: whether the ray crosses the
// triangle at 0 < t < 1.  The FP64 recomputation of the edge functions runs when some lane of the wave has one
// exactly zero, and applies to those lanes; the sign test is min(U, V, W) < 0 < max(U, V, W) on the sign
// bits (-0 and +0 count as zero, as in rc_wt; U, V, W are finite for finite scenes); det = 0 makes t
// infinite or NaN, which fails the range test as rc_wt's det test does; the wave skips the depth once no
// lane is inside all three edges.
__device__ inline bool rc_wt_segment(const TravRay& r, float ax, float ay, float az, float bx, float by, float bz,
                                     float cx, float cy, float cz)
{
    const float A0 = ax - r.o[0], A1 = ay - r.o[1], A2 = az - r.o[2];
    const float B0 = bx - r.o[0], B1 = by - r.o[1], B2 = bz - r.o[2];
    const float C0 = cx - r.o[0], C1 = cy - r.o[1], C2 = cz - r.o[2];
    const float Akz = rc_pick(A0, A1, A2, r.kz), Bkz = rc_pick(B0, B1, B2, r.kz), Ckz = rc_pick(C0, C1, C2, r.kz);
    float p, q;
    p = r.sx * Akz; const float Ax = rc_pick(A0, A1, A2, r.kx) - p;
    p = r.sy * Akz; const float Ay = rc_pick(A0, A1, A2, r.ky) - p;
    p = r.sx * Bkz; const float Bx = rc_pick(B0, B1, B2, r.kx) - p;
    p = r.sy * Bkz; const float By = rc_pick(B0, B1, B2, r.ky) - p;
    p = r.sx * Ckz; const float Cx = rc_pick(C0, C1, C2, r.kx) - p;
    p = r.sy * Ckz; const float Cy = rc_pick(C0, C1, C2, r.ky) - p;
    p = Cx * By; q = Cy * Bx; float U = p - q;
    p = Ax * Cy; q = Ay * Cx; float V = p - q;
    p = Bx * Ay; q = By * Ax; float W = p - q;
    const bool z = U == 0.0f || V == 0.0f || W == 0.0f;
    if (__ballot(z) != 0) {
        const float U2 = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        const float V2 = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        const float W2 = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
        U = z ? U2 : U;
        V = z ? V2 : V;
        W = z ? W2 : W;
    }
    // all ones when one edge function is negative and another positive (x + 0 and 0 - x turn -0 into +0)
    const float mn = fminf(fminf(U, V), W), mx = fmaxf(fmaxf(U, V), W);
    const uint32_t mixed = (uint32_t)((int32_t)__float_as_uint(mn + 0.0f) >> 31) &
                           (uint32_t)((int32_t)__float_as_uint(0.0f - mx) >> 31);
    if (__ballot(mixed == 0u) == 0) return false;
    float det = U + V;
    det = det + W;
    const float Az = r.sz * Akz, Bz = r.sz * Bkz, Cz = r.sz * Ckz;
    p = U * Az;
    q = V * Bz;
    float T = p + q;
    p = W * Cz;
    T = T + p;
    const float t = T * __builtin_amdgcn_rcpf(det);
    return ((__float_as_uint(t) - 1u) | mixed) < 0x3F7FFFFFu;
}

// The triangle test of the scene: Moller-Trumbore on (v0, e1, e2) records, or the watertight test on
// (v0, v1, v2) records.
template <bool WT>
__device__ inline bool rc_tri(const TravRay& r, const float4& A, const float4& B, const float4& C, float& t, float& u,
                              float& v)
{
    if (WT) return rc_wt(r, A.x, A.y, A.z, B.x, B.y, B.z, C.x, C.y, C.z, t, u, v);
    return rc_mt(r, A.x, A.y, A.z, B.x, B.y, B.z, C.x, C.y, C.z, t, u, v);
}

// Test the triangles of the leaf s.cur (FP32, the scene's triangle test), then pop; an any-hit ray ends at its
// first hit (occluded = true, s.cur = RC_STACK_EMPTY).
template <bool TWO = false, bool WT = false, class Stack>
__device__ inline void trav_test_leaf(const DevScene& sc, TravRay& r, TravState& s, Stack& st, bool any,
                                      uint32_t& occluded, uint32_t& tri_tests, TravWorld* w = nullptr)
{
    if (TWO && w->in_blas == 0u) {
        // top-level leaf: enter the instance (map the ray, mark the return point on the stack)
        const DevInst& I = sc.inst[rc_leaf_first(s.cur)];
        rc_map_ray(I.w2o, w->o, w->d, r);
        st.push(s.sp, RC_INST_RETURN, -INFINITY);
        w->in_blas = 1u;
        s.cur = I.root;
        return;
    }
    uint32_t first = rc_leaf_first(s.cur), cnt = rc_leaf_count(s.cur);
    for (uint32_t i = 0; i < cnt; ++i) {
        ++tri_tests;
        const float4* tp = sc.tris + 3 * (size_t)(first + i);
        float4 A = tp[0], B = tp[1], C = tp[2];
        float t, u, v;
        bool hit = rc_tri<WT>(r, A, B, C, t, u, v);
        if (any) {
            if (hit && t < 1.0f) { occluded = 1u; break; }
        } else {
            uint32_t id = __float_as_uint(A.w);
            if (hit && (t < s.best_t || (t == s.best_t && id < s.best_id))) {
                s.best_t = t; s.best_u = u; s.best_v = v; s.best_id = id;
            }
        }
    }
    s.cur = occluded != 0u ? RC_STACK_EMPTY : trav_pop<TWO>(r, s, st, any, w);
}

// Advance every busy lane of the wave: first the lanes standing at an internal node visit nodes, then the
// lanes standing at a leaf test leaves.  NODE_STEPS / LEAF_STEPS bound the rounds of each phase per call (0:
// until no lane stands at a node / leaf).  Unbounded phases run fewer SIMD steps that execute both code paths,
// but a lane that reaches a leaf early then idles until the last lane of the wave has reached one; with the
// traversal latency-bound (each step waits on its node or triangle loads), short phases keep more lanes moving:
// 3 node rounds and 1 leaf round per call took 1080p camera rays on 7.3M triangles from 0.70 to 0.57 ms.  A
// lane's own sequence of visits is the same whatever the other lanes do; only the grouping of the work into
// SIMD steps changes.
template <bool TWO = false, bool WT = false, int NODE_STEPS = 0, int LEAF_STEPS = 0, class Stack>
__device__ inline void trav_advance(const DevScene& sc, TravRay& r, TravState& s, Stack& st, bool busy,
                                    bool any, uint32_t& occluded, uint32_t& node_visits, uint32_t& tri_tests,
                                    TravWorld* w = nullptr)
{
    for (int it = 0;; ++it) {
        bool inner = busy && !rc_is_leaf(s.cur);
        if (__ballot(inner) == 0 || (NODE_STEPS > 0 && it >= NODE_STEPS)) break;
        if (inner) {
            ++node_visits;
            trav_visit_node<TWO>(sc, r, s, st, any, w);
        }
    }
    for (int it = 0;; ++it) {
        bool leaf = busy && s.cur != RC_STACK_EMPTY && rc_is_leaf(s.cur);
        if (__ballot(leaf) == 0 || (LEAF_STEPS > 0 && it >= LEAF_STEPS)) break;
        if (leaf) trav_test_leaf<TWO, WT>(sc, r, s, st, any, occluded, tri_tests, w);
    }
}

// Shadow-ray target for light index j of a shaded point: a point light, or sample j of the rect
// light (Philox counter (pixel, j, 1 + stream, 0)).  Sets the ray (origin os, direction target - os)
// and returns whether it is cast: n . d > 0 and, for the rect light, the light faces the point.
__device__ inline bool rc_shadow_ray(const float* point_light, const float* rect, const float* nL, bool is_rect,
                                     uint32_t pixel, uint32_t j, uint32_t stream, uint32_t seed, uint32_t frame,
                                     const float os[3], const float nf[3], TravRay& r)
{
    float tgt[3];
    if (!is_rect) {
        tgt[0] = point_light[0]; tgt[1] = point_light[1]; tgt[2] = point_light[2];
    } else {
        uint32_t q[4];
        rc_philox(pixel, j, 1u + stream, 0u, seed, frame, q);
        float x1 = rc_unit24(q[0]) - 0.5f, x2 = rc_unit24(q[1]) - 0.5f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float t1 = x1 * rect[3 + a];
            float t2 = x2 * rect[6 + a];
            tgt[a] = (rect[a] + t1) + t2;
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) { r.o[a] = os[a]; r.d[a] = tgt[a] - os[a]; }
    float nd = nf[0] * r.d[0] + nf[1] * r.d[1];
    nd = nd + nf[2] * r.d[2];
    bool ok = nd > 0.0f;
    if (is_rect) {
        float ld = nL[0] * r.d[0] + nL[1] * r.d[1];
        ld = ld + nL[2] * r.d[2];
        ok = ok && ld < 0.0f;
    }
    return ok;
}

// Radiance of one camera sample (FP64), as the shading stage defines it.
__device__ inline float4 rc_shade_sample(const DevScene& sc, const DevCamera& cam, const float* lights, int n_point,
                                         const float* rect, double vis, uint32_t pixel, uint32_t k, uint32_t tri,
                                         uint32_t mask)
{
    Surface S = rc_surface(sc, cam, pixel, k, tri);
    const float* mat = sc.mats + 5 * (size_t)sc.tri_mat[tri];
    double rgb[3] = {0.0, 0.0, 0.0};
    for (int l = 0; l < n_point; ++l) {
        if (!((mask >> l) & 1u)) continue;
        const float* L = lights + 6 * l;
        D3 lp = d3(L[0], L[1], L[2]);
        D3 tl = d3sub(lp, S.p);
        double d2 = d3dot(tl, tl);
        D3 wi = d3nrm(tl);
        double f[3];
        rc_brdf(S.ns, S.wo, wi, mat, f);
        double cosi = fmax(d3dot(S.ns, wi), 0.0);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) rgb[ch] += f[ch] * (double)L[3 + ch] * cosi / d2;
    }
    if (rect) {
        D3 C = d3(rect[0], rect[1], rect[2]);
        D3 eu = d3(rect[3], rect[4], rect[5]), ev = d3(rect[6], rect[7], rect[8]);
        D3 nraw = d3cross(eu, ev);
        double area = sqrt(d3dot(nraw, nraw));
        D3 nL = d3nrm(nraw);
        D3 tl = d3sub(C, S.p);
        double d2 = d3dot(tl, tl);
        D3 wi = d3nrm(tl);
        double cosl = fmax(-d3dot(nL, wi), 0.0);
        double cosi = fmax(d3dot(S.ns, wi), 0.0);
        double f[3];
        rc_brdf(S.ns, S.wo, wi, mat, f);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) rgb[ch] += f[ch] * (double)rect[9 + ch] * area * cosl * cosi / d2 * vis;
    }
    return make_float4((float)rgb[0], (float)rgb[1], (float)rgb[2], 1.0f);
}
