// Ray traversal kernels for gfx950: camera rays (closest hit into the G-buffer) and shadow
// rays (any hit) towards point lights or rectangular-light samples.
//
// Persistent waves: each 64-lane wave keeps its lanes busy from a device work counter.
// A lane owns one work item (a camera sample, or a shaded point with its list of shadow
// rays); when enough lanes of a wave have finished, the idle lanes are refilled together
// (ballot of idle lanes, one atomicAdd for the wave, prefix count for the lane's slot),
// which regroups live rays into full waves without moving ray state.
//
// Traversal: 4-wide BVH, all child boxes of a node in one 128-byte record; ray/box slab
// tests with the octant-selected near/far planes and a conservative far distance; ordered
// descent (nearest child first) for closest hits; per-lane stack of (node, entry distance)
// in LDS with a lane-interleaved global overflow area.  Triangles: Moller-Trumbore in FP32.
#include <algorithm>

#include "rc_trav.h"

namespace {

constexpr int BLOCK = RC_TRACE_BLOCK;
#ifndef RC_SKIP_EMPTY
#define RC_SKIP_EMPTY 1   // the wave walk skips the slab tests of empty child slots 2 and 3
#endif
constexpr int SL = RC_STACK_LDS;
constexpr int REFILL_AT = 40;    // refill once a wave has at most this many busy lanes
constexpr uint32_t ITEM_CHUNK = 256;
constexpr uint32_t RECT_CHUNK = 64;   // packets per chunk dealt to one XCD

enum { MODE_PRIMARY = 0, MODE_POINT = 1, MODE_RECT = 2 };

struct KParams {
    DevScene sc;
    DevCamera cam;
    DevLights L;
    float nL[3];              // unit normal of the rect light (emitting side)
    uint4* gbuf_out;
    const uint4* gbuf_in;
    uint32_t* mask;
    float* vis;
    const float4* setup;      // shadow rays: per sample (origin, 1 | 0 without a hit) and (normal, 0), k_shadow_setup
    TraceWork w;
    uint32_t n_items;
    uint32_t slot;
    uint32_t claim;           // work positions a wave claims with one atomic (set by the launcher)
};

// Positions per claim: large enough that the atomics stay few, small enough that every wave makes about
// `per_wave` claims, so that the last claims of the waves end close together.
inline uint32_t claim_size(uint64_t n_work, int grid, uint32_t per_wave, uint32_t lo, uint32_t hi)
{
    uint64_t waves = (uint64_t)grid * (BLOCK / 64);
    uint64_t c = n_work / (waves * per_wave);
    return (uint32_t)std::min<uint64_t>(hi, std::max<uint64_t>(lo, c));
}

// The flat-tree camera-ray instance is compiled for 6 waves per SIMD (at most 80 registers; 5 waves otherwise),
// which measured 3% faster (0.701 vs 0.724 ms for 1080p camera rays on 7.3M triangles).
template <int MODE, bool TWO, bool WT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(MODE == MODE_PRIMARY && !TWO && !WT ? 6 : 1))) void k_trace(KParams P)
{
    constexpr bool ANY = MODE != MODE_PRIMARY;

    const int tid = threadIdx.x;
    const uint32_t lane = __lane_id();
    const uint32_t glane = blockIdx.x * BLOCK + tid;
    const DevScene sc = P.sc;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    TravStack<SL, BLOCK, !ANY> st{tid, reinterpret_cast<uint2*>(P.w.overflow), P.w.overflow_depth, P.w.n_lanes,
                                   glane, P.w.error_flag};

    int state = 0;                    // 0 idle, 1 tracing
    uint32_t px = 0, pk = 0;          // pixel and sample of the current item
    uint32_t j = 0, acc = 0;          // shadow: current light / light sample, result accumulator
    uint32_t n_rays = 0;
    float os[3] = {0, 0, 0}, nf[3] = {0, 0, 0};
    TravRay ray;
    TravState ts;
    TravWorld tw;
    TravWorld* twp = TWO ? &tw : nullptr;
    const uint32_t root = TWO ? sc.tlas_root : 0u;
    bool queue_empty = false;
    const XcdQueue<ITEM_CHUNK> queue(P.w.counters, P.slot, P.n_items);
    uint32_t pool_next = 0, pool_end = 0;   // wave-uniform range of claimed, not yet started positions
    uint32_t rays_cast = 0, node_visits = 0, tri_tests = 0;

    // shadow items: set up the next ray that is cast, or return false
    auto next_shadow_ray = [&]() -> bool {
        while (j < n_rays) {
            if (rc_shadow_ray(P.L.point[MODE == MODE_POINT ? j : 0], P.L.rect, P.nL, MODE == MODE_RECT, px, j,
                              P.L.area_stream, P.cam.seed, P.cam.frame, os, nf, ray)) {
                trav_begin(ray, ts, root, twp);
                ++rays_cast;
                return true;
            }
            ++j;
        }
        return false;
    };

    auto finish_item = [&]() {
        if (MODE == MODE_POINT) P.mask[(size_t)px * (P.cam.ssaa * P.cam.ssaa) + pk] = acc;
        if (MODE == MODE_RECT) P.vis[px] = (float)acc / (float)n_rays;
    };

    auto start_item = [&](uint32_t item) -> bool {
        if (!rc_item_to_sample(P.cam, item, px, pk)) return false;
        if (MODE == MODE_PRIMARY) {
            rc_camera_ray(P.cam, px, pk, ray.o, ray.d);
            trav_begin(ray, ts, root, twp);
            ++rays_cast;
            return true;
        } else {
            // origin and normal from the setup pass (the FP64 reconstruction stays out of this kernel)
            size_t s = (size_t)px * (P.cam.ssaa * P.cam.ssaa) + pk;
            const float4 a = P.setup[2 * s];
            acc = 0;
            j = 0;
            n_rays = MODE == MODE_POINT ? (uint32_t)P.L.n_point : (uint32_t)P.L.area_samples;
            if (a.w == 0.0f) { finish_item(); return false; }
            const float4 b = P.setup[2 * s + 1];
            os[0] = a.x; os[1] = a.y; os[2] = a.z;
            nf[0] = b.x; nf[1] = b.y; nf[2] = b.z;
            if (next_shadow_ray()) return true;
            finish_item();
            return false;
        }
    };

    // a ray ended: record it; returns true when the lane continues with another ray of its item
    auto end_ray = [&](bool occluded) -> bool {
        if (MODE == MODE_PRIMARY) {
            P.gbuf_out[(size_t)px * (P.cam.ssaa * P.cam.ssaa) + pk] =
                make_uint4(ts.best_id, __float_as_uint(ts.best_t), __float_as_uint(ts.best_u), __float_as_uint(ts.best_v));
            return false;
        } else {
            if (!occluded) acc += (MODE == MODE_POINT) ? (1u << j) : 1u;
            ++j;
            if (next_shadow_ray()) return true;
            finish_item();
            return false;
        }
    };

    for (;;) {
        // ---- refill idle lanes from the work counter
        for (;;) {
            uint64_t need = __ballot(state == 0);
            if (need == 0 || queue_empty) break;
            if (pool_next == pool_end) {   // the wave's pool is used up: claim the next POOL positions
                pool_next = queue.claim(P.claim);
                pool_end = pool_next + P.claim;
                if (queue.exhausted(pool_next)) { queue_empty = true; break; }
            }
            const uint32_t cnt = min((uint32_t)__popcll(need), pool_end - pool_next);
            const uint32_t base = pool_next;
            pool_next += cnt;
            if (state == 0) {
                uint32_t rank = (uint32_t)__popcll(need & below);
                uint64_t my = queue.at(base + rank);
                if (rank < cnt && my < P.n_items && start_item((uint32_t)my)) state = 1;
            }
            if (queue.exhausted(pool_next)) queue_empty = true;
        }
        if (__ballot(state == 1) == 0) break;

        // ---- traversal: node phase then leaf phase for all busy lanes, until enough lanes are idle
        for (;;) {
            uint32_t occluded = 0u;
            trav_advance<TWO, WT, 3, 1>(sc, ray, ts, st, state == 1, ANY, occluded, node_visits, tri_tests, twp);
            if (state == 1 && ts.cur == RC_STACK_EMPTY) {
                if (!end_ray(occluded != 0u)) state = 0;
            }
            uint32_t n_act = (uint32_t)__popcll(__ballot(state == 1));
            if (n_act == 0) break;
            if (!queue_empty && n_act <= (uint32_t)REFILL_AT) break;
        }
    }

    if (P.w.ray_count) {
        unsigned long long cnt[3] = {rays_cast, node_visits, tri_tests};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            unsigned long long v = cnt[q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) atomicAdd(P.w.ray_count + 2 * q, v);
        }
    }
}

// Rect-light visibility with one ray per lane.  The N light samples of a pixel occupy N consecutive
// ray slots, so a wave traces the samples of one pixel (N >= 64) or of 64/N neighbouring pixels
// together: its lanes start from the same point towards nearby targets and mostly fetch the same
// nodes.  A wave claims 64 ray slots at a time, advances them to completion, and adds the visible
// count of each pixel segment (ballot + popcount) to a per-pixel counter.
template <bool TWO, bool WT>
__global__ __launch_bounds__(BLOCK) void k_rect_packets(KParams P, uint32_t* counts)
{
    const int tid = threadIdx.x;
    const uint32_t lane = __lane_id();
    const uint32_t glane = blockIdx.x * BLOCK + tid;
    const DevScene sc = P.sc;
    TravStack<SL, BLOCK, false> st{tid, reinterpret_cast<uint2*>(P.w.overflow), P.w.overflow_depth, P.w.n_lanes,
                                   glane, P.w.error_flag};
    const uint64_t N = (uint64_t)P.L.area_samples;
    const uint64_t total = (uint64_t)P.n_items * N;
    const uint64_t n_blocks = (total + 63) / 64;
    uint32_t rays_cast = 0, node_visits = 0, tri_tests = 0;
    TravRay ray;
    TravState ts;
    TravWorld tw;
    TravWorld* twp = TWO ? &tw : nullptr;
    const XcdQueue<RECT_CHUNK> queue(P.w.counters, P.slot, n_blocks);
    uint32_t pos = 0, pos_end = 0;   // wave-uniform range of claimed positions
    for (;;) {
        if (pos == pos_end) {
            pos = queue.claim(P.claim);
            pos_end = pos + P.claim;
        }
        const uint32_t j = pos++;
        if (queue.exhausted(j)) break;
        const uint64_t blk = queue.at(j);
        if (blk >= n_blocks) continue;
        const uint64_t r = (uint64_t)blk * 64 + lane;
        const uint32_t item = (uint32_t)(r / N), k = (uint32_t)(r % N);
        uint32_t px = 0, pk = 0;
        const bool in_image = r < total && rc_item_to_sample(P.cam, item, px, pk);
        bool busy = false;
        if (in_image) {
            const float4 a = P.setup[2 * (size_t)px];   // one sample per pixel: setup entry px
            if (a.w != 0.0f) {
                const float4 b = P.setup[2 * (size_t)px + 1];
                float os[3] = {a.x, a.y, a.z};
                float nf[3] = {b.x, b.y, b.z};
                busy = rc_shadow_ray(P.L.point[0], P.L.rect, P.nL, true, px, k, P.L.area_stream, P.cam.seed,
                                     P.cam.frame, os, nf, ray);
                if (busy) {
                    trav_begin(ray, ts, TWO ? sc.tlas_root : 0u, twp);
                    ++rays_cast;
                }
            }
        }
        uint32_t occluded = 0u;
        while (__ballot(busy && ts.cur != RC_STACK_EMPTY) != 0)
            trav_advance<TWO, WT, 3, 1>(sc, ray, ts, st, busy, true, occluded, node_visits, tri_tests, twp);
        const uint64_t vis = __ballot(busy && occluded == 0u);
        if (in_image && (lane == 0 || k == 0)) {
            uint32_t end = (uint32_t)min<uint64_t>(64, lane + (N - k));
            uint64_t seg = (end >= 64 ? ~0ull : ((1ull << end) - 1)) & ~((1ull << lane) - 1);
            uint32_t c = (uint32_t)__popcll(vis & seg);
            if (c) atomicAdd(counts + px, c);
        }
    }
    if (P.w.ray_count) {
        unsigned long long cnt[3] = {rays_cast, node_visits, tri_tests};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            unsigned long long v = cnt[q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) atomicAdd(P.w.ray_count + 2 * q, v);
        }
    }
}

// Per-sample shadow-ray setup of the shadow passes: (origin, 1) and (unit normal, 0) in FP32 from the
// FP64 surface reconstruction, or (0, 0, 0, 0) for samples without a primary hit.  Keeps the FP64 code
// (and its registers) out of the traversal kernels, wave-uniform and per-lane alike.
__global__ __launch_bounds__(256) void k_shadow_setup(DevScene sc, DevCamera cam, const uint4* gbuf, uint32_t n_samples,
                                                      float4* setup)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_samples) return;
    const uint32_t spp = (uint32_t)(cam.ssaa * cam.ssaa);
    const uint4 h = gbuf[i];
    float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b = a;
    if (h.x != RC_NO_HIT) {
        Surface S = rc_surface(sc, cam, i / spp, i % spp, h.x);
        D3 O = rc_shadow_origin(S);
        a = make_float4((float)O.x, (float)O.y, (float)O.z, 1.0f);
        b = make_float4((float)S.n.x, (float)S.n.y, (float)S.n.z, 0.0f);
    }
    setup[2 * (size_t)i] = a;
    setup[2 * (size_t)i + 1] = b;
}

// Rect-light visibility, wave-uniform traversal.  The 64 ray slots of a wave (the samples of one
// pixel, or the N samples of each of 64 / N neighbouring pixels) walk the BVH together: the wave visits a node
// when any of its live rays hits one of its boxes, so node and triangle records are read once per wave
// through the scalar cache, and the traversal stack is wave-uniform, held one entry per lane in one
// register (64 entries) or two (128; the host picks the smallest that holds 3 x depth + 1 entries).  Each lane still
// tests its own ray against every box and triangle the wave visits, with the same FP32 arithmetic as
// the per-lane traversal; a triangle that a lane's own boxes would not have led to can only report a
// true crossing, so the occlusion result of every ray is the one the per-lane traversal finds.
// Children that some live ray enters are visited nearest first by lane 0's entry distance.  The
// distances are non-negative, so their bit patterns order like the values; the two lowest bits carry the
// child's slot instead (children whose keys differ only there are ordered by slot), so the keys sort with
// plain minima and maxima on the scalar unit and the child word is then taken by slot.  When all live
// rays share a direction octant (the usual case for a small light), the near and far plane blocks of the
// node are loaded at byte offsets picked by the octant; otherwise each lane picks its own planes.
typedef float rc_v4f __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) rc_v4f rc_const_v4f;
typedef float rc_v8f __attribute__((ext_vector_type(8)));
typedef const __attribute__((address_space(4))) rc_v8f rc_const_v8f;
typedef uint32_t rc_v4u __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) rc_v4u rc_const_v4u;

extern "C" __device__ uint32_t __ockl_wfred_max_u32(uint32_t);   // ROCm device library: wavefront maximum
// the compiler intrinsic behind v_writelane_b32 (no clang builtin in this toolchain): returns `old` with lane
// `lane` (wave-uniform) replaced by the wave-uniform `value`
extern "C" __device__ int rc_writelane(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

#define RC_KEY_MISS 0x7F800000u   // keys >= this: no live ray enters the child

// The child's key when any lane enters it: lane 0's entry distance (every lane computes one, hit or not, and
// the rays of a wave start at or near one point, so it orders the children about as any hitting lane's would),
// clamped below the miss key; otherwise a miss key.  The entry distance is >= 0, so its bits order like the
// value, and the two low bits carry the slot.  This replaces a select per lane and a find-first-hitting-lane
// by scalar operations (the wave kernel is bound by vector issue), and measured slightly fewer node visits.
__device__ inline uint32_t wave_key(bool hit, float t0, uint32_t slot)
{
    const uint64_t m = __ballot(hit);
    const uint32_t k0 = min((uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(t0), 0) & 0x7FFFFFFCu, 0x7F7FFFFCu);
    return m != 0 ? (k0 | slot) : (RC_KEY_MISS | slot);
}

// Slab test of the wave kernels for a segment 0 <= t <= 1: the entry distance, clamped to [0, 1] in one
// median, against the exit distance.  Against max(entry, 0) <= min(exit, 1) it also accepts boxes that the
// line meets only beyond t = 1 (beyond the light): extra visits, no change in any result, and one vector
// operation less per child.  Finished and idle lanes carry far-plane addends of -inf (wave_mute), so their
// exit distance is -inf (or NaN) and no box accepts them.
__device__ inline bool rc_slab_seg(const TravRay& r, float nx, float ny, float nz, float fx, float fy, float fz,
                                   float& t0)
{
    const float u = fmaxf(fmaxf(fmaf(nx, r.inv[0], r.cn[0]), fmaf(ny, r.inv[1], r.cn[1])), fmaf(nz, r.inv[2], r.cn[2]));
    t0 = __builtin_amdgcn_fmed3f(u, 0.0f, 1.0f);
    const float v = fminf(fminf(fmaf(fx, r.invf[0], r.cf[0]), fmaf(fy, r.invf[1], r.cf[1])), fmaf(fz, r.invf[2], r.cf[2]));
    return t0 <= v;
}

// A lane whose ray is finished (live == 0) takes part in no slab test: its far-plane addends become -inf.  An
// idle lane's traversal constants were never set (set == false): they become 0 first, so that every far
// distance is -inf (or NaN for an infinite plane) and the entry distance finite (or NaN).
__device__ inline void wave_mute(TravRay& r, uint32_t live, bool set)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!set) {
            r.inv[a] = 0.0f;
            r.cn[a] = 0.0f;
            r.invf[a] = 0.0f;
        }
        r.cf[a] = live != 0u ? r.cf[a] : -INFINITY;
    }
}

// CLAMP: rc_slab_seg (finished lanes muted); otherwise rc_slab with bound, 1 for live rays and -1 for finished
// ones, which then never hit (t0 >= 0)
template <bool CLAMP>
__device__ inline void wave_keys_uniform(const rc_v4f& nx, const rc_v4f& fx, const rc_v4f& ny, const rc_v4f& fy,
                                         const rc_v4f& nz, const rc_v4f& fz, const TravRay& ray, float bound,
                                         uint32_t key[4])
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float t0;
        const bool hit = CLAMP ? rc_slab_seg(ray, nx[c], ny[c], nz[c], fx[c], fy[c], fz[c], t0)
                                 : rc_slab(ray, nx[c], ny[c], nz[c], fx[c], fy[c], fz[c], bound, t0);
        key[c] = wave_key(hit, t0, (uint32_t)c);
    }
}

// As wave_keys_uniform, for a node whose child words `chw` (wave-uniform) are known: slots 2 and 3 that hold no
// child get a miss key without their slab tests (a uniform branch), since an empty slot's box never hits.
template <bool CLAMP>
__device__ inline void wave_keys_uniform_skip(const rc_v4f& nx, const rc_v4f& fx, const rc_v4f& ny, const rc_v4f& fy,
                                              const rc_v4f& nz, const rc_v4f& fz, const TravRay& ray, float bound,
                                              const uint32_t chw[4], uint32_t key[4])
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (RC_SKIP_EMPTY && c >= 2 && chw[c] == RC_EMPTY_CHILD) {
            key[c] = RC_KEY_MISS | (uint32_t)c;
            continue;
        }
        float t0;
        const bool hit = CLAMP ? rc_slab_seg(ray, nx[c], ny[c], nz[c], fx[c], fy[c], fz[c], t0)
                                 : rc_slab(ray, nx[c], ny[c], nz[c], fx[c], fy[c], fz[c], bound, t0);
        key[c] = wave_key(hit, t0, (uint32_t)c);
    }
}

template <bool CLAMP>
__device__ inline void wave_keys_mixed(const rc_v4f& lx, const rc_v4f& hx, const rc_v4f& ly, const rc_v4f& hy,
                                       const rc_v4f& lz, const rc_v4f& hz, const TravRay& ray, float bound,
                                       uint32_t key[4])
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float nx = ray.inv[0] >= 0.0f ? lx[c] : hx[c], fx = ray.inv[0] >= 0.0f ? hx[c] : lx[c];
        const float ny = ray.inv[1] >= 0.0f ? ly[c] : hy[c], fy = ray.inv[1] >= 0.0f ? hy[c] : ly[c];
        const float nz = ray.inv[2] >= 0.0f ? lz[c] : hz[c], fz = ray.inv[2] >= 0.0f ? hz[c] : lz[c];
        float t0;
        const bool hit = CLAMP ? rc_slab_seg(ray, nx, ny, nz, fx, fy, fz, t0) : rc_slab(ray, nx, ny, nz, fx, fy, fz, bound, t0);
        key[c] = wave_key(hit, t0, (uint32_t)c);
    }
}

// Two-level structures: at a top-level leaf every lane maps its ray into the instance (rc_map_ray), the
// wave pushes an end marker and descends into the instance's tree; popping the marker restores the world
// rays (and the wave's octant).
// The walk of wave_occluded.  BIG: the stack spans two registers (128 entries); otherwise one (64 entries,
// when 3 x depth + 1 <= 64).
// OCT: 0..7, every busy ray in that direction octant (fixed for the whole walk, as in flat trees): the node's
// plane blocks come with three 32-byte loads at constant offsets and the near/far choice is made when
// compiling; 8: mixed octants (each lane picks its planes); -1: decided at run time, per instance for
// two-level structures (the mapped rays' octant changes at each instance).
template <bool WT, bool BIG, bool CLAMP, bool COUNT>
__device__ __attribute__((always_inline)) inline uint32_t wave_walk_flat(const DevScene& sc, const char* nodes_b,
                                                                       const char* tris_b, TravRay& ray, bool busy,
                                                                       uint32_t& node_visits, uint32_t& tri_tests,
                                                                       uint32_t* error_flag, uint32_t root);

// CLAMP: the slab test rc_slab_seg with muted lanes (flat trees, Moller-Trumbore: 10 vector operations per child
// instead of 12); otherwise rc_slab with a bound per lane (two-level structures and the watertight test, whose
// walks hold more registers and measured slower with the muting)
// COUNT: the walk counts node visits and triangle tests of live lanes (frames timed by stage report them)
template <bool TWO, bool WT, bool BIG, int OCT, bool CLAMP, bool COUNT>
__device__ __attribute__((always_inline)) inline uint32_t wave_walk(const DevScene& sc, const char* nodes_b,
                                                                  const char* tris_b, TravRay& ray, bool busy,
                                                                  uint32_t& node_visits, uint32_t& tri_tests,
                                                                  uint32_t* error_flag, uint32_t root)
{
    const uint32_t lane = __lane_id();
    const uint64_t busy_mask = __ballot(busy);
    uint32_t oct = 0, on0 = 0, on1 = 32, on2 = 64, of0 = 16, of1 = 48, of2 = 80;
    bool uniform_oct = false;
    auto set_octant = [&]() {
        const uint32_t my_oct = (ray.inv[0] < 0.0f ? 1u : 0u) | (ray.inv[1] < 0.0f ? 2u : 0u) |
                                (ray.inv[2] < 0.0f ? 4u : 0u);
        oct = 0;
        if (busy_mask != 0) oct = (uint32_t)__builtin_amdgcn_readlane((int)my_oct, __builtin_ctzll(busy_mask));
        uniform_oct = __ballot(busy && my_oct != oct) == 0;
        // byte offsets of the near- and far-plane blocks (axis a: lo at 32 a, hi at 32 a + 16)
        on0 = (oct & 1u) ? 16u : 0u;
        on1 = (oct & 2u) ? 48u : 32u;
        on2 = (oct & 4u) ? 80u : 64u;
        of0 = on0 ^ 16u;
        of1 = on1 ^ 16u;
        of2 = on2 ^ 16u;
        // opaque to the compiler (no instruction): keeps node + offset in the scalar-offset form of the loads
        asm volatile("" : "+s"(on0), "+s"(on1), "+s"(on2), "+s"(of0), "+s"(of1), "+s"(of2));
    };
    if constexpr (OCT < 0) set_octant();
    float wo[3] = {ray.o[0], ray.o[1], ray.o[2]}, wd[3] = {ray.d[0], ray.d[1], ray.d[2]};   // world ray
    // per-lane state as 32-bit words: occ (an occluder found) and live (busy and not occluded); lanes that
    // are not live take part in no slab test (muted, or bound = -1)
    uint32_t occ = 0u, live = busy ? 1u : 0u;
    float bound = busy ? 1.0f : -1.0f;
    if constexpr (CLAMP) wave_mute(ray, live, busy);
    uint32_t cur = busy_mask != 0 ? (TWO ? sc.tlas_root : root) : RC_STACK_EMPTY;
    int sp = 0;
    uint32_t stk0 = 0, stk1 = 0;   // entry e of the wave's stack lives in lane e % 64 of stk{e / 64}
    // next entry of the wave's stack
    auto pop_next = [&]() -> uint32_t {
        if (sp == 0) return RC_STACK_EMPTY;
        --sp;
        return BIG ? (uint32_t)__builtin_amdgcn_readlane((int)(sp < 64 ? stk0 : stk1), sp & 63)
                   : (uint32_t)__builtin_amdgcn_readlane((int)stk0, sp);
    };
    auto push_entry = [&](uint32_t w) {
        if (sp < 64) {
            stk0 = (uint32_t)rc_writelane((int)w, sp, (int)stk0);
            ++sp;
        } else if (BIG && sp < 128) {
            stk1 = (uint32_t)rc_writelane((int)w, sp - 64, (int)stk1);
            ++sp;
        } else if (lane == 0) {
            *error_flag = 1u;   // beyond the bound the host checked: entry dropped, reported
        }
    };
    while (cur != RC_STACK_EMPTY) {
        if (!rc_is_leaf(cur)) {
            // 32-bit byte offsets into the node array (the host keeps it below 4 GiB for this kernel), so
            // that each block load takes its offset in a scalar register
            const uint32_t nofs = cur << 7;
            auto blk = [&](uint32_t off) { return *(rc_const_v4f*)(const void*)(nodes_b + (uint32_t)(nofs + off)); };
            uint32_t key[4];
            if constexpr (OCT >= 0) {
                // axis a: lo[4] then hi[4] in one 32-byte block at 32 a
                const char* np = nodes_b + nofs;
                const rc_v8f X = *(rc_const_v8f*)(const void*)np, Y = *(rc_const_v8f*)(const void*)(np + 32),
                             Z = *(rc_const_v8f*)(const void*)(np + 64);
                const rc_v4f lx = X.lo, hx = X.hi, ly = Y.lo, hy = Y.hi, lz = Z.lo, hz = Z.hi;
                if constexpr (OCT < 8) {
                    const rc_v4u cw = *(rc_const_v4u*)(const void*)(np + 96);
                    const uint32_t cws[4] = {cw[0], cw[1], cw[2], cw[3]};
                    wave_keys_uniform_skip<CLAMP>((OCT & 1) ? hx : lx, (OCT & 1) ? lx : hx, (OCT & 2) ? hy : ly,
                                           (OCT & 2) ? ly : hy, (OCT & 4) ? hz : lz, (OCT & 4) ? lz : hz, ray, bound,
                                           cws, key);
                } else
                    wave_keys_mixed<CLAMP>(lx, hx, ly, hy, lz, hz, ray, bound, key);
            } else if (uniform_oct) {
                wave_keys_uniform<CLAMP>(blk(on0), blk(of0), blk(on1), blk(of1), blk(on2), blk(of2), ray, bound, key);
            } else {
                wave_keys_mixed<CLAMP>(blk(0), blk(16), blk(32), blk(48), blk(64), blk(80), ray, bound, key);
            }
            if constexpr (COUNT) node_visits += live;
#define RC_CS(a, b)                                                                   \
{                                                                                 \
    const uint32_t lo = min(key[a], key[b]), hi = max(key[a], key[b]);            \
    key[a] = lo; key[b] = hi;                                                     \
}
            RC_CS(0, 1) RC_CS(2, 3) RC_CS(0, 2) RC_CS(1, 3) RC_CS(1, 2)
#undef RC_CS
            const rc_v4u chw = OCT >= 0 ? *(rc_const_v4u*)(const void*)(nodes_b + nofs + 96u)
                                        : *(rc_const_v4u*)(const void*)(nodes_b + (uint32_t)(nofs + 96u));
            const uint64_t c01 = ((uint64_t)chw[1] << 32) | chw[0], c23 = ((uint64_t)chw[3] << 32) | chw[2];
            auto child = [&](uint32_t k) {
                const uint64_t pr = (k & 2u) ? c23 : c01;
                return (k & 1u) ? (uint32_t)(pr >> 32) : (uint32_t)pr;
            };
            if (sp <= 61) {
                // room for the (at most 3) pushes of this node in the first stack register
#pragma unroll
                for (int c = 3; c >= 1; --c)
                    if (key[c] < RC_KEY_MISS) {
                        stk0 = (uint32_t)rc_writelane((int)child(key[c]), sp, (int)stk0);
                        ++sp;
                    }
            } else {
#pragma unroll
                for (int c = 3; c >= 1; --c)
                    if (key[c] < RC_KEY_MISS) push_entry(child(key[c]));
            }
            cur = key[0] < RC_KEY_MISS ? child(key[0]) : pop_next();
        } else if (TWO) {
            // top-level leaf: every ray mapped into the instance, whose tree the flat walk takes (compiled for
            // the mapped rays' octant, with a stack of its own) for the rays still live; then back to world
            // space
            rc_const_v4f* ip = (rc_const_v4f*)(const void*)(sc.inst + rc_leaf_first(cur));
            const rc_v4f q0 = ip[0], q1 = ip[1], q2 = ip[2], q3 = ip[3];
            const float W[12] = {q0[0], q0[1], q0[2], q0[3], q1[0], q1[1], q1[2], q1[3],
                                 q2[0], q2[1], q2[2], q2[3]};
            rc_map_ray(W, wo, wd, ray);
            const uint32_t ob = wave_walk_flat<WT, false, false, COUNT>(sc, nodes_b, tris_b, ray, live != 0u, node_visits,
                                                          tri_tests, error_flag, __float_as_uint(q3[0]));
            occ |= ob;
            live &= ob ^ 1u;
#pragma unroll
            for (int a = 0; a < 3; ++a) { ray.o[a] = wo[a]; ray.d[a] = wd[a]; }
            rc_ray_inv(ray);
            bound = live != 0u ? bound : -1.0f;
            cur = __ballot(live != 0u) == 0 ? RC_STACK_EMPTY : pop_next();
        } else {
            // every lane tests every triangle of the leaf, without lane branches: a finished lane only
            // repeats work (its flag stays set; idle lanes' flags are never read), and the counter
            // takes the tests of live lanes
            const uint32_t first = rc_leaf_first(cur), cnt = rc_leaf_count(cur);
            const uint32_t tofs = first * 48u;   // 32-bit byte offset (the host keeps the array below 4 GiB)
            uint32_t o = occ;
            for (uint32_t i = 0; i < cnt; ++i) {
                rc_const_v4f* tp = (rc_const_v4f*)(const void*)(tris_b + (uint32_t)(tofs + 48u * i));
                const rc_v4f A = tp[0], B = tp[1], C = tp[2];
                if constexpr (COUNT) tri_tests += live & (o ^ 1u);
                const bool hit = WT ? rc_wt_segment(ray, A.x, A.y, A.z, B.x, B.y, B.z, C.x, C.y, C.z)
                                    : rc_mt_segment(ray, A.x, A.y, A.z, B.x, B.y, B.z, C.x, C.y, C.z);
                o |= hit ? 1u : 0u;
            }
            occ = o;
            live &= o ^ 1u;
            if constexpr (CLAMP) wave_mute(ray, live, true);
            else bound = live != 0u ? bound : -1.0f;
            cur = __ballot(live != 0u) == 0 ? RC_STACK_EMPTY : pop_next();
        }
        cur = __builtin_amdgcn_readfirstlane(cur);
    }
    return occ;
}

// Any-hit traversal of the segments o + t d, 0 <= t <= 1, of a wave's rays (called by all 64 lanes; busy
// lanes hold a ray whose traversal constants rc_ray_inv set): returns 1 in the lanes whose segment is
// occluded.  Flat trees: one walk specialised for the wave's octant, or for mixed octants.
template <bool TWO, bool WT, bool BIG, bool COUNT>
__device__ __attribute__((always_inline)) inline uint32_t wave_occluded(const DevScene& sc, const char* nodes_b,
                                                                      const char* tris_b, TravRay& ray, bool busy,
                                                                      uint32_t& node_visits, uint32_t& tri_tests,
                                                                      uint32_t* error_flag)
{
    if constexpr (TWO)
        return wave_walk<TWO, WT, BIG, -1, false, COUNT>(sc, nodes_b, tris_b, ray, busy, node_visits, tri_tests, error_flag,
                                                        0u);
    else
        return wave_walk_flat<WT, BIG, !WT, COUNT>(sc, nodes_b, tris_b, ray, busy, node_visits, tri_tests, error_flag, 0u);
}

// The flat walk from node `root`, compiled once per direction octant of the busy rays and once for mixed
// octants.  For two-level structures it walks an instance's tree with a one-register stack: the host takes
// the wave kernels only when 3 x (deepest instance tree + 24) + 2 <= 128, so an instance tree is at most 18
// levels deep and its walk needs at most 55 stack entries.
template <bool WT, bool BIG, bool CLAMP, bool COUNT>
__device__ __attribute__((always_inline)) inline uint32_t wave_walk_flat(const DevScene& sc, const char* nodes_b,
                                                                       const char* tris_b, TravRay& ray, bool busy,
                                                                       uint32_t& node_visits, uint32_t& tri_tests,
                                                                       uint32_t* error_flag, uint32_t root)
{
#define RC_WALK(o) \
    wave_walk<false, WT, BIG, o, CLAMP, COUNT>(sc, nodes_b, tris_b, ray, busy, node_visits, tri_tests, error_flag, root)
    const uint64_t busy_mask = __ballot(busy);
    const uint32_t my_oct = (ray.inv[0] < 0.0f ? 1u : 0u) | (ray.inv[1] < 0.0f ? 2u : 0u) |
                            (ray.inv[2] < 0.0f ? 4u : 0u);
    const uint32_t oct = busy_mask != 0
                             ? (uint32_t)__builtin_amdgcn_readlane((int)my_oct, __builtin_ctzll(busy_mask))
                             : 0u;
    if (__ballot(busy && my_oct != oct) != 0) return RC_WALK(8);
    switch (oct) {
    case 0: return RC_WALK(0);
    case 1: return RC_WALK(1);
    case 2: return RC_WALK(2);
    case 3: return RC_WALK(3);
    case 4: return RC_WALK(4);
    case 5: return RC_WALK(5);
    case 6: return RC_WALK(6);
    default: return RC_WALK(7);
    }
#undef RC_WALK
}

template <bool TWO, bool WT, bool BIG, bool COUNT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(TWO || WT ? 1 : 8))) void k_rect_wave(KParams P, uint32_t* counts, const float4* setup)
{
    const uint32_t lane = __lane_id();
    const DevScene sc = P.sc;
    const uint64_t N = (uint64_t)P.L.area_samples;
    const uint64_t total = (uint64_t)P.n_items * N;
    const uint64_t n_blocks = (total + 63) / 64;
    uint32_t rays_cast = 0, node_visits = 0, tri_tests = 0;
    const char* nodes_b = (const char*)(const void*)sc.nodes;
    const char* tris_b = (const char*)(const void*)sc.tris;
    const XcdQueue<RECT_CHUNK> queue(P.w.counters, P.slot, n_blocks);
    uint32_t pos = 0, pos_end = 0;   // wave-uniform range of claimed positions
    for (;;) {
        if (pos == pos_end) {
            pos = queue.claim(P.claim);
            pos_end = pos + P.claim;
        }
        const uint32_t j = pos++;
        if (queue.exhausted(j)) break;
        const uint64_t blk = queue.at(j);
        if (blk >= n_blocks) continue;
        const uint64_t r = (uint64_t)blk * 64 + lane;
        const uint32_t item = (uint32_t)(r / N), k = (uint32_t)(r % N);
        uint32_t px = 0, pk = 0;
        const bool in_image = r < total && rc_item_to_sample(P.cam, item, px, pk);
        TravRay ray;
        bool busy = false;
        if (in_image) {
            const float4 a = setup[2 * (size_t)px], b = setup[2 * (size_t)px + 1];
            if (a.w != 0.0f) {
                float os[3] = {a.x, a.y, a.z}, nf[3] = {b.x, b.y, b.z};
                busy = rc_shadow_ray(P.L.point[0], P.L.rect, P.nL, true, px, k, P.L.area_stream, P.cam.seed,
                                     P.cam.frame, os, nf, ray);
                if (busy) {
                    rc_ray_inv(ray);
                    ++rays_cast;
                }
            }
        }
        const uint32_t occ = wave_occluded<TWO, WT, BIG, COUNT>(sc, nodes_b, tris_b, ray, busy, node_visits, tri_tests,
                                                         P.w.error_flag);
        const uint64_t vis = __ballot(busy && occ == 0u);
        if (in_image && (lane == 0 || k == 0)) {
            uint32_t end = (uint32_t)min<uint64_t>(64, lane + (N - k));
            uint64_t seg = (end >= 64 ? ~0ull : ((1ull << end) - 1)) & ~((1ull << lane) - 1);
            uint32_t c = (uint32_t)__popcll(vis & seg);
            if (c) atomicAdd(counts + px, c);
        }
    }
    if (P.w.ray_count) {
        unsigned long long cnt[3] = {rays_cast, node_visits, tri_tests};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            unsigned long long v = cnt[q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) atomicAdd(P.w.ray_count + 2 * q, v);
        }
    }
}

// Point-light shadow rays, wave-uniform traversal.  The 64 lanes of a wave hold 64 consecutive samples
// (neighbouring pixels); the wave walks the tree once per light, each lane casting its sample's segment to
// that light where the light lies above the surface, with the same tests and results as the per-lane kernel.
// Mask bit l of a sample: the ray to light l is cast and not occluded.
template <bool TWO, bool WT, bool BIG, bool COUNT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(TWO || WT ? 1 : 8))) void k_point_wave(KParams P, const float4* setup)
{
    const uint32_t lane = __lane_id();
    const DevScene sc = P.sc;
    const uint32_t spp = (uint32_t)(P.cam.ssaa * P.cam.ssaa);
    const uint64_t n_blocks = ((uint64_t)P.n_items + 63) / 64;
    uint32_t rays_cast = 0, node_visits = 0, tri_tests = 0;
    const char* nodes_b = (const char*)(const void*)sc.nodes;
    const char* tris_b = (const char*)(const void*)sc.tris;
    const XcdQueue<RECT_CHUNK> queue(P.w.counters, P.slot, n_blocks);
    uint32_t pos = 0, pos_end = 0;   // wave-uniform range of claimed positions
    for (;;) {
        if (pos == pos_end) {
            pos = queue.claim(P.claim);
            pos_end = pos + P.claim;
        }
        const uint32_t j = pos++;
        if (queue.exhausted(j)) break;
        const uint64_t blk = queue.at(j);
        if (blk >= n_blocks) continue;
        const uint64_t item = blk * 64 + lane;
        uint32_t px = 0, pk = 0;
        const bool in_image = item < P.n_items && rc_item_to_sample(P.cam, (uint32_t)item, px, pk);
        const size_t smp = (size_t)px * spp + pk;
        float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b = a;
        if (in_image) {
            a = setup[2 * smp];
            b = setup[2 * smp + 1];
        }
        float os[3] = {a.x, a.y, a.z}, nf[3] = {b.x, b.y, b.z};
        uint32_t mask = 0;
        for (int l = 0; l < P.L.n_point; ++l) {
            TravRay ray;
            bool busy = false;
            if (a.w != 0.0f) {
                busy = rc_shadow_ray(P.L.point[l], P.L.rect, P.nL, false, px, (uint32_t)l, P.L.area_stream,
                                     P.cam.seed, P.cam.frame, os, nf, ray);
                if (busy) {
                    rc_ray_inv(ray);
                    ++rays_cast;
                }
            }
            const uint32_t occ = wave_occluded<TWO, WT, BIG, COUNT>(sc, nodes_b, tris_b, ray, busy, node_visits, tri_tests,
                                                             P.w.error_flag);
            if (busy && occ == 0u) mask |= 1u << l;
        }
        if (in_image) P.mask[smp] = mask;
    }
    if (P.w.ray_count) {
        unsigned long long cnt[3] = {rays_cast, node_visits, tri_tests};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            unsigned long long v = cnt[q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) atomicAdd(P.w.ray_count + 2 * q, v);
        }
    }
}

// Camera rays, wave-uniform closest-hit traversal.  The 64 samples of a packet (an 8x8-pixel tile, or 4x4
// pixels x 4 samples) share the eye point and walk the BVH together, reading nodes and triangles once per
// wave through the scalar cache; every lane keeps its own closest hit (t, then the smaller id) and tests
// only what its own bound allows.  A child that any lane's box test accepts is pushed with a bound shared
// by all lanes: the squared distance from the eye to its box, a lower bound on every lane's entry distance.
// A popped entry is skipped when that bound exceeds the largest closest-hit distance of the wave (with a
// relative margin of 1e-5 that covers the FP32 rounding of the slab tests and of |d| = 1).  Results equal
// the per-lane traversal's: extra triangle tests can only report true crossings.
template <bool WT>
__global__ __launch_bounds__(BLOCK) void k_primary_wave(KParams P)
{
    const uint32_t lane = __lane_id();
    const DevScene sc = P.sc;
    const uint32_t n_packets = (P.n_items + 63) / 64;
    const uint32_t KEY_MISS = 0x7F800000u;
    const float ex = P.cam.eye[0], ey = P.cam.eye[1], ez = P.cam.eye[2];
    uint32_t rays_cast = 0, node_visits = 0, tri_tests = 0;
    const XcdQueue<RECT_CHUNK> queue(P.w.counters, P.slot, n_packets);
    uint32_t pos = 0, pos_end = 0;
    for (;;) {
        if (pos == pos_end) {
            pos = queue.claim(P.claim);
            pos_end = pos + P.claim;
        }
        const uint32_t j = pos++;
        if (queue.exhausted(j)) break;
        const uint64_t blk = queue.at(j);
        if (blk >= n_packets) continue;
        const uint32_t item = (uint32_t)blk * 64 + lane;
        uint32_t px = 0, pk = 0;
        const bool valid = item < P.n_items && rc_item_to_sample(P.cam, item, px, pk);
        TravRay ray;
        ray.o[0] = ex; ray.o[1] = ey; ray.o[2] = ez;
        ray.d[0] = 1.0f; ray.d[1] = 0.0f; ray.d[2] = 0.0f;
        float best_t = -INFINITY, best_u = 0.0f, best_v = 0.0f;   // invalid lanes accept nothing
        uint32_t best_id = RC_NO_HIT;
        if (valid) {
            rc_camera_ray(P.cam, px, pk, ray.o, ray.d);
            best_t = INFINITY;
            ++rays_cast;
        }
        rc_ray_inv(ray);
        float wmax = INFINITY;                                    // largest closest-hit distance of the wave
        uint32_t cur = __ballot(valid) != 0 ? 0u : RC_STACK_EMPTY;
        int sp = 0;
        uint32_t stk0 = 0, stk1 = 0, lbs0 = 0, lbs1 = 0;         // entry e: lane e % 64 of {stk,lbs}{e / 64}
        auto pop = [&]() -> uint32_t {
            const float lim = wmax * 1.00001f;
            const float lim2 = lim * lim;
            while (sp > 0) {
                --sp;
                const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)(sp < 64 ? stk0 : stk1), sp & 63);
                const float lb = __uint_as_float(
                    (uint32_t)__builtin_amdgcn_readlane((int)(sp < 64 ? lbs0 : lbs1), sp & 63));
                if (!(lb > lim2)) return w;
            }
            return RC_STACK_EMPTY;
        };
        while (cur != RC_STACK_EMPTY) {
            if (!rc_is_leaf(cur)) {
                rc_const_v4f* np = (rc_const_v4f*)(const void*)(sc.nodes + cur);
                const rc_v4f lx = np[0], hx = np[1], ly = np[2], hy = np[3], lz = np[4], hz = np[5];
                const rc_v4f chf = np[6];
                uint32_t key[4], cw[4];
                float lb[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    float nx = ray.inv[0] >= 0.0f ? lx[c] : hx[c], fx = ray.inv[0] >= 0.0f ? hx[c] : lx[c];
                    float ny = ray.inv[1] >= 0.0f ? ly[c] : hy[c], fy = ray.inv[1] >= 0.0f ? hy[c] : ly[c];
                    float nz = ray.inv[2] >= 0.0f ? lz[c] : hz[c], fz = ray.inv[2] >= 0.0f ? hz[c] : lz[c];
                    float t0;
                    const bool hit = rc_slab(ray, nx, ny, nz, fx, fy, fz, best_t, t0);
                    uint64_t m = __ballot(hit);
                    uint32_t k = KEY_MISS;
                    if (m != 0) {
                        int first = __builtin_ctzll(m);
                        k = (uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(t0), first) & 0x7FFFFFFFu;
                    }
                    key[c] = k;
                    cw[c] = __float_as_uint(chf[c]);
                    // squared distance from the eye to the child box (uniform)
                    float qx = fmaxf(fmaxf(lx[c] - ex, ex - hx[c]), 0.0f);
                    float qy = fmaxf(fmaxf(ly[c] - ey, ey - hy[c]), 0.0f);
                    float qz = fmaxf(fmaxf(lz[c] - ez, ez - hz[c]), 0.0f);
                    float q2 = qx * qx + qy * qy;
                    lb[c] = q2 + qz * qz;
                }
                if (valid) ++node_visits;
#define RC_CS(a, b)                                                                   \
    {                                                                                 \
        bool sw = key[b] < key[a];                                                    \
        uint32_t ka = sw ? key[b] : key[a], kb = sw ? key[a] : key[b];                \
        uint32_t ca = sw ? cw[b] : cw[a], cb = sw ? cw[a] : cw[b];                    \
        float la = sw ? lb[b] : lb[a], lbb = sw ? lb[a] : lb[b];                      \
        key[a] = ka; key[b] = kb; cw[a] = ca; cw[b] = cb; lb[a] = la; lb[b] = lbb;    \
    }
                RC_CS(0, 1) RC_CS(2, 3) RC_CS(0, 2) RC_CS(1, 3) RC_CS(1, 2)
#undef RC_CS
#pragma unroll
                for (int c = 3; c >= 1; --c) {
                    if (key[c] < KEY_MISS) {
                        if (sp < 64) {
                            stk0 = (int)lane == sp ? cw[c] : stk0;
                            lbs0 = (int)lane == sp ? __float_as_uint(lb[c]) : lbs0;
                            ++sp;
                        } else if (sp < 128) {
                            stk1 = (int)lane == sp - 64 ? cw[c] : stk1;
                            lbs1 = (int)lane == sp - 64 ? __float_as_uint(lb[c]) : lbs1;
                            ++sp;
                        } else if (lane == 0) {
                            *P.w.error_flag = 1u;   // beyond the bound the host checked: entry dropped, reported
                        }
                    }
                }
                cur = key[0] < KEY_MISS ? cw[0] : pop();
            } else {
                const uint32_t first = rc_leaf_first(cur), cnt = rc_leaf_count(cur);
                for (uint32_t i = 0; i < cnt; ++i) {
                    rc_const_v4f* tp = (rc_const_v4f*)(const void*)(sc.tris + 3 * (size_t)(first + i));
                    const rc_v4f A = tp[0], B = tp[1], C = tp[2];
                    if (valid) {
                        ++tri_tests;
                        float t, u, v;
                        bool hit = WT ? rc_wt(ray, A.x, A.y, A.z, B.x, B.y, B.z, C.x, C.y, C.z, t, u, v)
                                      : rc_mt(ray, A.x, A.y, A.z, B.x, B.y, B.z, C.x, C.y, C.z, t, u, v);
                        const uint32_t id = __float_as_uint(A.w);
                        if (hit && (t < best_t || (t == best_t && id < best_id))) {
                            best_t = t; best_u = u; best_v = v; best_id = id;
                        }
                    }
                }
                // largest closest-hit distance over the wave's valid lanes (non-negative floats order like
                // their bit patterns; invalid lanes, at -inf, count as 0), reduced in registers
                wmax = __uint_as_float(__ockl_wfred_max_u32(__float_as_uint(fmaxf(best_t, 0.0f))));
                cur = pop();
            }
            cur = __builtin_amdgcn_readfirstlane(cur);
        }
        if (valid)
            P.gbuf_out[(size_t)px * (P.cam.ssaa * P.cam.ssaa) + pk] =
                make_uint4(best_id, __float_as_uint(best_t), __float_as_uint(best_u), __float_as_uint(best_v));
    }
    if (P.w.ray_count) {
        unsigned long long cnt[3] = {rays_cast, node_visits, tri_tests};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            unsigned long long v = cnt[q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) atomicAdd(P.w.ray_count + 2 * q, v);
        }
    }
}

__global__ void k_rect_finish(const uint32_t* counts, uint32_t n_pix, uint32_t N, float* vis)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pix) vis[i] = (float)counts[i] / (float)N;
}

template <int MODE>
constexpr size_t lds_bytes() { return TravStack<SL, BLOCK, MODE == MODE_PRIMARY>::lds_bytes(); }

// compute units of the device and resident blocks of a kernel per compute unit (1 if a query fails)
int cu_count(int device)
{
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n < 1) n = 1;
    return n;
}

int blocks_per_cu(const void* kernel, size_t lds)
{
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, BLOCK, lds) != hipSuccess || b < 1) b = 1;
    return b;
}

}  // namespace

// Launch the instance of KERNEL (written with RC_TWO and RC_WT in its template arguments) that matches the
// scene: flat or two-level structure, Moller-Trumbore or watertight triangle test (`two`, `wt` in scope).
#define RC_LAUNCH_ONE(TWO_, WT_, KERNEL, ...)                   \
    do {                                                         \
        constexpr bool RC_TWO = TWO_, RC_WT = WT_;               \
        hipLaunchKernelGGL(KERNEL, __VA_ARGS__);                 \
    } while (0)
#define RC_LAUNCH_TW(KERNEL, ...)                                                  \
    do {                                                                           \
        if (two) {                                                                 \
            if (wt) RC_LAUNCH_ONE(true, true, KERNEL, __VA_ARGS__);                \
            else RC_LAUNCH_ONE(true, false, KERNEL, __VA_ARGS__);                  \
        } else {                                                                   \
            if (wt) RC_LAUNCH_ONE(false, true, KERNEL, __VA_ARGS__);               \
            else RC_LAUNCH_ONE(false, false, KERNEL, __VA_ARGS__);                 \
        }                                                                          \
    } while (0)

// persistent grid of the traversal kernels: compute units x the largest resident block count among them
int rc_trace_grid(int device)
{
    const int blocks[] = {
        blocks_per_cu(reinterpret_cast<const void*>(&k_trace<MODE_PRIMARY, false, false>), lds_bytes<MODE_PRIMARY>()),
        blocks_per_cu(reinterpret_cast<const void*>(&k_trace<MODE_POINT, false, false>), lds_bytes<MODE_POINT>()),
        blocks_per_cu(reinterpret_cast<const void*>(&k_trace<MODE_RECT, false, false>), lds_bytes<MODE_RECT>()),
        blocks_per_cu(reinterpret_cast<const void*>(&k_rect_packets<false, false>), TravStack<SL, BLOCK, false>::lds_bytes()),
        blocks_per_cu(reinterpret_cast<const void*>(&k_rect_wave<false, false, false, false>), 0),
        blocks_per_cu(reinterpret_cast<const void*>(&k_primary_wave<false>), 0),
        blocks_per_cu(reinterpret_cast<const void*>(&k_point_wave<false, false, false, false>), 0)};
    int b = 1;
    for (int x : blocks) b = std::max(b, x);
    return cu_count(device) * b;
}

void rc_launch_primary(const DevScene& sc, const DevCamera& cam, uint4* gbuf, const TraceWork& w, int grid,
                       bool per_lane, hipStream_t st)
{
    KParams P = {};
    P.sc = sc;
    P.cam = cam;
    P.gbuf_out = gbuf;
    P.w = w;
    P.n_items = rc_n_items(cam.width, cam.height, cam.ssaa);
    P.slot = 0;
    // the wave-uniform traversal pays off with 2x2 supersampling (a wave holds 4 samples of each of 16
    // neighbouring pixels); with one sample per pixel, 8x8-pixel tiles diverge more and per-lane is faster
    // (two-level structures always use the per-lane kernel for camera rays)
    const bool two = sc.inst != nullptr, wt = sc.watertight != 0u;
    if (sc.max_stack <= 128 && !per_lane && cam.ssaa > 1 && !two) {
        P.claim = claim_size((P.n_items + 63) / 64, grid, 64, 1, 4);
        if (wt)
            hipLaunchKernelGGL(k_primary_wave<true>, dim3(grid), dim3(BLOCK), 0, st, P);
        else
            hipLaunchKernelGGL(k_primary_wave<false>, dim3(grid), dim3(BLOCK), 0, st, P);
    } else {
        P.claim = claim_size(P.n_items, grid, 16, 32, 128);
        RC_LAUNCH_TW((k_trace<MODE_PRIMARY, RC_TWO, RC_WT>), dim3(grid), dim3(BLOCK), lds_bytes<MODE_PRIMARY>(), st, P);
    }
}

void rc_launch_shadow(const DevScene& sc, const DevCamera& cam, const DevLights& L, const uint4* gbuf,
                      uint32_t* mask, float* visibility, uint32_t* counts, float4* setup, const TraceWork& w,
                      int grid, RcKernels kernels, hipStream_t st)
{
    KParams P = {};
    P.sc = sc;
    P.cam = cam;
    P.L = L;
    P.gbuf_in = gbuf;
    P.mask = mask;
    P.vis = visibility;
    P.w = w;
    P.n_items = rc_n_items(cam.width, cam.height, cam.ssaa);
    const bool two = sc.inst != nullptr, wt = sc.watertight != 0u;
    const bool count = w.ray_count != nullptr;   // the wave kernels count visits only when asked
    // the wave-uniform kernels address nodes and triangles by 32-bit byte offsets and hold at most 128 stack
    // entries; they read each sample's shadow-ray origin and normal from `setup`
    const bool wave_ok = sc.max_stack <= 128 && kernels != RC_KERNELS_LANE && sc.n_nodes < (1u << 25) &&
                         (uint64_t)sc.n_tris * 48u < (1ull << 32);
    // By default they serve the passes with many rays.  A wave-uniform pass cannot end before its slowest
    // wave, whose 64 rays (an 8x8-pixel tile at one sample per pixel) may diverge over detailed geometry and
    // walk the union of their paths, some hundreds of dependent node steps.  With few rays that walk sets the
    // pass's duration and the per-lane kernels finish first; with many, the wave kernels' shared node loads
    // win.  Measured on the 7.3M-triangle scene: one point light, per-lane / wave 0.24 / 0.46 ms at 960x540,
    // 0.44 / 0.41 ms at 1920x1080, 1.23 / 0.79 ms at 3840x2160; rect light, 1 sample per pixel at 1080p
    // 0.41 / 0.54 ms, 2 samples 0.62 / 0.53 ms, 1 sample at 2160p 1.10 / 0.89 ms.
    const uint64_t n_samples_img = (uint64_t)cam.width * cam.height * cam.ssaa * cam.ssaa;
    const bool big_point = n_samples_img >= 1500000u;
    const bool big_rect = n_samples_img * (uint64_t)(L.has_rect ? L.area_samples : 0) >= 3000000u;
    const bool wave_point = wave_ok && (kernels == RC_KERNELS_WAVE || big_point);
    const bool wave_rect = wave_ok && (kernels == RC_KERNELS_WAVE || big_rect);
    P.setup = setup;
    if (L.n_point > 0 || L.has_rect) {
        // one setup entry per sample of the image (the item count is padded to whole tiles); every shadow kernel
        // reads its rays' origins and normals from there
        const uint32_t n_samples = (uint32_t)(cam.width * cam.height * cam.ssaa * cam.ssaa);
        hipLaunchKernelGGL(k_shadow_setup, dim3((n_samples + 255) / 256), dim3(256), 0, st, sc, cam, gbuf, n_samples,
                           setup);
    }
    if (L.n_point > 0) {
        P.slot = 1;
        if (wave_point) {
            P.claim = claim_size((P.n_items + 63) / 64, grid, 64, 1, 4);
            if (sc.max_stack <= 64) {
                if (count)
                    RC_LAUNCH_TW((k_point_wave<RC_TWO, RC_WT, false, true>), dim3(grid), dim3(BLOCK), 0, st, P,
                                 (const float4*)setup);
                else
                    RC_LAUNCH_TW((k_point_wave<RC_TWO, RC_WT, false, false>), dim3(grid), dim3(BLOCK), 0, st, P,
                                 (const float4*)setup);
            } else {
                if (count)
                    RC_LAUNCH_TW((k_point_wave<RC_TWO, RC_WT, true, true>), dim3(grid), dim3(BLOCK), 0, st, P,
                                 (const float4*)setup);
                else
                    RC_LAUNCH_TW((k_point_wave<RC_TWO, RC_WT, true, false>), dim3(grid), dim3(BLOCK), 0, st, P,
                                 (const float4*)setup);
            }
        } else {
            P.claim = claim_size(P.n_items, grid, 16, 32, 128);
            RC_LAUNCH_TW((k_trace<MODE_POINT, RC_TWO, RC_WT>), dim3(grid), dim3(BLOCK), lds_bytes<MODE_POINT>(), st, P);
        }
    }
    if (L.has_rect) {
        // unit normal of the emitting side, from FP64 and rounded once
        double eu[3] = {L.rect[3], L.rect[4], L.rect[5]}, ev[3] = {L.rect[6], L.rect[7], L.rect[8]};
        double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2], eu[0] * ev[1] - eu[1] * ev[0]};
        double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int a = 0; a < 3; ++a) P.nL[a] = (float)(n[a] / len);
        P.slot = 2;
        const uint64_t n_packets = ((uint64_t)P.n_items * (uint64_t)L.area_samples + 63) / 64;
        P.claim = claim_size(n_packets, grid, 64, 1, 4);
        uint32_t n_pix = (uint32_t)(cam.width * cam.height);
        rc_launch_fill_u32(counts, 0u, n_pix, st);
        // the wave-uniform traversal: a wave holds the samples of one pixel, or of 64 / N neighbouring
        // pixels, whose rays start close together
        if (wave_rect) {
            if (sc.max_stack <= 64) {
                if (count)
                    RC_LAUNCH_TW((k_rect_wave<RC_TWO, RC_WT, false, true>), dim3(grid), dim3(BLOCK), 0, st, P, counts,
                                 (const float4*)setup);
                else
                    RC_LAUNCH_TW((k_rect_wave<RC_TWO, RC_WT, false, false>), dim3(grid), dim3(BLOCK), 0, st, P, counts,
                                 (const float4*)setup);
            } else {
                if (count)
                    RC_LAUNCH_TW((k_rect_wave<RC_TWO, RC_WT, true, true>), dim3(grid), dim3(BLOCK), 0, st, P, counts,
                                 (const float4*)setup);
                else
                    RC_LAUNCH_TW((k_rect_wave<RC_TWO, RC_WT, true, false>), dim3(grid), dim3(BLOCK), 0, st, P, counts,
                                 (const float4*)setup);
            }
        } else {
            const size_t lds = TravStack<SL, BLOCK, false>::lds_bytes();
            RC_LAUNCH_TW((k_rect_packets<RC_TWO, RC_WT>), dim3(grid), dim3(BLOCK), lds, st, P, counts);
        }
        hipLaunchKernelGGL(k_rect_finish, dim3((n_pix + 255) / 256), dim3(256), 0, st, counts, n_pix,
                           (uint32_t)L.area_samples, visibility);
    }
}
