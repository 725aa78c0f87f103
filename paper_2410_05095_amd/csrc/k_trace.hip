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
#include "rc_trav.h"

namespace {

constexpr int BLOCK = RC_TRACE_BLOCK;
constexpr int SL = RC_STACK_LDS;
constexpr int REFILL_AT = 40;   // refill once a wave has at most this many busy lanes

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
    TraceWork w;
    uint32_t n_items;
    uint32_t slot;
};

template <int MODE>
__global__ __launch_bounds__(BLOCK) void k_trace(KParams P)
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
    bool queue_empty = false;
    uint32_t rays_cast = 0, node_visits = 0, tri_tests = 0;

    // shadow items: set up the next ray that is cast, or return false
    auto next_shadow_ray = [&]() -> bool {
        while (j < n_rays) {
            if (rc_shadow_ray(P.L.point[MODE == MODE_POINT ? j : 0], P.L.rect, P.nL, MODE == MODE_RECT, px, j,
                              P.L.area_stream, P.cam.seed, P.cam.frame, os, nf, ray)) {
                trav_begin(ray, ts);
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
            trav_begin(ray, ts);
            ++rays_cast;
            return true;
        } else {
            size_t s = (size_t)px * (P.cam.ssaa * P.cam.ssaa) + pk;
            uint4 h = P.gbuf_in[s];
            acc = 0;
            j = 0;
            n_rays = MODE == MODE_POINT ? (uint32_t)P.L.n_point : (uint32_t)P.L.area_samples;
            if (h.x == RC_NO_HIT) { finish_item(); return false; }
            Surface S = rc_surface(sc, P.cam, px, pk, h.x);
            D3 O = rc_shadow_origin(S);
            os[0] = (float)O.x; os[1] = (float)O.y; os[2] = (float)O.z;
            nf[0] = (float)S.n.x; nf[1] = (float)S.n.y; nf[2] = (float)S.n.z;
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
            int leader = __ffsll((unsigned long long)need) - 1;
            uint32_t cnt = (uint32_t)__popcll(need);
            uint32_t base = 0;
            if ((int)lane == leader) base = atomicAdd(&P.w.counters[P.slot], cnt);
            base = __shfl(base, leader);
            if (base + cnt >= P.n_items) queue_empty = true;
            if (state == 0) {
                uint32_t my = base + (uint32_t)__popcll(need & below);
                if (my < P.n_items && start_item(my)) state = 1;
            }
        }
        if (__ballot(state == 1) == 0) break;

        // ---- traversal: node phase then leaf phase for all busy lanes, until enough lanes are idle
        for (;;) {
            bool occluded = false;
            trav_advance(sc, ray, ts, st, state == 1, ANY, occluded, node_visits, tri_tests);
            if (state == 1 && ts.cur == RC_STACK_EMPTY) {
                if (!end_ray(occluded)) state = 0;
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
    for (;;) {
        uint32_t blk = 0;
        if (lane == 0) blk = atomicAdd(&P.w.counters[P.slot], 1u);
        blk = __shfl(blk, 0);
        if (blk >= n_blocks) break;
        const uint64_t r = (uint64_t)blk * 64 + lane;
        const uint32_t item = (uint32_t)(r / N), k = (uint32_t)(r % N);
        uint32_t px = 0, pk = 0;
        const bool in_image = r < total && rc_item_to_sample(P.cam, item, px, pk);
        bool busy = false;
        if (in_image) {
            uint4 h = P.gbuf_in[px];
            if (h.x != RC_NO_HIT) {
                Surface S = rc_surface(sc, P.cam, px, 0, h.x);
                D3 O = rc_shadow_origin(S);
                float os[3] = {(float)O.x, (float)O.y, (float)O.z};
                float nf[3] = {(float)S.n.x, (float)S.n.y, (float)S.n.z};
                busy = rc_shadow_ray(P.L.point[0], P.L.rect, P.nL, true, px, k, P.L.area_stream, P.cam.seed,
                                     P.cam.frame, os, nf, ray);
                if (busy) {
                    trav_begin(ray, ts);
                    ++rays_cast;
                }
            }
        }
        bool occluded = false;
        while (__ballot(busy && ts.cur != RC_STACK_EMPTY) != 0)
            trav_advance(sc, ray, ts, st, busy, true, occluded, node_visits, tri_tests);
        const uint64_t vis = __ballot(busy && !occluded);
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

__global__ void k_rect_finish(const uint32_t* counts, uint32_t n_pix, uint32_t N, float* vis)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pix) vis[i] = (float)counts[i] / (float)N;
}

template <int MODE>
constexpr size_t lds_bytes() { return TravStack<SL, BLOCK, MODE == MODE_PRIMARY>::lds_bytes(); }

template <int MODE>
int occupancy_grid(int device)
{
    int n_cu = 0, blocks = 0;
    hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(&k_trace<MODE>), BLOCK,
                                                 lds_bytes<MODE>());
    if (blocks < 1) blocks = 1;
    return n_cu * blocks;
}

}  // namespace

int rc_trace_grid(int device)
{
    int a = occupancy_grid<MODE_PRIMARY>(device);
    int b = occupancy_grid<MODE_POINT>(device);
    int c = occupancy_grid<MODE_RECT>(device);
    int d = 0, n_cu = 0;
    hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&d, reinterpret_cast<const void*>(&k_rect_packets), BLOCK,
                                                 TravStack<SL, BLOCK, false>::lds_bytes());
    return std::max(std::max(a, d * n_cu), std::max(b, c));
}

void rc_launch_primary(const DevScene& sc, const DevCamera& cam, uint4* gbuf, const TraceWork& w, int grid,
                       hipStream_t st)
{
    KParams P = {};
    P.sc = sc;
    P.cam = cam;
    P.gbuf_out = gbuf;
    P.w = w;
    P.n_items = rc_n_items(cam.width, cam.height, cam.ssaa);
    P.slot = 0;
    hipLaunchKernelGGL(k_trace<MODE_PRIMARY>, dim3(grid), dim3(BLOCK), lds_bytes<MODE_PRIMARY>(), st, P);
}

void rc_launch_shadow(const DevScene& sc, const DevCamera& cam, const DevLights& L, const uint4* gbuf,
                      uint32_t* mask, float* visibility, uint32_t* counts, const TraceWork& w, int grid,
                      hipStream_t st)
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
    if (L.n_point > 0) {
        P.slot = 1;
        hipLaunchKernelGGL(k_trace<MODE_POINT>, dim3(grid), dim3(BLOCK), lds_bytes<MODE_POINT>(), st, P);
    }
    if (L.has_rect) {
        // unit normal of the emitting side, from FP64 and rounded once
        double eu[3] = {L.rect[3], L.rect[4], L.rect[5]}, ev[3] = {L.rect[6], L.rect[7], L.rect[8]};
        double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2], eu[0] * ev[1] - eu[1] * ev[0]};
        double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int a = 0; a < 3; ++a) P.nL[a] = (float)(n[a] / len);
        P.slot = 2;
        uint32_t n_pix = (uint32_t)(cam.width * cam.height);
        rc_launch_fill_u32(counts, 0u, n_pix, st);
        const size_t lds = TravStack<SL, BLOCK, false>::lds_bytes();
        hipLaunchKernelGGL(k_rect_packets, dim3(grid), dim3(BLOCK), lds, st, P, counts);
        hipLaunchKernelGGL(k_rect_finish, dim3((n_pix + 255) / 256), dim3(256), 0, st, counts, n_pix,
                           (uint32_t)L.area_samples, visibility);
    }
}
