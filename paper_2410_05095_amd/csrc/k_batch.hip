// Batched rendering: every view of every scene in persistent launches fed by device work queues.
//
// Work items are pixels of all views, numbered view by view in tiles of tile_w x tile_h pixels; a
// wave claims `queue_depth` items per atomicAdd on its XCD's counter (XcdQueue) and hands them to its idle
// lanes.  In the one-kernel form (PASS 0) a lane renders its pixel completely: for each sample the camera
// ray (closest hit), the shadow rays towards the view's point lights (any hit), FP64 shading, and finally
// the fixed-order resolve.  In the three-kernel form the same stages run as three launches over all views:
// camera rays into the views' hit buffers (PASS 1), shadow rays into their masks (PASS 2), shading and
// resolve (PASS 3).  Each launch then holds only its own stage's code: the camera-ray kernel needs no FP64
// registers, and no kernel keeps a lane's FP64 shading state across a traversal.  The traversal, shading
// and resolve use the same device code as the single-view kernels, so every view is bit-identical to its
// single-view render whatever the form and tuning.
#include "rc_trav.h"

namespace {

constexpr int BLOCK = RC_TRACE_BLOCK;
constexpr int SL = RC_STACK_LDS;

// The view holding work item `item` (the largest v with item_first <= item), and the
// pixel of the item inside that view's tiles of tile_w x tile_h pixels (false for tile padding).
// Batches of up to VIEW_LDS views search a copy of the views' first items in LDS (rc_views_to_lds), others
// the view table in device memory.
constexpr uint32_t VIEW_LDS = 256;

__device__ inline void rc_views_to_lds(const BatchParams& P, uint32_t* first)
{
    if (P.n_views <= VIEW_LDS)
        for (uint32_t i = threadIdx.x; i < P.n_views; i += blockDim.x) first[i] = P.views[i].item_first;
    __syncthreads();
}

__device__ inline uint32_t rc_find_view(const DevView* views, const uint32_t* first, uint32_t n, uint32_t item)
{
    uint32_t lo = 0, hi = n;
    if (n <= VIEW_LDS) {
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (first[mid] <= item) lo = mid; else hi = mid;
        }
    } else {
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (views[mid].item_first <= item) lo = mid; else hi = mid;
        }
    }
    return lo;
}

__device__ inline bool rc_batch_pixel(const DevView& V, const BatchTune& t, uint32_t item, uint32_t& px)
{
    const uint32_t tile_pix = t.tile_w * t.tile_h;
    const uint32_t local = item - V.item_first;
    const uint32_t tile = local / tile_pix, w = local % tile_pix;
    const uint32_t i = (tile % V.tiles_x) * t.tile_w + w % t.tile_w;
    const uint32_t jj = (tile / V.tiles_x) * t.tile_h + w / t.tile_w;
    if (i >= (uint32_t)V.cam.width || jj >= (uint32_t)V.cam.height) return false;
    px = jj * (uint32_t)V.cam.width + i;
    return true;
}

// Register budgets of the one-stage kernels (64 views, three-kernel form): the camera-ray kernel at 6 waves per
// SIMD (80 registers) 3.74 against 4.21 ms at its natural 104; the shadow-ray kernel, whose FP64 surface
// reconstruction moved to k_batch_setup, at 5 (96 registers) 4.91 ms with the setup, against 5.46 at 4 and
// 5.47 at 6 waves.  The camera kernel at 5 waves (3.79 ms) and the shading kernel held to 5 or 6 waves (1.05,
// 1.42 against 0.66 ms at its natural 128 registers) were slower.
template <int PASS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(PASS == 1 ? 6 : PASS == 2 ? 5 : 1)))
void k_batch(BatchParams P)
{
    static_assert(PASS >= 0 && PASS <= 3, "pass");
    __shared__ uint32_t view_first[VIEW_LDS];
    rc_views_to_lds(P, view_first);
    const int tid = threadIdx.x;
    const uint32_t lane = __lane_id();
    const uint32_t glane = blockIdx.x * BLOCK + tid;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    TravStack<SL, BLOCK, true> st{tid, reinterpret_cast<uint2*>(P.w.overflow), P.w.overflow_depth, P.w.n_lanes,
                                  glane, P.w.error_flag};

    int state = 0;                 // 0 idle, 1 camera ray, 2 shadow ray
    uint32_t v = 0, px = 0, k = 0, spp = 1, j = 0, n_l = 0, mask = 0, hid = RC_NO_HIT;
    float os[3] = {0, 0, 0}, nf[3] = {0, 0, 0};
    float4 prev = make_float4(0, 0, 0, 0), pair = make_float4(0, 0, 0, 0);
    DevScene sc;                   // only nodes and tris are kept for traversal
    sc.nodes = nullptr;
    sc.tris = nullptr;
    TravRay ray;
    TravState ts;
    const XcdQueue<256> queue(P.w.counters, PASS <= 1 ? 3u : (uint32_t)PASS + 2u, P.n_items);
    uint32_t q_next = 0, q_end = 0;   // wave-local range of claimed positions of the XCD's share (wave-uniform)
    bool queue_empty = false;
    uint32_t rays_cast = 0, node_visits = 0, tri_tests = 0;

    // camera ray of sample k of pixel px (a closure without captures: the camera kernel keeps every lane's
    // ray and traversal state in registers only if no closure object holds their addresses)
    const auto start_camera = [](const DevCamera& cam, uint32_t px, uint32_t k, TravRay& ray, TravState& ts,
                                 uint32_t& rays_cast, int& state) __attribute__((always_inline)) {
        rc_camera_ray(cam, px, k, ray.o, ray.d);
        trav_begin(ray, ts);
        ++rays_cast;
        state = 1;
    };
    auto start_sample = [&]() __attribute__((always_inline)) {
        start_camera(P.views[v].cam, px, k, ray, ts, rays_cast, state);
    };

    // the next shadow ray of the sample from light j on (lights below the surface are skipped); false when
    // none is left.  Without captures, like start_camera.
    const auto start_shadow = [](const float* lights, uint32_t& j, uint32_t n_l, uint32_t px, const float* os,
                                 const float* nf, TravRay& ray, TravState& ts, uint32_t& rays_cast,
                                 int& state) __attribute__((always_inline)) -> bool {
        while (j < n_l) {
            if (rc_shadow_ray(lights + 6 * (size_t)j, nullptr, nullptr, false, px, j, 0u, 0u, 0u, os, nf, ray)) {
                trav_begin(ray, ts);
                ++rays_cast;
                state = 2;
                return true;
            }
            ++j;
        }
        return false;
    };
#define RC_NEXT_SHADOW() \
    start_shadow(P.lights + 6 * (size_t)P.views[v].light_first, j, n_l, px, os, nf, ray, ts, rays_cast, state)

    // shadow pass: from sample k on, the first sample whose camera ray hit starts its shadow rays; samples
    // before it get their (empty) masks; the pixel is done when none is left
    // (origin and normal from the setup entries that k_batch_setup wrote, so that this kernel holds no FP64 code)
    auto shadow_sample = [&]() __attribute__((always_inline)) {
        const DevView& V = P.views[v];
        for (; k < spp; ++k) {
            const size_t s = (size_t)px * spp + k;
            const float4 a = P.setup[2 * ((size_t)V.setup_first + s)];
            mask = 0;
            j = 0;
            if (a.w != 0.0f) {
                const float4 b = P.setup[2 * ((size_t)V.setup_first + s) + 1];
                os[0] = a.x; os[1] = a.y; os[2] = a.z;
                nf[0] = b.x; nf[1] = b.y; nf[2] = b.z;
                if (RC_NEXT_SHADOW()) return;
            }
            V.shadow[s] = mask;
        }
        state = 0;
    };

    // shading pass: every sample of the pixel from its hit and mask, folded in the resolve's order
    auto shade_pixel = [&]() __attribute__((always_inline)) {
        const DevView& V = P.views[v];
        const DevScene full = P.scenes[V.scene];
        float4 c4[4];
        for (uint32_t q = 0; q < spp; ++q) {
            const size_t s = (size_t)px * spp + q;
            const uint32_t h = V.hit[s].x;
            c4[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (h != RC_NO_HIT)
                c4[q] = rc_shade_sample(full, V.cam, P.lights + 6 * (size_t)V.light_first, (int)V.n_lights, nullptr,
                                        0.0, px, q, h, V.shadow ? V.shadow[s] : 0u);
        }
        if (spp == 1) {
            reinterpret_cast<float4*>(V.rgba)[px] = c4[0];
            return;
        }
        float4 pr, b, r;
        pr.x = c4[0].x + c4[1].x; pr.y = c4[0].y + c4[1].y; pr.z = c4[0].z + c4[1].z; pr.w = c4[0].w + c4[1].w;
        b.x = c4[2].x + c4[3].x; b.y = c4[2].y + c4[3].y; b.z = c4[2].z + c4[3].z; b.w = c4[2].w + c4[3].w;
        r.x = (pr.x + b.x) * 0.25f; r.y = (pr.y + b.y) * 0.25f;
        r.z = (pr.z + b.z) * 0.25f; r.w = (pr.w + b.w) * 0.25f;
        reinterpret_cast<float4*>(V.rgba)[px] = r;
    };

    // sample k is done: write its mask, shade it, fold it into the resolve; next sample or pixel (one-kernel
    // form only: elsewhere the body is discarded, so that no closure holds the others' state in memory)
    auto finish_sample = [&]() __attribute__((always_inline)) {
      if constexpr (PASS == 0) {
        const DevView& V = P.views[v];
        size_t s = (size_t)px * spp + k;
        if (V.shadow) V.shadow[s] = mask;
        float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
        if (hid != RC_NO_HIT) {
            DevScene full = P.scenes[V.scene];
            c = rc_shade_sample(full, V.cam, P.lights + 6 * (size_t)V.light_first, (int)V.n_lights, nullptr, 0.0,
                                px, k, hid, mask);
        }
        if (spp == 1) {
            reinterpret_cast<float4*>(V.rgba)[px] = c;
            state = 0;
            return;
        }
        if (k == 0 || k == 2) {
            prev = c;
        } else if (k == 1) {
            pair.x = prev.x + c.x; pair.y = prev.y + c.y; pair.z = prev.z + c.z; pair.w = prev.w + c.w;
        } else {
            float4 b, r;
            b.x = prev.x + c.x; b.y = prev.y + c.y; b.z = prev.z + c.z; b.w = prev.w + c.w;
            r.x = (pair.x + b.x) * 0.25f; r.y = (pair.y + b.y) * 0.25f;
            r.z = (pair.z + b.z) * 0.25f; r.w = (pair.w + b.w) * 0.25f;
            reinterpret_cast<float4*>(V.rgba)[px] = r;
            state = 0;
            return;
        }
        ++k;
        start_sample();
      }
    };

    auto start_item = [&](uint32_t item) __attribute__((always_inline)) -> bool {
        v = rc_find_view(P.views, view_first, P.n_views, item);
        const DevView& V = P.views[v];
        if (!rc_batch_pixel(V, P.tune, item, px)) return false;
        spp = (uint32_t)(V.cam.ssaa * V.cam.ssaa);
        n_l = V.n_lights;
        const DevScene& S = P.scenes[V.scene];
        sc.nodes = S.nodes;
        sc.tris = S.tris;
        k = 0;
        if constexpr (PASS == 3) {
            shade_pixel();
            return false;
        } else if constexpr (PASS == 2) {
            if (n_l == 0) return false;
            shadow_sample();
            return state != 0;
        } else {
            start_camera(V.cam, px, k, ray, ts, rays_cast, state);
            return true;
        }
    };

    auto end_ray = [&](bool occluded) __attribute__((always_inline)) {
        if constexpr (PASS == 1) {   // camera ray done: its hit; next sample or pixel
            (void)occluded;
            const DevView& V = P.views[v];
            V.hit[(size_t)px * spp + k] =
                make_uint4(ts.best_id, __float_as_uint(ts.best_t), __float_as_uint(ts.best_u), __float_as_uint(ts.best_v));
            if (++k < spp) start_camera(V.cam, px, k, ray, ts, rays_cast, state);
            else state = 0;
        } else if constexpr (PASS == 2) {   // shadow ray done: next light, else the sample's mask and the next one
            if (!occluded) mask |= 1u << j;
            ++j;
            if (RC_NEXT_SHADOW()) return;
            P.views[v].shadow[(size_t)px * spp + k] = mask;
            ++k;
            shadow_sample();
        } else if (state == 1) {
            const DevView& V = P.views[v];
            V.hit[(size_t)px * spp + k] =
                make_uint4(ts.best_id, __float_as_uint(ts.best_t), __float_as_uint(ts.best_u), __float_as_uint(ts.best_v));
            hid = ts.best_id;
            mask = 0;
            j = 0;
            if (hid != RC_NO_HIT) {
                DevScene full = P.scenes[V.scene];
                Surface Sf = rc_surface(full, V.cam, px, k, hid);
                D3 O = rc_shadow_origin(Sf);
                os[0] = (float)O.x; os[1] = (float)O.y; os[2] = (float)O.z;
                nf[0] = (float)Sf.n.x; nf[1] = (float)Sf.n.y; nf[2] = (float)Sf.n.z;
                if (RC_NEXT_SHADOW()) return;
            }
            finish_sample();
        } else {
            if (!occluded) mask |= 1u << j;
            ++j;
            if (RC_NEXT_SHADOW()) return;
            finish_sample();
        }
    };

    for (;;) {
        // ---- refill idle lanes from the wave-local range, claiming queue_depth items at a time
        for (;;) {
            uint64_t need = __ballot(state == 0);
            if (need == 0) break;
            if (q_next >= q_end) {
                if (queue_empty) break;
                const uint32_t base = queue.claim(P.tune.queue_depth);
                if (queue.exhausted(base)) { queue_empty = true; break; }
                q_next = base;
                q_end = base + P.tune.queue_depth;
                if (queue.exhausted(q_end)) queue_empty = true;   // no later claim can hold work
            }
            uint32_t avail = q_end - q_next;
            uint32_t rank = (uint32_t)__popcll(need & below);
            if (state == 0 && rank < avail) {
                const uint64_t item = queue.at(q_next + rank);
                if (item >= P.n_items || !start_item((uint32_t)item)) state = 0;
            }
            q_next += min(avail, (uint32_t)__popcll(need));
        }
        if (__ballot(state != 0) == 0) break;
        if constexpr (PASS == 3) continue;   // no traversal: lanes stay idle and refill until the queue is done

        for (;;) {
            uint32_t occluded = 0u;
            // bounded traversal phases per step.  Where camera and shadow rays share a wave (one kernel), 16 node
            // rounds and 4 leaf rounds: 64 views in 28.4 instead of 29.6 ms unbounded (3 and 1 took 38 ms).
            // Camera rays alone: 3 and 1, as in the single-view kernel (2 and 1, 4 and 2 were slower).  Shadow
            // rays alone: 8 and 2 (5.34 against 5.47 ms for 3 and 1, 16 and 4 in between)
            constexpr int NODE_STEPS = PASS == 0 ? 16 : PASS == 1 ? 3 : 8;
            constexpr int LEAF_STEPS = PASS == 0 ? 4 : PASS == 1 ? 1 : 2;
            trav_advance<false, false, NODE_STEPS, LEAF_STEPS>(sc, ray, ts, st, state != 0, state == 2, occluded,
                                                               node_visits, tri_tests);
            if (state != 0 && ts.cur == RC_STACK_EMPTY) end_ray(occluded != 0u);
            uint32_t n_act = (uint32_t)__popcll(__ballot(state != 0));
            if (n_act == 0) break;
            if ((q_next < q_end || !queue_empty) && n_act < P.tune.min_rays) break;
        }
    }

    if (P.w.ray_count) {
        unsigned long long cnt[3] = {rays_cast, node_visits, tri_tests};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            unsigned long long vv = cnt[q];
            for (int off = 32; off > 0; off >>= 1) vv += __shfl_xor(vv, off);
            // the shadow pass counts into the second slot of each pair (the one-kernel form counts all rays in
            // the first)
            if (lane == 0) atomicAdd(P.w.ray_count + 2 * q + (PASS == 2 ? 1 : 0), vv);
        }
    }
#undef RC_NEXT_SHADOW
}

}  // namespace

// Shadow-ray setup of the three-kernel form: for every sample of every view with point lights, the origin
// (offset along the normal, in FP64 from the hit, as in the one-kernel form) and the normal, rounded to FP32,
// at the view's place in P.setup; (0, 0, 0, 0) for samples without a hit.
__global__ __launch_bounds__(256) void k_batch_setup(BatchParams P)
{
    __shared__ uint32_t view_first[VIEW_LDS];
    rc_views_to_lds(P, view_first);
    const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= P.n_items) return;
    const DevView& V = P.views[rc_find_view(P.views, view_first, P.n_views, item)];
    uint32_t px = 0;
    if (V.n_lights == 0 || !rc_batch_pixel(V, P.tune, item, px)) return;
    const uint32_t spp = (uint32_t)(V.cam.ssaa * V.cam.ssaa);
    const DevScene sc = P.scenes[V.scene];
    for (uint32_t k = 0; k < spp; ++k) {
        const size_t s = (size_t)px * spp + k;
        const uint32_t h = V.hit[s].x;
        float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b = a;
        if (h != RC_NO_HIT) {
            Surface Sf = rc_surface(sc, V.cam, px, k, h);
            D3 O = rc_shadow_origin(Sf);
            a = make_float4((float)O.x, (float)O.y, (float)O.z, 1.0f);
            b = make_float4((float)Sf.n.x, (float)Sf.n.y, (float)Sf.n.z, 0.0f);
        }
        P.setup[2 * ((size_t)V.setup_first + s)] = a;
        P.setup[2 * ((size_t)V.setup_first + s) + 1] = b;
    }
}

static const void* batch_kernel(int pass)
{
    switch (pass) {
    case 1: return reinterpret_cast<const void*>(&k_batch<1>);
    case 2: return reinterpret_cast<const void*>(&k_batch<2>);
    case 3: return reinterpret_cast<const void*>(&k_batch<3>);
    default: return reinterpret_cast<const void*>(&k_batch<0>);
    }
}

int rc_batch_max_blocks_per_cu(int device, int pass)
{
    int blocks = 0;
    (void)device;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_kernel(pass), BLOCK,
                                                     TravStack<SL, BLOCK, true>::lds_bytes()) != hipSuccess)
        blocks = 1;
    return blocks < 1 ? 1 : blocks;
}

void rc_launch_batch(const BatchParams& P, int pass, int grid, hipStream_t st)
{
    const size_t lds = pass == 3 ? 0 : TravStack<SL, BLOCK, true>::lds_bytes();
    if (grid < (int)RC_XCDS) grid = RC_XCDS;   // every XCD share of the queue needs workgroups
    switch (pass) {
    case 1: hipLaunchKernelGGL(k_batch<1>, dim3(grid), dim3(BLOCK), lds, st, P); break;
    case 2:
        hipLaunchKernelGGL(k_batch_setup, dim3((P.n_items + 255) / 256), dim3(256), 0, st, P);
        hipLaunchKernelGGL(k_batch<2>, dim3(grid), dim3(BLOCK), lds, st, P);
        break;
    case 3: hipLaunchKernelGGL(k_batch<3>, dim3(grid), dim3(BLOCK), lds, st, P); break;
    default: hipLaunchKernelGGL(k_batch<0>, dim3(grid), dim3(BLOCK), lds, st, P); break;
    }
}
