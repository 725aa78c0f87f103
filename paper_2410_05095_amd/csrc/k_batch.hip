// Batched rendering megakernel: every view of every scene in one persistent launch.
//
// Work items are pixels of all views, numbered view by view in tiles of tile_w x tile_h pixels; a
// wave claims `queue_depth` items per atomicAdd on its XCD's counter (XcdQueue) and hands them to its idle
// lanes.  A lane renders its pixel completely: for each sample the camera ray (closest hit), the
// shadow rays towards the view's point lights (any hit), FP64 shading, and finally the fixed-order
// resolve.  The traversal, shading and resolve use the same device code as the single-view kernels,
// so every view is bit-identical to its single-view render whatever the tuning.
#include "rc_trav.h"

namespace {

constexpr int BLOCK = RC_TRACE_BLOCK;
constexpr int SL = RC_STACK_LDS;

__device__ inline uint32_t find_view(const DevView* views, uint32_t n, uint32_t item)
{
    uint32_t lo = 0, hi = n;   // largest v with item_first <= item
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (views[mid].item_first <= item) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(BLOCK) void k_batch(BatchParams P)
{
    const int tid = threadIdx.x;
    const uint32_t lane = __lane_id();
    const uint32_t glane = blockIdx.x * BLOCK + tid;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    TravStack<SL, BLOCK, true> st{tid, reinterpret_cast<uint2*>(P.w.overflow), P.w.overflow_depth, P.w.n_lanes,
                                  glane, P.w.error_flag};
    const uint32_t tile_pix = P.tune.tile_w * P.tune.tile_h;

    int state = 0;                 // 0 idle, 1 camera ray, 2 shadow ray
    uint32_t v = 0, px = 0, k = 0, spp = 1, j = 0, n_l = 0, mask = 0, hid = RC_NO_HIT;
    float os[3] = {0, 0, 0}, nf[3] = {0, 0, 0};
    float4 prev = make_float4(0, 0, 0, 0), pair = make_float4(0, 0, 0, 0);
    DevScene sc;                   // only nodes and tris are kept for traversal
    sc.nodes = nullptr;
    sc.tris = nullptr;
    TravRay ray;
    TravState ts;
    const XcdQueue<256> queue(P.w.counters, 3, P.n_items);
    uint32_t q_next = 0, q_end = 0;   // wave-local range of claimed positions of the XCD's share (wave-uniform)
    bool queue_empty = false;
    uint32_t rays_cast = 0, node_visits = 0, tri_tests = 0;

    auto start_sample = [&]() {
        const DevView& V = P.views[v];
        rc_camera_ray(V.cam, px, k, ray.o, ray.d);
        trav_begin(ray, ts);
        ++rays_cast;
        state = 1;
    };

    auto next_shadow = [&]() -> bool {
        const DevView& V = P.views[v];
        while (j < n_l) {
            if (rc_shadow_ray(P.lights + 6 * (size_t)(V.light_first + j), nullptr, nullptr, false, px, j, 0u,
                              0u, 0u, os, nf, ray)) {
                trav_begin(ray, ts);
                ++rays_cast;
                state = 2;
                return true;
            }
            ++j;
        }
        return false;
    };

    // sample k is done: write its mask, shade it, fold it into the resolve; next sample or pixel
    auto finish_sample = [&]() {
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
    };

    auto start_item = [&](uint32_t item) -> bool {
        v = find_view(P.views, P.n_views, item);
        const DevView& V = P.views[v];
        uint32_t local = item - V.item_first;
        uint32_t tile = local / tile_pix, w = local % tile_pix;
        uint32_t i = (tile % V.tiles_x) * P.tune.tile_w + w % P.tune.tile_w;
        uint32_t jj = (tile / V.tiles_x) * P.tune.tile_h + w / P.tune.tile_w;
        if (i >= (uint32_t)V.cam.width || jj >= (uint32_t)V.cam.height) return false;
        px = jj * (uint32_t)V.cam.width + i;
        spp = (uint32_t)(V.cam.ssaa * V.cam.ssaa);
        n_l = V.n_lights;
        const DevScene& S = P.scenes[V.scene];
        sc.nodes = S.nodes;
        sc.tris = S.tris;
        k = 0;
        start_sample();
        return true;
    };

    auto end_ray = [&](bool occluded) {
        if (state == 1) {
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
                if (next_shadow()) return;
            }
            finish_sample();
        } else {
            if (!occluded) mask |= 1u << j;
            ++j;
            if (next_shadow()) return;
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

        for (;;) {
            uint32_t occluded = 0u;
            // at most 16 node rounds and 4 leaf rounds per step: 64 views in 28.4 instead of 29.6 ms (3 and 1,
            // the camera kernel's bounds, took 38 ms here, where camera and shadow rays share a wave)
            trav_advance<false, false, 16, 4>(sc, ray, ts, st, state != 0, state == 2, occluded, node_visits,
                                              tri_tests);
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
            if (lane == 0) atomicAdd(P.w.ray_count + 2 * q, vv);
        }
    }
}

}  // namespace

int rc_batch_max_blocks_per_cu(int device)
{
    int blocks = 0;
    (void)device;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(&k_batch), BLOCK,
                                                     TravStack<SL, BLOCK, true>::lds_bytes()) != hipSuccess)
        blocks = 1;
    return blocks < 1 ? 1 : blocks;
}

void rc_launch_batch(const BatchParams& P, int grid, hipStream_t st)
{
    const size_t lds = TravStack<SL, BLOCK, true>::lds_bytes();
    if (grid < (int)RC_XCDS) grid = RC_XCDS;   // every XCD share of the queue needs workgroups
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(BLOCK), lds, st, P);
}
