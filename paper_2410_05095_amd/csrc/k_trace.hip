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
#include "rc_device.h"

namespace {

constexpr int BLOCK = RC_TRACE_BLOCK;
constexpr int SL = RC_STACK_LDS;
constexpr uint32_t STACK_EMPTY = 0xFFFFFFFEu;
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

// conservative growth of the far slab distance (covers FP32 rounding of the slab tests)
constexpr float FAR_GROW = 1.000001f;

template <int MODE>
__global__ __launch_bounds__(BLOCK) void k_trace(KParams P)
{
    constexpr bool ANY = MODE != MODE_PRIMARY;
    __shared__ uint32_t s_node[SL][BLOCK];
    __shared__ float s_t[ANY ? 1 : SL][BLOCK];

    const int tid = threadIdx.x;
    const uint32_t lane = __lane_id();
    const uint32_t glane = blockIdx.x * BLOCK + tid;
    const DevScene sc = P.sc;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    int state = 0;                    // 0 idle, 1 tracing
    uint32_t px = 0, pk = 0;          // pixel and sample of the current item
    uint32_t j = 0, acc = 0;          // shadow: current light / light sample, result accumulator
    uint32_t n_rays = 0;
    float os[3] = {0, 0, 0}, nf[3] = {0, 0, 0};
    float o[3], d[3], inv[3];
    uint32_t cur = 0;
    int sp = 0;
    uint32_t best_id = RC_NO_HIT;
    float best_t = INFINITY, best_u = 0.f, best_v = 0.f;
    bool queue_empty = false;
    uint32_t rays_cast = 0, node_visits = 0, tri_tests = 0;

    auto set_dir = [&]() {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float dd = fabsf(d[a]) < 1e-20f ? copysignf(1e-20f, d[a]) : d[a];
            inv[a] = 1.0f / dd;
        }
        cur = 0;
        sp = 0;
        rays_cast++;
    };

    auto push = [&](uint32_t node, float t) {
        if (sp < SL) {
            s_node[sp][tid] = node;
            if (!ANY) s_t[sp][tid] = t;
        } else if ((uint32_t)(sp - SL) < P.w.overflow_depth) {
            uint2* g = reinterpret_cast<uint2*>(P.w.overflow) + (size_t)(sp - SL) * P.w.n_lanes + glane;
            *g = make_uint2(node, __float_as_uint(t));
        } else {
            *P.w.error_flag = 1u;   // bound exceeded: drop the entry (flagged, never expected)
            return;
        }
        ++sp;
    };

    auto pop = [&]() -> uint32_t {
        for (;;) {
            if (sp == 0) return STACK_EMPTY;
            --sp;
            uint32_t node;
            float t;
            if (sp < SL) {
                node = s_node[sp][tid];
                t = ANY ? 0.0f : s_t[sp][tid];
            } else {
                uint2 g = reinterpret_cast<const uint2*>(P.w.overflow)[(size_t)(sp - SL) * P.w.n_lanes + glane];
                node = g.x;
                t = __uint_as_float(g.y);
            }
            if (ANY || t <= best_t) return node;
        }
    };

    // shadow items: set up the next ray with n . d > 0 (and facing the rect light), or return false
    auto next_shadow_ray = [&]() -> bool {
        while (j < n_rays) {
            float tgt[3];
            if (MODE == MODE_POINT) {
                tgt[0] = P.L.point[j][0]; tgt[1] = P.L.point[j][1]; tgt[2] = P.L.point[j][2];
            } else {
                uint32_t r[4];
                rc_philox(px, j, 1u + P.L.area_stream, 0u, P.cam.seed, P.cam.frame, r);
                float x1 = rc_unit24(r[0]) - 0.5f, x2 = rc_unit24(r[1]) - 0.5f;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    float t1 = x1 * P.L.rect[3 + a];
                    float t2 = x2 * P.L.rect[6 + a];
                    tgt[a] = (P.L.rect[a] + t1) + t2;
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) { o[a] = os[a]; d[a] = tgt[a] - os[a]; }
            float nd = nf[0] * d[0] + nf[1] * d[1];
            nd = nd + nf[2] * d[2];
            bool ok = nd > 0.0f;
            if (MODE == MODE_RECT) {
                float ld = P.nL[0] * d[0] + P.nL[1] * d[1];
                ld = ld + P.nL[2] * d[2];
                ok = ok && ld < 0.0f;
            }
            if (ok) { set_dir(); return true; }
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
            rc_camera_ray(P.cam, px, pk, o, d);
            best_id = RC_NO_HIT;
            best_t = INFINITY;
            best_u = best_v = 0.0f;
            set_dir();
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
                make_uint4(best_id, __float_as_uint(best_t), __float_as_uint(best_u), __float_as_uint(best_v));
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

        // ---- traversal steps: one node or one leaf per lane and step
        for (;;) {
            if (state == 1) {
                bool ended = false, occluded = false;
                if (!rc_is_leaf(cur)) {
                    ++node_visits;
                    const float4* np = reinterpret_cast<const float4*>(sc.nodes + cur);
                    float4 lx = np[0], hx = np[1], ly = np[2], hy = np[3], lz = np[4], hz = np[5];
                    uint4 ch = reinterpret_cast<const uint4*>(np)[6];
                    const float bound = ANY ? 1.0f : best_t;
                    float lxs[4] = {lx.x, lx.y, lx.z, lx.w}, hxs[4] = {hx.x, hx.y, hx.z, hx.w};
                    float lys[4] = {ly.x, ly.y, ly.z, ly.w}, hys[4] = {hy.x, hy.y, hy.z, hy.w};
                    float lzs[4] = {lz.x, lz.y, lz.z, lz.w}, hzs[4] = {hz.x, hz.y, hz.z, hz.w};
                    uint32_t cw[4] = {ch.x, ch.y, ch.z, ch.w};
                    float tn[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        float nx = inv[0] >= 0.0f ? lxs[c] : hxs[c], fx = inv[0] >= 0.0f ? hxs[c] : lxs[c];
                        float ny = inv[1] >= 0.0f ? lys[c] : hys[c], fy = inv[1] >= 0.0f ? hys[c] : lys[c];
                        float nz = inv[2] >= 0.0f ? lzs[c] : hzs[c], fz = inv[2] >= 0.0f ? hzs[c] : lzs[c];
                        float t0 = fmaxf(fmaxf((nx - o[0]) * inv[0], (ny - o[1]) * inv[1]),
                                         fmaxf((nz - o[2]) * inv[2], 0.0f));
                        float t1 = fminf(fminf((fx - o[0]) * inv[0], (fy - o[1]) * inv[1]), (fz - o[2]) * inv[2]);
                        bool hit = t0 <= fminf(t1 * FAR_GROW, bound);
                        tn[c] = hit ? t0 : INFINITY;
                    }
                    if (!ANY) {
                        // sort (distance, child) ascending: misses (inf) sink to the end
#define RC_CS(a, b)                                                                   \
    {                                                                                 \
        bool sw = tn[b] < tn[a];                                                      \
        float ta = sw ? tn[b] : tn[a], tb = sw ? tn[a] : tn[b];                       \
        uint32_t ca = sw ? cw[b] : cw[a], cb = sw ? cw[a] : cw[b];                    \
        tn[a] = ta; tn[b] = tb; cw[a] = ca; cw[b] = cb;                               \
    }
                        RC_CS(0, 1) RC_CS(2, 3) RC_CS(0, 2) RC_CS(1, 3) RC_CS(1, 2)
#undef RC_CS
                        if (tn[3] < INFINITY) push(cw[3], tn[3]);
                        if (tn[2] < INFINITY) push(cw[2], tn[2]);
                        if (tn[1] < INFINITY) push(cw[1], tn[1]);
                        cur = tn[0] < INFINITY ? cw[0] : pop();
                    } else {
                        uint32_t next = STACK_EMPTY;
#pragma unroll
                        for (int c = 3; c >= 0; --c) {
                            if (tn[c] < INFINITY) {
                                if (next != STACK_EMPTY) push(next, 0.0f);
                                next = cw[c];
                            }
                        }
                        cur = next != STACK_EMPTY ? next : pop();
                    }
                } else {
                    uint32_t first = rc_leaf_first(cur), cnt = rc_leaf_count(cur);
                    for (uint32_t i = 0; i < cnt; ++i) {
                        ++tri_tests;
                        const float4* tp = sc.tris + 3 * (size_t)(first + i);
                        float4 A = tp[0], B = tp[1], C = tp[2];
                        // Moller-Trumbore
                        float px_ = d[1] * C.z - d[2] * C.y;
                        float py_ = d[2] * C.x - d[0] * C.z;
                        float pz_ = d[0] * C.y - d[1] * C.x;
                        float det = B.x * px_ + B.y * py_;
                        det = det + B.z * pz_;
                        float idet = __builtin_amdgcn_rcpf(det);
                        float sx = o[0] - A.x, sy = o[1] - A.y, sz = o[2] - A.z;
                        float su = sx * px_ + sy * py_;
                        su = su + sz * pz_;
                        float u = su * idet;
                        float qx = sy * B.z - sz * B.y;
                        float qy = sz * B.x - sx * B.z;
                        float qz = sx * B.y - sy * B.x;
                        float sv = d[0] * qx + d[1] * qy;
                        sv = sv + d[2] * qz;
                        float v = sv * idet;
                        float st = C.x * qx + C.y * qy;
                        st = st + C.z * qz;
                        float t = st * idet;
                        bool hit = u >= 0.0f && v >= 0.0f && u + v <= 1.0f && t > 0.0f;
                        if (ANY) {
                            if (hit && t < 1.0f) { occluded = true; break; }
                        } else {
                            uint32_t id = __float_as_uint(A.w);
                            if (hit && (t < best_t || (t == best_t && id < best_id))) {
                                best_t = t; best_u = u; best_v = v; best_id = id;
                            }
                        }
                    }
                    cur = occluded ? STACK_EMPTY : pop();
                }
                if (cur == STACK_EMPTY) ended = true;
                if (ended) {
                    if (!end_ray(occluded)) state = 0;
                }
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

template <int MODE>
int occupancy_grid(int device)
{
    int n_cu = 0, blocks = 0;
    hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(&k_trace<MODE>), BLOCK, 0);
    if (blocks < 1) blocks = 1;
    return n_cu * blocks;
}

}  // namespace

int rc_trace_grid(int device)
{
    int a = occupancy_grid<MODE_PRIMARY>(device);
    int b = occupancy_grid<MODE_POINT>(device);
    int c = occupancy_grid<MODE_RECT>(device);
    return std::max(a, std::max(b, c));
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
    hipLaunchKernelGGL(k_trace<MODE_PRIMARY>, dim3(grid), dim3(BLOCK), 0, st, P);
}

void rc_launch_shadow(const DevScene& sc, const DevCamera& cam, const DevLights& L, const uint4* gbuf,
                      uint32_t* mask, float* visibility, const TraceWork& w, int grid, hipStream_t st)
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
        hipLaunchKernelGGL(k_trace<MODE_POINT>, dim3(grid), dim3(BLOCK), 0, st, P);
    }
    if (L.has_rect) {
        // unit normal of the emitting side, from FP64 and rounded once
        double eu[3] = {L.rect[3], L.rect[4], L.rect[5]}, ev[3] = {L.rect[6], L.rect[7], L.rect[8]};
        double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2], eu[0] * ev[1] - eu[1] * ev[0]};
        double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int a = 0; a < 3; ++a) P.nL[a] = (float)(n[a] / len);
        P.slot = 2;
        hipLaunchKernelGGL(k_trace<MODE_RECT>, dim3(grid), dim3(BLOCK), 0, st, P);
    }
}
