// Internal types shared by the host runtime and the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#define RC_NO_HIT 0xFFFFFFFFu
#define RC_EMPTY_CHILD 0xFFFFFFFFu
#define RC_LEAF_BIT 0x80000000u

// 4-wide BVH node: the four child boxes in structure-of-arrays form followed by the
// child words and bookkeeping, 128 bytes = one cache line of the CDNA L2.
struct alignas(128) Node4 {
    float lo_x[4], hi_x[4], lo_y[4], hi_y[4], lo_z[4], hi_z[4];
    uint32_t child[4];   // internal index | (RC_LEAF_BIT | (count-1) << 28 | first) | RC_EMPTY_CHILD
    uint32_t parent;     // parent node index (0xFFFFFFFF for the root)
    uint32_t level;      // depth of this node (root = 0)
    uint32_t pad[2];
};
static_assert(sizeof(Node4) == 128, "node must be one 128-byte line");

__host__ __device__ inline bool rc_is_leaf(uint32_t c) { return (c & RC_LEAF_BIT) != 0u && c != RC_EMPTY_CHILD; }
__host__ __device__ inline uint32_t rc_leaf_first(uint32_t c) { return c & 0x0FFFFFFFu; }
__host__ __device__ inline uint32_t rc_leaf_count(uint32_t c) { return ((c >> 28) & 7u) + 1u; }
__host__ __device__ inline uint32_t rc_make_leaf(uint32_t first, uint32_t count)
{
    return RC_LEAF_BIT | ((count - 1u) << 28) | first;
}

// Packed triangle in leaf order: three float4 = 48 bytes,
// (v0.xyz, original id as bits), (e1.xyz, 0), (e2.xyz, 0) with e1 = v1 - v0, e2 = v2 - v0 in FP32.

// Instance of a two-level structure: world-to-object map [M | m] (row-major 3x4) and the root node of
// its bottom-level tree.  64 bytes.
struct alignas(64) DevInst {
    float w2o[12];
    uint32_t root;
    uint32_t pad[3];
};

struct DevScene {
    const float* pos;         // n_vertices x 3 (current positions)
    const uint32_t* idx;      // n_tris x 3
    const uint32_t* tri_mat;  // n_tris
    const float* mats;        // n_materials x 5
    const Node4* nodes;
    const float4* tris;       // 3 per slot
    uint32_t n_tris, n_nodes;
    uint32_t max_stack;
    float scale;              // max |coordinate| of the scene (for diagnostics)
    const DevInst* inst;      // two-level structures: instances (NULL for a flat BVH)
    uint32_t tlas_root;       // two-level structures: root node of the top level
    uint32_t watertight;      // triangles packed as (v0, v1, v2) and tested watertight (else (v0, e1, e2), MT)
    const float* nrm;         // n_vertices x 3 vertex normals (current pose), or NULL
};

struct DevCamera {
    float eye[3], f[3], r[3], u[3];
    float tan_half, x_scale;
    int32_t width, height, ssaa;
    uint32_t seed, frame;
};

struct DevLights {
    int n_point;
    float point[16][6];       // position, intensity
    int has_rect;
    float rect[12];           // center, edge_u, edge_v, radiance
    int area_samples;
    uint32_t area_stream;
};

// Host-built BVH (binned SAH, collapsed to 4-wide, nodes in breadth-first order).
struct HostBvh {
    std::vector<Node4> nodes;
    std::vector<uint32_t> tri_order;     // slot -> original triangle id
    std::vector<uint32_t> level_start;   // node index where each level starts (size depth+1)
    uint32_t depth = 0;
    uint32_t max_stack = 0;
    uint64_t n_leaves = 0;
    double sah_cost = 0.0;
};

bool rc_build_bvh_host(const float* pos, const uint32_t* idx, uint32_t n_tris,
                       uint32_t bins, uint32_t max_leaf, float node_cost, HostBvh& out);
double rc_bvh_sah(const std::vector<Node4>& nodes);
// Device LBVH builds (k_build.hip); see rc_bvh_build.
hipError_t rc_build_bvh_device(const float* d_pos, const uint32_t* d_idx, uint32_t n, uint32_t max_leaf,
                               const uint32_t* d_seg, const std::vector<uint32_t>& seg_first,
                               const std::vector<uint32_t>& seg_count, Node4** d_nodes_out, uint32_t* n_nodes_out,
                               uint32_t* d_order, std::vector<uint32_t>& level_start, hipStream_t st);
// Device binned-SAH build (k_build.hip): the host builder's algorithm on the GPU (bins <= 64); outputs as
// rc_build_bvh_device.
hipError_t rc_build_bvh_device_sah(const float* d_pos, const uint32_t* d_idx, uint32_t n, uint32_t bins,
                                   uint32_t max_leaf, float node_cost, Node4** d_nodes_out, uint32_t* n_nodes_out,
                                   uint32_t* d_order, std::vector<uint32_t>& level_start, hipStream_t st);
// Top-level workspace (all device memory, sized for n instances at allocation).
struct TlasWork {
    uint32_t n = 0, cap = 0;
    size_t temp_bytes = 0;
    void *box = nullptr, *cen = nullptr, *partial = nullptr, *bounds = nullptr, *keys = nullptr, *keys_s = nullptr,
         *vals = nullptr, *order = nullptr, *flags = nullptr, *child = nullptr, *range = nullptr, *parent = nullptr,
         *nbox = nullptr, *lvl = nullptr, *info = nullptr, *temp = nullptr;   // info: {nodes, levels, error}
};
#define RC_TLAS_MAX_LEVELS 24
hipError_t rc_tlas_alloc(TlasWork& w, uint32_t n);
void rc_tlas_free(TlasWork& w);
hipError_t rc_tlas_build(TlasWork& w, const float* o2w, Node4* nodes, uint32_t tlas_base, DevInst* inst,
                         uint32_t max_levels, uint32_t* error_flag, hipStream_t st);

// Traversal launch geometry
#define RC_TRACE_BLOCK 128
// Work-queue counters: words [0, 8) single queues, [8] sticky bound-exceeded flag, [9] sticky invalid-value flag
// (an input a kernel cannot use, e.g. a hit id beyond the scene); from word RC_QUEUE_BASE, per queue slot
// one counter per XCD, each on its own 256-byte line.
#define RC_XCDS 8
#define RC_QUEUE_SLOTS 6
#define RC_QUEUE_BASE 64
#define RC_COUNTER_WORDS (RC_QUEUE_BASE + RC_QUEUE_SLOTS * RC_XCDS * 64)
#define RC_STACK_LDS 12

struct TraceWork {
    uint32_t* counters;       // device work-queue counters
    uint32_t* overflow;       // per-lane overflow stack (lane-interleaved), entries of 2 words
    uint32_t overflow_depth;  // entries per lane beyond the LDS part
    uint32_t n_lanes;         // lanes of the persistent grid
    uint32_t* error_flag;     // set on stack overflow
    unsigned long long* ray_count; // [0] rays cast, [2] nodes visited, [4] triangles tested (NULL = not counted)
};

// Launchers (k_trace.hip)
void rc_launch_primary(const DevScene& sc, const DevCamera& cam, uint4* gbuf, const TraceWork& w,
                       int grid, bool per_lane, hipStream_t st);
// shadow-ray kernels: chosen by pass size (AUTO), or forced one ray per lane or wave-uniform
enum RcKernels { RC_KERNELS_AUTO = 0, RC_KERNELS_LANE = 1, RC_KERNELS_WAVE = 2 };
void rc_launch_shadow(const DevScene& sc, const DevCamera& cam, const DevLights& L, const uint4* gbuf,
                      uint32_t* mask, float* visibility, uint32_t* counts, float4* setup, const TraceWork& w,
                      int grid, RcKernels kernels, hipStream_t st);
int rc_trace_grid(int device);
// Display post pass (k_post.hip): tone map + sRGB8 into `out`, or into `scratch` followed by FXAA into `out`
void rc_launch_postprocess(const float* rgba, uint32_t w, uint32_t h, bool fxaa, uint8_t* scratch, uint8_t* out,
                           hipStream_t st);
// Fixed per-device scratch of rc_postprocess_noalloc (k_post.hip): rc_post_scratch_init obtains its device
// address on `device` (once; called by rc_create), rc_post_scratch returns it (NULL before init).
constexpr uint32_t RC_POST_SCRATCH_PIXELS = 1u << 22;   // = RC_POST_NOALLOC_MAX_PIXELS of the C ABI
hipError_t rc_post_scratch_init(int device);
uint8_t* rc_post_scratch(int device);

// Batched rendering: one persistent launch over many views of several scenes.
struct DevView {
    DevCamera cam;
    uint32_t scene;           // index into the scene table
    uint32_t light_first;     // index of the first light (6 floats each) in the light table
    uint32_t n_lights;
    uint32_t item_first;      // first work item of this view (exclusive prefix over views)
    uint32_t tiles_x;         // tiles per image row
    uint32_t setup_first;     // first sample of this view in the shadow-ray setup buffer (three-kernel form)
    float* rgba;
    uint4* hit;
    uint32_t* shadow;
};

struct BatchTune {
    uint32_t tile_w, tile_h;      // work-item tile in pixels
    uint32_t queue_depth;         // items a wave claims per atomic (multiple of 64)
    uint32_t min_rays;            // a wave refills its idle lanes once fewer rays are in flight
    uint32_t waves_per_simd;      // resident waves per SIMD of the persistent grid
    uint32_t passes;              // 1: one kernel per pixel's whole render; 3: one kernel per stage
};

struct BatchParams {
    const DevScene* scenes;
    const DevView* views;
    const float* lights;
    float4* setup;            // three-kernel form: per sample (shadow-ray origin, 1 | 0) and (normal, 0)
    uint32_t n_views;
    uint32_t n_items;
    BatchTune tune;
    TraceWork w;
};

// pass 0: the one-kernel form; 1, 2, 3: camera rays, shadow rays, shading + resolve (work-queue slots 3, 4, 5);
// the shadow pass first fills P.setup from the camera hits
void rc_launch_batch(const BatchParams& P, int pass, int grid, hipStream_t st);
int rc_batch_max_blocks_per_cu(int device, int pass);

// Launchers (k_shade.hip)
void rc_launch_shade(const DevScene& sc, const DevCamera& cam, const DevLights& L, const uint4* gbuf,
                     const uint32_t* mask, const float* visibility, float* rgba, float* sample_rgba,
                     uint32_t* bad_value, hipStream_t st);
void rc_launch_camera_rays(const DevCamera& cam, float* o, float* d, uint32_t n, hipStream_t st);
void rc_launch_pack_features(const DevScene& sc, const DevCamera& cam, const uint4* gbuf, const float* vis,
                             float inv_log_norm, uint16_t* feat, uint32_t* bad_value, hipStream_t st);
void rc_launch_pack(const float* pos, const uint32_t* idx, const uint32_t* order, uint32_t n_tris,
                    float4* tris, bool raw, hipStream_t st);
void rc_launch_fill_u32(uint32_t* p, uint32_t value, uint32_t n, hipStream_t st);
void rc_launch_record_o2w(const float* xf, const uint32_t* body_ids, uint32_t n, uint32_t scene_bodies, float* o2w,
                          hipStream_t st);
void rc_launch_transform(const float* rest, float* pos, const float* nrm_rest, float* nrm,
                         const uint32_t* body_vrange, const float* xf, const uint32_t* body_ids, uint32_t n_bodies,
                         uint32_t max_count, uint32_t scene_bodies, uint32_t* bad_value, hipStream_t st);
void rc_launch_refit_level(Node4* nodes, const float* pos, const uint32_t* idx, const uint32_t* order,
                           uint32_t first, uint32_t count, hipStream_t st);
// Refit touching only moved bodies (k_shade.hip): tri_node[t] = node holding triangle t in a leaf; moved
// bodies mark the nodes holding their triangles; the refit recomputes, level by level from the deepest, the
// marked nodes, which mark their parents.
void rc_launch_tri_nodes(const Node4* nodes, uint32_t n_nodes, const uint32_t* order, uint32_t* tri_node,
                         hipStream_t st);
void rc_launch_mark_dirty(const uint32_t* body_ids, uint32_t n, uint32_t n_bodies, uint32_t max_body_tris,
                          const uint32_t* tri_off, const uint32_t* body_tris, const uint32_t* tri_node, uint32_t* dirty,
                          uint32_t n_nodes, hipStream_t st);
void rc_launch_refit_dirty(Node4* nodes, const float* pos, const uint32_t* idx, const uint32_t* order, float4* tris,
                           bool raw, uint32_t* dirty, const std::vector<uint32_t>& level_start, hipStream_t st);
