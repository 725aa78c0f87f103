// Library-owned objects behind the opaque handles of the C ABI.
#pragma once

#include <vector>

#include "rc_internal.h"

struct rc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int grid = 0;                         // persistent traversal grid (blocks)
    uint32_t* d_counters = nullptr;       // RC_COUNTER_WORDS: work queues and the error flag
    unsigned long long* d_rays = nullptr; // [0] primary, [1] shadow rays cast
    uint32_t* d_overflow = nullptr;
    size_t overflow_words = 0;
    uint32_t* d_counts = nullptr;         // rect-light counters per pixel, then shadow-ray setup per sample
    size_t counts_cap = 0;                // in 32-bit words
    uint8_t* d_post = nullptr;            // tone-mapped image between the two post-pass kernels
    size_t post_cap = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool timed = false;
    bool timed_batch = false;
    int sticky = RC_OK;
    // batched rendering: device table, pinned staging copy, captured graph
    uint8_t* d_table = nullptr;
    uint8_t* h_table = nullptr;
    size_t table_cap = 0;
    hipEvent_t ev_staging = nullptr;
    bool staging_pending = false;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    uint64_t graph_key = 0;
    float4* d_bsetup = nullptr;           // shadow-ray setup of the batch's three-kernel form, per sample
    size_t bsetup_cap = 0;                // in float4
};

struct rc_scene {
    std::vector<float> pos;
    std::vector<uint32_t> idx, tri_mat, body_vr;
    std::vector<float> mats;
    uint32_t nv = 0, nt = 0, nm = 0, nb = 0, max_body_verts = 0;
    float* d_pos = nullptr;
    float* d_rest = nullptr;
    std::vector<float> nrm;            // vertex normals as given (empty: none)
    float* d_nrm = nullptr;            // current vertex normals
    float* d_nrm_rest = nullptr;       // vertex normals at creation (when bodies can move)
    uint32_t* d_idx = nullptr;
    uint32_t* d_tri_mat = nullptr;
    float* d_mats = nullptr;
    uint32_t* d_body_vr = nullptr;
    bool host_pos_stale = false;
    // BVH
    bool built = false;
    HostBvh hb;
    Node4* d_nodes = nullptr;
    uint32_t* d_order = nullptr;
    float4* d_tris = nullptr;
    double build_ms = 0.0;
    float scale = 1.0f;
    bool sah_stale = false;   // boxes refit on the device since the host copy was made
    // two-level structure (RC_BUILD_TWO_LEVEL): bottom-level trees = nodes 0 .. blas_nodes-1 (body b's root
    // is node b, over rest positions), top level from node blas_nodes on, rebuilt from the bodies' maps
    float* d_o2w = nullptr;   // per body [R | t], row-major 3x4 (identity until the body is moved)
    bool two_level = false;
    bool watertight = false;  // triangle records (v0, v1, v2) and the watertight test (RC_BUILD_WATERTIGHT)
    DevInst* d_inst = nullptr;
    uint32_t blas_nodes = 0, blas_depth = 0;
    TlasWork tlas;
    // dirty-node refit of a flat BVH: per body the triangles with a vertex in it (CSR over bodies, built at
    // creation when the bodies' vertex ranges do not overlap), per triangle the node holding it in a leaf, per
    // node a flag marked by moved bodies (both allocated with a flat BVH of a scene with bodies)
    uint32_t* d_body_tri_off = nullptr;
    uint32_t* d_body_tris = nullptr;
    uint32_t max_body_tris = 0;
    uint32_t* d_tri_node = nullptr;
    uint32_t* d_dirty = nullptr;      // one mark per node
    uint32_t refit_nodes = 0;         // nodes covered by d_dirty
};
