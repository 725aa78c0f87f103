/*
 * raycast.h — C ABI of the MI355X ray-cast rendering library.
 *
 * The library renders triangle scenes by software ray casting on AMD CDNA4
 * (gfx950): primary visibility into a G-buffer, shadow rays towards point
 * lights (hard shadows) or a rectangular area light (soft shadows),
 * Cook-Torrance/GGX shading and a 2x2 supersampling resolve.  These are the
 * rendering features of the paper's Sec. IV-B (physically based rendering,
 * anti-aliasing, ray-traced shadows), recast as compute kernels; the
 * acceleration structure is the BVH that Sec. IV-B ("Ray-traced shadows")
 * builds for logarithmic-time ray queries.
 *
 * Conventions for every entry point
 *  - Return value: RC_OK (0) or a negative rc_status.  No C++ exception crosses
 *    the ABI.  A failed call leaves its outputs unspecified and all handles valid.
 *  - Pointers named d_* are device pointers (e.g. from torch); all others are host
 *    pointers.  The caller owns every input and output buffer; the library owns the
 *    handles it creates and every device buffer reachable only through them.
 *  - Work is enqueued on the context's HIP stream and is asynchronous: outputs are
 *    valid after that stream is synchronised.  Host inputs may be freed when the call
 *    returns; device inputs must stay valid until the stream reaches the work.
 *  - Device faults detected after a call returned are sticky: rc_get_last_error
 *    reports (and clears) them.
 *  - A context is used by one host thread at a time.
 */
#ifndef RAYCAST_H
#define RAYCAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rc_status {
    RC_OK = 0,
    RC_ERR_INVALID_ARG = -1,     /* null pointer, zero or out-of-range size, unknown option */
    RC_ERR_INVALID_VALUE = -2,   /* NaN/Inf coordinate, index out of range, bad material */
    RC_ERR_OUT_OF_MEMORY = -3,   /* device allocation failed */
    RC_ERR_HIP = -4,             /* HIP runtime error (no device, launch failure, fault) */
    RC_ERR_NOT_BUILT = -5,       /* render or refit before rc_bvh_build */
    RC_ERR_QUEUE_OVERFLOW = -6,  /* a device work queue or traversal stack exceeded its bound */
    RC_ERR_BAD_CHECKPOINT = -7,  /* denoiser checkpoint unreadable, wrong magic/version/shape/CRC */
    RC_ERR_UNSUPPORTED = -8      /* valid request this build does not implement */
} rc_status;

typedef struct rc_ctx rc_ctx;
typedef struct rc_scene rc_scene;

/* Static string for a status code (never NULL). */
const char* rc_status_string(int status);

/* Library version as major*10000 + minor*100 + patch. */
int rc_version(void);

/* Create a context on HIP device `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  Fails with RC_ERR_HIP when no usable gfx9 device exists. */
int rc_create(rc_ctx** out, int device, void* hip_stream);
int rc_destroy(rc_ctx* ctx);
int rc_set_stream(rc_ctx* ctx, void* hip_stream);
/* Report and clear the sticky device errors (synchronises the stream): RC_ERR_QUEUE_OVERFLOW when a
 * kernel exceeded a work-queue or stack bound, else RC_ERR_INVALID_VALUE when a kernel met an input it
 * cannot use (a hit id beyond the scene's triangles in rc_shade / rc_pack_features), else any error of
 * an asynchronous call, else RC_OK. */
int rc_get_last_error(rc_ctx* ctx);

/* ---------------------------------------------------------------- scene ---- */
/* Geometry and materials, all host arrays copied at creation.
 *  positions      n_vertices x 3 float, world space, finite
 *  indices        n_tris x 3 uint32 < n_vertices (counter-clockwise winding gives
 *                 the geometric normal e1 x e2; shading is two-sided)
 *  tri_material   n_tris uint32 < n_materials
 *  materials      n_materials x 5 float: albedo rgb in [0,1] (linear), roughness r in
 *                 [0.01,1] (GGX alpha = r^2), metallic in [0,1] (glTF metallic-roughness)
 *  body_vertex_range  n_bodies x 2 uint32 (first vertex, count): the rigid bodies that
 *                 rc_scene_set_transforms may move (may be NULL when n_bodies = 0).
 *  normals        NULL, or n_vertices x 3 float vertex normals (finite, not zero; need not
 *                 be unit): the shading normal of a hit is then their barycentric
 *                 interpolation (see rc_render); moved bodies rotate them with R.
 * Zero-area triangles are accepted and never hit.  Errors: RC_ERR_INVALID_ARG,
 * RC_ERR_INVALID_VALUE, RC_ERR_OUT_OF_MEMORY. */
typedef struct rc_scene_desc {
    const float* positions;
    uint32_t n_vertices;
    const uint32_t* indices;
    uint32_t n_tris;
    const uint32_t* tri_material;
    const float* materials;
    uint32_t n_materials;
    const uint32_t* body_vertex_range;
    uint32_t n_bodies;
    const float* normals;
} rc_scene_desc;

int rc_scene_create(rc_ctx* ctx, const rc_scene_desc* desc, rc_scene** out);
int rc_scene_destroy(rc_ctx* ctx, rc_scene* scene);

/* --------------------------------------------------------------- BVH ---- */
/* Build the scene's BVH, the acceleration structure that lets a ray find its hits in
 * logarithmic time (Sec. IV-B, "Ray-traced shadows"), as a 4-wide BVH with all four
 * child boxes of a node in one 128-byte record, nodes in breadth-first level order.
 * `method` RC_BUILD_HOST_SAH (0, default): binned SAH on the host (`bins` bins per axis,
 * default 32; `node_cost` = SAH cost of visiting a node relative to one triangle test,
 * default 4, range (0, 64], deciding when a range of at most max_leaf triangles becomes a
 * leaf), then uploaded.  RC_BUILD_DEVICE_LBVH (1): built on the GPU from the positions
 * already there: triangles sorted by the 63-bit Morton code of their box centroid in the
 * centroid bounds (stable, ties by triangle id), the binary radix tree over the sorted
 * codes, exact FP32 boxes bottom-up, then collapsed level by level to 4-wide (a node
 * repeatedly opens its child of largest box surface that holds more than max_leaf
 * triangles, until it has four children); every subtree of at most max_leaf triangles
 * is one leaf (`bins` and `node_cost` are ignored).  RC_BUILD_TWO_LEVEL (2): the paper's
 * two-level structure (Sec. IV-B "Ray-traced shadows": one structure per mesh, instances
 * with transforms under a top level rebuilt every frame): one bottom-level tree per body
 * over its rest-frame triangles (the positions given at creation), built on the GPU like
 * RC_BUILD_DEVICE_LBVH in one pass over all bodies, and a top level with one leaf per body
 * over the bodies' world boxes (the rest box's corners mapped by the body's current rigid
 * map [R | t] in FP32, padded by 2^-18 of the largest coordinate magnitude, at least 1).
 * Rays meet a body in its own frame: o' = M o + m, d' = M d with M = R^T and
 * m = -(R^T t), every component evaluated in FP32 as ((M0 a0 + M1 a1) + M2 a2) [+ m_k]
 * (m_k likewise from R and t), then the same FP32 box and triangle tests.  Every triangle
 * must belong to a body (all three vertices in one body's vertex range) and the bodies
 * must own consecutive triangle ranges in body order (else RC_ERR_INVALID_VALUE; no bodies:
 * RC_ERR_INVALID_ARG).  All methods give exact child boxes (FP32 min/max of what the child
 * holds) and leaves of at most `max_leaf` (1..4, default 4) triangles.  Replaces any previous
 * BVH.  Synchronous with respect to the host (works on the context stream and waits for it). */
enum { RC_BUILD_HOST_SAH = 0u, RC_BUILD_DEVICE_LBVH = 1u, RC_BUILD_TWO_LEVEL = 2u, RC_BUILD_DEVICE_SAH = 3u };
/* RC_BUILD_DEVICE_SAH (3): the binned SAH of RC_BUILD_HOST_SAH built on the GPU from the positions already there,
 * with the same arithmetic (bins per axis from the centroid bounds, bin = (int)(((double)c - lo) * (bins /
 * (double)(hi - lo))), split costs area(left) n_left + area(right) n_right in FP64 from exact FP32 boxes, the first
 * minimum over axis then bin, the same leaf rule, coinciding centroids halved), so that it chooses the host build's
 * splits; ranges are partitioned stably (the leaf order within a range may differ from the host build's), and the
 * binary tree is collapsed to 4-wide by the same rule (open the child of largest surface until four children).
 * bins <= 64 (else RC_ERR_UNSUPPORTED). */
/* flags: RC_BUILD_WATERTIGHT makes every ray/triangle test of the scene the watertight test
 * of Woop, Benthin and Wald (JCGT 2013) instead of Moller-Trumbore: vertices relative to the
 * ray origin, sheared with kz = axis of the largest |d| (first on ties), kx and ky the next
 * axes cyclically (swapped when d[kz] < 0), Sx = d[kx]/d[kz], Sy = d[ky]/d[kz], Sz = 1/d[kz]
 * (FP32, correctly rounded), X' = X[kx] - Sx X[kz], Y' = X[ky] - Sy X[kz]; edge functions
 * U = C'x B'y - C'y B'x, V = A'x C'y - A'y C'x, W = B'x A'y - B'y A'x (each product rounded,
 * then the difference; all three recomputed in FP64 and rounded to FP32 when one is zero);
 * a crossing needs U, V, W of one sign (zeros allowed, not all); det = (U + V) + W != 0,
 * T = (U Sz A[kz] + V Sz B[kz]) + W Sz C[kz] (products rounded, sums left to right),
 * t = T rcp(det), u = V rcp(det), v = W rcp(det) with the hardware reciprocal, hit when
 * t > 0 and within the ray's range.  Rays aimed at a shared edge or vertex of a mesh then
 * never pass between its triangles.  Triangles are stored as raw vertices; batched
 * rendering (rc_render_batch) does not support such scenes (RC_ERR_UNSUPPORTED). */
enum { RC_BUILD_WATERTIGHT = 1u };
typedef struct rc_build_opts {
    uint32_t bins;
    uint32_t max_leaf;
    float node_cost;
    uint32_t method;
    uint32_t flags;
} rc_build_opts;
int rc_bvh_build(rc_ctx* ctx, rc_scene* scene, const rc_build_opts* opts);

/* Rigid motion of bodies: for i < n, body d_body_ids[i] gets vertices
 * x' = R x_rest + t with d_xforms[12 i ..] = row-major [R | t] (3x4 float), each component
 * as ((R_k0 x + R_k1 y) + R_k2 z) + t_k in FP32, where x_rest are the positions given at
 * creation; vertex normals (if any) become ((R_k0 nx + R_k1 ny) + R_k2 nz) of the normals
 * given at creation; and [R | t] becomes the body's current map
 * (read by two-level structures).  Bodies not listed keep their current positions and map.
 * Does not touch the BVH: call rc_bvh_refit (or rc_tlas_rebuild) before rendering. */
int rc_scene_set_transforms(rc_ctx* ctx, rc_scene* scene, const float* d_xforms,
                            const uint32_t* d_body_ids, uint32_t n);

/* Copy the current vertex positions (n_vertices x 3 float) to host memory `out`.  Synchronous. */
int rc_scene_get_positions(rc_ctx* ctx, const rc_scene* scene, float* out);

/* Recompute every node box bottom-up from the current vertex positions, keeping the
 * tree topology (exact FP32 min/max, so boxes equal a fresh computation bit for bit).
 * For a two-level structure: rebuild the top level from the bodies' current maps
 * (rc_tlas_rebuild on the context stream).  RC_ERR_NOT_BUILT without a prior rc_bvh_build. */
int rc_bvh_refit(rc_ctx* ctx, rc_scene* scene);

/* Rebuild the top level of a two-level structure from the bodies' current maps on `stream`
 * (a hipStream_t; NULL = the context stream): instance records, then the top-level tree
 * (LBVH over the bodies' world boxes, collapsed in one workgroup).  Enqueues only: no host
 * synchronisation and no allocation, so it can run on a second stream beside other work.
 * The caller orders it after the rc_scene_set_transforms it depends on and before the
 * renders that read it (events), and does not render the scene while it runs.  A top level
 * deeper than 24 levels leaves an empty tree and sets the context's error flag.
 * RC_ERR_UNSUPPORTED for scenes without a two-level structure. */
int rc_tlas_rebuild(rc_ctx* ctx, rc_scene* scene, void* stream);

/* Copy the instance records of a two-level structure to host memory: 16 words per body,
 * the world-to-object map [M | m] (12 floats, row-major) then the body's root node index
 * (uint32) and 3 zero words.  Synchronous. */
int rc_tlas_export(rc_ctx* ctx, const rc_scene* scene, float* inst_out);

typedef struct rc_bvh_stats {
    uint64_t n_nodes;      /* 4-wide internal nodes */
    uint64_t n_leaves;
    uint64_t n_tris;
    uint32_t depth;        /* levels of 4-wide nodes */
    uint32_t max_stack;    /* traversal stack entries that suffice for any ray */
    double sah_cost;       /* SAH cost (node 1, triangle 1) relative to the root box, of the current
                              (possibly refit) boxes */
    double build_ms;       /* time of the last rc_bvh_build (first kernel or host step to finished tree) */
    uint32_t n_instances;  /* two-level structures: bodies under the top level (0 for a flat BVH) */
    uint32_t tlas_levels;  /* two-level structures: levels of the current top level.  For these, n_nodes
                              counts bottom- and top-level nodes, depth = deepest bottom level + top
                              levels, and sah_cost is 0 (not computed) */
    uint32_t tlas_root;    /* two-level structures: node index of the top level's root (= bottom-level nodes) */
    uint32_t reserved;
} rc_bvh_stats;
int rc_bvh_get_stats(rc_ctx* ctx, const rc_scene* scene, rc_bvh_stats* out);

/* Copy the BVH to host memory for inspection: n_nodes*32 floats/uint32 words per node
 * (lo_x[4] hi_x[4] lo_y[4] hi_y[4] lo_z[4] hi_z[4] child[4] meta[4]) and the
 * triangle order (n_tris uint32, original triangle id per leaf slot).  Either pointer
 * may be NULL.  Child word: bit 31 set = leaf with (bits 28..30) = count - 1 and
 * (bits 0..27) = first slot; 0xFFFFFFFF = empty; otherwise an internal node index.
 * Two-level structures: the bottom-level nodes (body b's root is node b) followed by the
 * current top level (root at node n_nodes - top-level nodes); top-level leaf words hold
 * the body index in bits 0..27 (count 1). */
int rc_bvh_export(rc_ctx* ctx, const rc_scene* scene, uint32_t* nodes_out, uint32_t* tri_order_out);

/* ------------------------------------------------------------- render ---- */
/* Pinhole camera: right-handed, y up, pixel row 0 at the top; forward
 * f = normalize(target - eye), right r = normalize(f x up), up u = r x f.  Sample
 * offsets are (0.5, 0.5) for ssaa = 1; for ssaa = 2, sample k in 0..3 of pixel p lies
 * in sub-pixel cell (k & 1, k >> 1) with a jitter from Philox4x32-10 keyed by
 * (seed, frame) with counter (p, k, 0, 0). */
typedef struct rc_camera {
    float eye[3], target[3], up[3];
    float vfov_deg;
    int32_t width, height;
    int32_t ssaa;            /* 1 or 2 (2x2 samples) */
    uint32_t seed, frame;
} rc_camera;

typedef struct rc_point_light {
    float position[3];
    float intensity[3];      /* radiant intensity, RGB; falloff 1/d^2 */
} rc_point_light;

/* One-sided rectangle: emits radiance `radiance` towards the side of edge_u x edge_v. */
typedef struct rc_rect_light {
    float center[3], edge_u[3], edge_v[3];
    float radiance[3];
} rc_rect_light;

enum {
    RC_FLAG_TIMING = 1u,     /* record per-stage device times (rc_get_stage_times) */
    RC_FLAG_PER_LANE = 4u,     /* trace camera rays and shadow rays one ray per lane with per-lane stacks
                                  even where the wave-uniform traversal would be used (camera rays with
                                  ssaa = 2; point-light shadow rays from 1.5M samples per light and
                                  rect-light shadow rays from 3M rays per frame; BVH depth <= 42, under 2^25
                                  nodes and 2^32 bytes of packed triangles); same results outside the FP32
                                  band, for comparison */
    RC_FLAG_NO_SHADE = 8u,     /* rc_render: stop after the visibility stages; d_rgba and d_sample_rgba are
                                  left untouched (for a caller that shades later with rc_shade, e.g. from a
                                  denoised visibility) */
    RC_FLAG_COUNT = 16u,       /* rc_render: count rays cast, nodes visited and triangles tested
                                  (rc_get_stage_times); without it the wave-uniform shadow kernels run
                                  without their counters */
    RC_FLAG_WAVE = 32u         /* rc_render: shadow rays through the wave-uniform kernels (where the BVH
                                  allows them) also for passes below the sizes above, which by default go
                                  one ray per lane: a small pass lasts as long as its most divergent wave's
                                  walk.  Same results outside the FP32 band.  With RC_FLAG_PER_LANE:
                                  RC_ERR_INVALID_ARG */
};

typedef struct rc_render_opts {
    uint32_t area_samples;   /* light samples per pixel for the rect light (1..4096 when rect != NULL) */
    uint32_t area_stream;    /* independent Philox stream of the rect-light samples */
    uint32_t flags;
} rc_render_opts;

/* Outputs, all caller-owned device buffers, S = ssaa^2 samples per pixel:
 *  d_rgba         W*H*4 float: resolved linear RGBA (alpha = coverage)
 *  d_hit          W*H*S*4 uint32 per sample: (triangle id, t, u, v) with t, u, v as
 *                 float bits; id 0xFFFFFFFF on a miss (t = +inf)
 *  d_shadow       W*H*S uint32 per sample: bit l set iff point light l lights it
 *                 (required when n_lights > 0)
 *  d_visibility   W*H float: fraction of rect-light samples that reach the point
 *                 (required when rect != NULL; ssaa must then be 1)
 *  d_sample_rgba  optional W*H*S*4 float: per-sample radiance before the resolve. */
typedef struct rc_outputs {
    float* d_rgba;
    uint32_t* d_hit;
    uint32_t* d_shadow;
    float* d_visibility;
    float* d_sample_rgba;
} rc_outputs;

/* Render one camera.  Shading (linear HDR, no ambient term) sums over point lights
 * with bit set: f(wo, wi) I cos(n, wi) / d^2, with f = Lambert (1 - F)(1 - m) albedo / pi
 * + Cook-Torrance D F G / (4 (n.wo)(n.wi)): D = GGX with alpha = r^2, F = Schlick with
 * F0 = mix(0.04, albedo, m), G = Schlick-GGX with k = (r + 1)^2 / 8.  A rect light
 * adds its unshadowed centre-point term (intensity L_e A cos_L) times the visibility.
 * In f and cos, n is the shading normal: with vertex normals n0, n1, n2 (current pose,
 * FP32), normalize((1 - u - v) n0 + u n1 + v n2) in FP64 with the hit's barycentrics,
 * negated when it points away from the geometric normal ng (unit e1 x e2 turned towards
 * the viewer); without vertex normals, ng.  Shadow rays use ng: they start at
 * p + ng 2^-18 max(1, |p|_inf) and test hits with 0 < t < 1 on the segment to the light
 * (or light sample); they are cast only when ng . d > 0.
 * Errors: RC_ERR_INVALID_ARG, RC_ERR_NOT_BUILT, RC_ERR_UNSUPPORTED (ssaa not 1/2, or
 * ssaa 2 with a rect light), RC_ERR_HIP. */
int rc_render(rc_ctx* ctx, rc_scene* scene, const rc_camera* cam,
              const rc_point_light* lights, uint32_t n_lights,
              const rc_rect_light* rect, const rc_render_opts* opts, const rc_outputs* out);

/* The shading + resolve stage of rc_render alone, from given G-buffer, shadow masks and
 * visibility (for example a denoised visibility).  Same layouts, rules and argument checks as rc_render
 * (RC_ERR_NOT_BUILT before rc_bvh_build; RC_ERR_INVALID_VALUE for a non-finite camera or light).  A sample
 * whose hit id is neither 0xFFFFFFFF nor below the scene's triangle count (a G-buffer of another scene) is
 * shaded as a miss and sets the sticky RC_ERR_INVALID_VALUE reported by rc_get_last_error. */
int rc_shade(rc_ctx* ctx, rc_scene* scene, const rc_camera* cam, const rc_point_light* lights, uint32_t n_lights,
             const rc_rect_light* rect, const uint32_t* d_hit, const uint32_t* d_shadow, const float* d_visibility,
             float* d_rgba, float* d_sample_rgba);

/* Display post pass of a rendered image (Sec. IV-B: the main pass tone maps and gamma-corrects, the
 * post-processing pass applies FXAA).  d_rgba: W*H*4 float linear RGBA (16-byte aligned), e.g.
 * rc_render's d_rgba; d_out: W*H*4 uint8 sRGB RGBA.
 *  1. Per channel r = c / (1 + c) in FP32 with c = max(c, 0) (Reinhard); the sRGB transfer function of
 *     IEC 61966-2-1 in FP64 (12.92 v for v <= 0.0031308, else 1.055 v^(1/2.4) - 0.055) quantised as
 *     floor(255 s + 0.5); alpha quantised as floor(255 clamp(a, 0, 1) + 0.5).
 *  2. With flags & RC_POST_FXAA, fast approximate anti-aliasing on that 8-bit image (borders clamp):
 *     integer luma 77 R + 150 G + 29 B; a pixel is processed when the luma range of itself and its four
 *     neighbours is >= 2048 and 8 x range >= their maximum.  The edge runs along x when the second
 *     differences across rows, |NW - 2W + SW| + 2 |N - 2C + S| + |NE - 2E + SE|, are >= those across
 *     columns; the side is the neighbour across the edge with the larger luma step (N, or W, on ties);
 *     S2 = C + side, grad = that step.  Along the edge, for i = 1..12 in each direction, the sum of the
 *     luma at i and of its side neighbour ends the search where 2 |sum - S2| >= grad.  With d+, d- the
 *     end distances (13 when not found) and the nearer end (d+ < d-, else d-) found and departing from
 *     S2 in the opposite sense to 2C - S2, w_edge = 0.5f - (float)min(d+, d-) / (float)(d+ + d-), else 0.
 *     Sub-pixel: s = fminf((float)|2(N+S+E+W) + (NE+NW+SE+SW) - 12 C| / (float)(12 range), 1),
 *     t = ((-2 s + 3) s) s, w_sub = (t t) 0.75 (FP32, in that order); w = max(w_edge, w_sub);
 *     each colour channel a becomes floor(a + w (b - a) + 0.5) with b the side neighbour's; alpha kept.
 * Allocates a W*H*4-byte image on first use of a larger size (with FXAA).  Errors: RC_ERR_INVALID_ARG. */
enum { RC_POST_FXAA = 1u };
int rc_postprocess(rc_ctx* ctx, const float* d_rgba, uint32_t width, uint32_t height, uint32_t flags,
                   uint8_t* d_out);

/* rc_postprocess without any allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid allocation after set-up).  Same arguments, definition
 * and output as rc_postprocess; the tone-mapped intermediate image of the FXAA pass lives in a fixed per-GPU
 * scratch array of RC_POST_NOALLOC_MAX_PIXELS (2^22) pixels x 4 bytes = 16 MiB, set up by rc_create and held
 * until the process ends.  width x height above 2^22 gives RC_ERR_INVALID_ARG.  Every call on one GPU shares
 * that GPU's scratch: calls that overlap on one GPU (two streams, two contexts or two threads) race and must
 * be ordered by the caller.  Enqueues kernels only: no hipMalloc, hipFree or synchronisation.  RC_ERR_HIP if
 * rc_create could not obtain the scratch's device address. */
enum { RC_POST_NOALLOC_MAX_PIXELS = 1 << 22 };
int rc_postprocess_noalloc(rc_ctx* ctx, const float* d_rgba, uint32_t width, uint32_t height, uint32_t flags,
                           uint8_t* d_out);

/* Camera rays of every sample, exactly as the traversal generates them: d_origins and
 * d_dirs receive W*H*S x 3 float each (sample s = pixel * S + k).  For verification of the
 * FP32 ray definition. */
int rc_camera_rays(rc_ctx* ctx, const rc_camera* cam, float* d_origins, float* d_dirs);

/* Device milliseconds of the stages of the last rc_render made with RC_FLAG_TIMING:
 * ms[0] primary traversal, ms[1] shadow traversal, ms[2] shade + resolve, ms[3] whole
 * render.  Counts of the last rc_render made with RC_FLAG_COUNT, [0] primary and [1] shadow
 * traversal: rays cast, 4-wide nodes visited, triangles tested.  Synchronises the stream. */
typedef struct rc_stage_times {
    float ms[8];
    uint64_t rays[2];
    uint64_t node_visits[2];
    uint64_t tri_tests[2];
} rc_stage_times;
int rc_get_stage_times(rc_ctx* ctx, rc_stage_times* out);

/* ------------------------------------------------------------- batch ---- */
/* One view of a batch: a camera on one of the batch's scenes, lit by a range of the batch's
 * point lights, with its own outputs (layouts as in rc_outputs; d_shadow may be NULL when
 * n_lights = 0). */
typedef struct rc_view {
    uint32_t scene;            /* index into the scenes array */
    rc_camera camera;
    uint32_t light_first;      /* first light in the lights array */
    uint32_t n_lights;         /* <= 16 */
    float* d_rgba;
    uint32_t* d_hit;
    uint32_t* d_shadow;
} rc_view;

/* Tuning of the persistent batched kernels.  Zero fields take defaults (8, 8, 256, 40, max, 3). */
typedef struct rc_tune {
    uint32_t tile_w, tile_h;   /* work-item tile in pixels; tile_w * tile_h in 16..1024 */
    uint32_t queue_depth;      /* pixels a wave claims per atomic on the device queue (64..4096, multiple of 64) */
    uint32_t min_rays;         /* rays per wave kept in flight: a wave refills its idle lanes when fewer are busy (1..64) */
    uint32_t waves_per_simd;   /* resident waves per SIMD of the persistent grids (1..occupancy limit of the form's
                                  largest kernel; each launch is capped at its own kernel's limit) */
    uint32_t passes;           /* 1: one kernel traces, shades and resolves each pixel; 3: three kernels over all
                                  views (camera rays, shadow rays, shading + resolve), each with its own work queue */
} rc_tune;

enum {
    RC_FLAG_GRAPH = 2u         /* rc_render_batch: capture the launch as a hipGraph once per batch shape, then replay */
};

/* Render all views in persistent launches fed by device work queues (point lights and 2x2 or 1
 * sample per pixel): one launch, or one per stage (rc_tune.passes); with RC_FLAG_GRAPH one graph launch
 * either way.  Every view's outputs are bit-identical to rc_render of that view
 * alone with RC_FLAG_PER_LANE (the same per-lane traversal), for any tuning.  flags: RC_FLAG_TIMING (rc_get_stage_times ms[3]; with three passes and no graph also ms[0..2] per pass), RC_FLAG_COUNT (its counts: all rays in [0] for one pass, camera and shadow rays in [0] and [1] for three), RC_FLAG_GRAPH.  All
 * scenes must be built (flat BVHs: two-level structures give RC_ERR_UNSUPPORTED).  Errors:
 * RC_ERR_INVALID_ARG, RC_ERR_NOT_BUILT, RC_ERR_UNSUPPORTED, RC_ERR_HIP. */
int rc_render_batch(rc_ctx* ctx, rc_scene* const* scenes, uint32_t n_scenes, const rc_view* views, uint32_t n_views,
                    const rc_point_light* lights, uint32_t n_lights_total, const rc_tune* tune, uint32_t flags);

/* Time every candidate tuning (`reps` timed launches after one warm-up, median) on this batch and
 * return the fastest in *best (and its median ms in *best_ms).  candidates = NULL uses a built-in grid.
 * With cache_path != NULL, a JSON-lines file keyed by (GPU arch, CU count, batch-shape hash) is read
 * first (a hit skips the search) and the result appended.  Overwrites the views' outputs. */
int rc_autotune(rc_ctx* ctx, rc_scene* const* scenes, uint32_t n_scenes, const rc_view* views, uint32_t n_views,
                const rc_point_light* lights, uint32_t n_lights_total, const rc_tune* candidates, uint32_t n_candidates,
                uint32_t reps, const char* cache_path, rc_tune* best, float* best_ms);

/* ---------------------------------------------------------- denoiser ---- */
/* A U-Net that maps 1-sample area-light visibility plus G-buffer features to the many-sample
 * visibility.  Input features: N x H x W x 8 bfloat16 (NHWC, 16-byte aligned): 1-spp visibility,
 * log depth log(1+t)/log(1+depth_norm), shading normal xyz, albedo rgb; background pixels hold
 * (1, 1, 0, 0, 0, 0, 0, 0).  H and W must be multiples of 4.  Architecture: two 3x3 conv + ReLU
 * layers per level with 32/64/128 channels, 2x2 average pooling, nearest 2x upsampling with skip
 * concatenation, 1x1 head + sigmoid; 472,993 parameters in the order (per layer w[Cout][3][3][Cin],
 * b[Cout]) e1a e1b e2a e2b bna bnb d2a d2b d1a d1b, head w[32], head b[1].  BF16 weights and
 * activations with FP32 accumulation on the matrix cores; FP32 master weights and Adam state. */
typedef struct rc_denoiser rc_denoiser;
int rc_denoiser_n_params(void);
/* He-normal initialisation from `seed`, Adam state zero. */
int rc_denoiser_create(rc_ctx* ctx, uint32_t seed, rc_denoiser** out);
int rc_denoiser_destroy(rc_ctx* ctx, rc_denoiser* den);
/* Host copies (rc_denoiser_n_params() floats) of the FP32 parameters / the gradients of the last
 * training step; set_params also resets the Adam state.  Synchronous. */
int rc_denoiser_get_params(rc_ctx* ctx, const rc_denoiser* den, float* out);
int rc_denoiser_set_params(rc_ctx* ctx, rc_denoiser* den, const float* in);
int rc_denoiser_get_grads(rc_ctx* ctx, const rc_denoiser* den, float* out);
/* d_out: N*H*W float visibility in (0, 1), device memory, 4-byte aligned (else RC_ERR_INVALID_ARG), written
 * directly by the last layer's kernel (it must not overlap the features). */
int rc_denoiser_infer(rc_ctx* ctx, rc_denoiser* den, const uint16_t* d_features, uint32_t n, uint32_t h, uint32_t w,
                      float* d_out);
/* The same network evaluated in FP32 from the FP32 master weights (FP32 activations and accumulation,
 * the BF16 features as input): the full-precision copy that the BF16 inference is compared against.
 * Arguments as rc_denoiser_infer. */
int rc_denoiser_infer_fp32(rc_ctx* ctx, rc_denoiser* den, const uint16_t* d_features, uint32_t n, uint32_t h,
                           uint32_t w, float* d_out);
/* One Adam step (beta 0.9/0.999, eps 1e-8, bias-corrected) on the loss
 * sum(mask (y - target)^2) / max(sum(mask), 1); d_target and d_mask are N*H*W floats.  *loss_out
 * (optional, synchronises) receives the loss before the step. */
int rc_denoiser_train_step(rc_ctx* ctx, rc_denoiser* den, const uint16_t* d_features, const float* d_target,
                           const float* d_mask, uint32_t n, uint32_t h, uint32_t w, float lr, float* loss_out);
/* Checkpoint: header (magic, version, parameter count, step), FP32 weights, Adam m and v, CRC-32.
 * load rejects any mismatch with RC_ERR_BAD_CHECKPOINT and leaves the denoiser unchanged; the
 * caller then falls back to the plain many-sample shadow path. */
int rc_denoiser_save(rc_ctx* ctx, const rc_denoiser* den, const char* path);
int rc_denoiser_load(rc_ctx* ctx, rc_denoiser* den, const char* path);

/* Denoiser input features of a 1-sample-per-pixel render (d_hit and d_visibility as written by
 * rc_render with a rect light) into d_features (W*H*8 bfloat16).  A hit id beyond the scene's triangles is
 * packed as background and sets the sticky RC_ERR_INVALID_VALUE (rc_get_last_error).  RC_ERR_NOT_BUILT
 * before rc_bvh_build. */
int rc_pack_features(rc_ctx* ctx, rc_scene* scene, const rc_camera* cam, const uint32_t* d_hit,
                     const float* d_visibility, float depth_norm, uint16_t* d_features);

#ifdef __cplusplus
}
#endif
#endif /* RAYCAST_H */
