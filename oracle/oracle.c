/*
 * CPU oracle for the ray-cast rendering path — TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load this library.  The product (the HIP library) never calls it, and the two
 * share no code: no headers, helpers, tables or constants.
 *
 * Everything here is the plain definition, evaluated in FP64 from the FP32
 * inputs (which FP64 holds exactly), except where a bit-exact FP32 mirror is
 * the definition itself (camera rays, vertex transforms, the resolve order):
 *
 *  - Closest hit / any hit (the acceleration structure of Sec. IV-B "Ray-traced
 *    shadows" only speeds up an exact answer): the closest, resp. any, hit over
 *    ALL triangles, Moller-Trumbore in FP64, ties to the smaller triangle id.
 *    The oracle's own BVH (median split) only prunes; it is checked against
 *    brute force.  Every query also reports whether the answer is inside the
 *    FP32 "band": the set of rays for which some triangle's FP32 hit decision
 *    or hit order is not certain under a running forward-error bound of the
 *    FP32 Moller-Trumbore evaluation (times a safety factor c).
 *  - Hard shadows (Sec. IV-B): a ray from the surface point towards the light;
 *    any opaque hit strictly between them means the light is blocked.
 *  - Shading (Sec. IV-B, the Cook-Torrance equation): GGX normal distribution,
 *    Schlick Fresnel with F0 from the metallic-roughness workflow, Schlick-GGX
 *    geometry term; plus a Lambert diffuse lobe.
 *  - Anti-aliasing (Sec. IV-B): supersampling, i.e. every sample shaded and
 *    the samples box-averaged in a fixed order.
 *
 * Readings where the paper is silent are listed in the design notes; the
 * ones that change numbers are restated next to the code that uses them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_API __attribute__((visibility("default")))
#define NO_HIT 0xFFFFFFFFu

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the        */
/* multiply-xorshift round with the published multipliers and Weyl key bumps. */
/* ------------------------------------------------------------------------- */
OR_API void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 24-bit uniform in [0,1): exact in FP32 and FP64. */
static double unit24(uint32_t x) { return (double)(x >> 8) * 0x1p-24; }
static float unit24f(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

/* ------------------------------------------------------------------------- */
/* Camera: FP32 mirror of the ray definition (no contraction, IEEE RNE,       */
/* correctly rounded sqrt and divide).  Right-handed, y up; pixel row 0 is   */
/* the top row.                                                               */
/* ------------------------------------------------------------------------- */
typedef struct {
    float eye[3], target[3], up[3];
    float vfov_deg;
    int32_t width, height, ssaa;
    uint32_t seed, frame;
} or_camera;

typedef struct { float f[3], r[3], u[3]; float tan_half, x_scale; } cam_basis;

static void f_normalize(float v[3])
{
    float n2 = v[0] * v[0] + v[1] * v[1];
    n2 = n2 + v[2] * v[2];
    float len = sqrtf(n2);
    v[0] = v[0] / len; v[1] = v[1] / len; v[2] = v[2] / len;
}

static void f_cross(const float a[3], const float b[3], float o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static void camera_basis(const or_camera* c, cam_basis* b)
{
    for (int k = 0; k < 3; ++k) b->f[k] = c->target[k] - c->eye[k];
    f_normalize(b->f);
    f_cross(b->f, c->up, b->r);
    f_normalize(b->r);
    f_cross(b->r, b->f, b->u);
    /* half field of view: tan evaluated in FP64, rounded once to FP32 */
    b->tan_half = (float)tan((double)c->vfov_deg * (3.14159265358979323846 / 360.0));
    float aspect = (float)c->width / (float)c->height;
    b->x_scale = b->tan_half * aspect;
}

static void sample_offset(const or_camera* c, uint32_t pixel, uint32_t k, float* ox, float* oy)
{
    if (c->ssaa <= 1) { *ox = 0.5f; *oy = 0.5f; return; }
    uint32_t ctr[4] = {pixel, k, 0u, 0u}, key[2] = {c->seed, c->frame}, r[4];
    or_philox4x32_10(ctr, key, r);
    *ox = ((float)(k & 1u) + unit24f(r[0])) * 0.5f;
    *oy = ((float)(k >> 1) + unit24f(r[1])) * 0.5f;
}

static void gen_ray(const or_camera* c, const cam_basis* b, int64_t s, float o[3], float d[3])
{
    int64_t spp = (int64_t)c->ssaa * c->ssaa;
    uint32_t pixel = (uint32_t)(s / spp), k = (uint32_t)(s % spp);
    uint32_t i = pixel % (uint32_t)c->width, j = pixel / (uint32_t)c->width;
    float ox, oy;
    sample_offset(c, pixel, k, &ox, &oy);
    float px = (2.0f * ((float)i + ox)) / (float)c->width;
    px = (px - 1.0f) * b->x_scale;
    float py = (2.0f * ((float)j + oy)) / (float)c->height;
    py = (1.0f - py) * b->tan_half;
    for (int a = 0; a < 3; ++a) {
        float t0 = px * b->r[a];
        float t1 = py * b->u[a];
        d[a] = (t0 + t1) + b->f[a];
        o[a] = c->eye[a];
    }
    f_normalize(d);
}

OR_API void or_gen_rays(const or_camera* c, const int64_t* samples, int64_t n, float* o, float* d)
{
    cam_basis b;
    camera_basis(c, &b);
    for (int64_t q = 0; q < n; ++q) gen_ray(c, &b, samples[q], o + 3 * q, d + 3 * q);
}

/* ------------------------------------------------------------------------- */
/* FP64 vectors                                                               */
/* ------------------------------------------------------------------------- */
typedef struct { double x, y, z; } v3;
static v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 cross(v3 a, v3 b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static double len(v3 a) { return sqrt(dot(a, a)); }
static v3 nrm(v3 a) { return scl(a, 1.0 / len(a)); }
static double amax(v3 a) { return fmax(fabs(a.x), fmax(fabs(a.y), fabs(a.z))); }
static double comp(v3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
static v3 from_f(const float* p) { return mk(p[0], p[1], p[2]); }

/* ------------------------------------------------------------------------- */
/* Running forward-error bounds of an FP32 evaluation.                        */
/* ev = (value computed in FP64 ~ exact, bound on |FP32 result - value|).     */
/* u = 2^-24 is the FP32 unit roundoff.                                       */
/* ------------------------------------------------------------------------- */
typedef struct { double v, e; } ev;
static const double U32R = 0x1p-24;
static ev ev_x(double v, double e) { ev r = {v, e}; return r; }
static ev ev_add(ev a, ev b) { double v = a.v + b.v, e = a.e + b.e; return ev_x(v, e + U32R * (fabs(v) + e)); }
static ev ev_sub(ev a, ev b) { double v = a.v - b.v, e = a.e + b.e; return ev_x(v, e + U32R * (fabs(v) + e)); }
static ev ev_mul(ev a, ev b)
{
    double v = a.v * b.v;
    double e = fabs(a.v) * b.e + fabs(b.v) * a.e + a.e * b.e;
    return ev_x(v, e + U32R * (fabs(v) + e));
}
typedef struct { ev x, y, z; } ev3;
static ev3 ev3_sub(ev3 a, ev3 b) { ev3 r = {ev_sub(a.x, b.x), ev_sub(a.y, b.y), ev_sub(a.z, b.z)}; return r; }
static ev ev3_dot(ev3 a, ev3 b) { return ev_add(ev_add(ev_mul(a.x, b.x), ev_mul(a.y, b.y)), ev_mul(a.z, b.z)); }
static ev3 ev3_cross(ev3 a, ev3 b)
{
    ev3 r = {ev_sub(ev_mul(a.y, b.z), ev_mul(a.z, b.y)),
             ev_sub(ev_mul(a.z, b.x), ev_mul(a.x, b.z)),
             ev_sub(ev_mul(a.x, b.y), ev_mul(a.y, b.x))};
    return r;
}
static ev3 ev3_exact(v3 a) { ev3 r = {{a.x, 0}, {a.y, 0}, {a.z, 0}}; return r; }
/* correctly rounded FP32 quotient; the divisor's interval must exclude zero (else the bound is infinite) */
static ev ev_div(ev a, ev b)
{
    double v = a.v / b.v;
    double lo = fabs(b.v) - b.e;
    double e = lo > 0.0 ? (a.e + fabs(v) * b.e) / lo : INFINITY;
    return ev_x(v, e + U32R * (fabs(v) + e));
}
static ev ev3_comp(ev3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
/* an FP64 vector that the FP32 side holds rounded to FP32 (<= half an ulp per component) */
static ev3 ev3_rounded(v3 a) { ev3 r = {{a.x, U32R * fabs(a.x)}, {a.y, U32R * fabs(a.y)}, {a.z, U32R * fabs(a.z)}}; return r; }

/* ------------------------------------------------------------------------- */
/* Triangles and the exact Moller-Trumbore test with FP32 certainty.          */
/* ------------------------------------------------------------------------- */
struct or_inst;
typedef struct {
    const float* pos; int64_t nv;
    const uint32_t* idx; int64_t nt;
    const uint32_t* tri_mat;
    const float* mats; int64_t nmat;    /* albedo rgb, roughness, metallic */
    const struct or_inst* inst;         /* NULL, or the instances that answer hit queries (two-level) */
    int64_t flags;                      /* bit 0: the FP32 side tests triangles watertight (band model) */
    const float* nrm;                   /* NULL, or nv x 3 vertex normals (smooth shading normal) */
} or_scene;

static void tri_verts(const or_scene* s, uint32_t t, v3* a, v3* b, v3* c)
{
    const uint32_t* ix = s->idx + 3 * (int64_t)t;
    *a = from_f(s->pos + 3 * (int64_t)ix[0]);
    *b = from_f(s->pos + 3 * (int64_t)ix[1]);
    *c = from_f(s->pos + 3 * (int64_t)ix[2]);
}

enum { ST_FAIL = 0, ST_PASS = 1, ST_UNC = 2 };

typedef struct {
    int exact_hit;          /* FP64 Moller-Trumbore says hit, with tmin < t < tmax */
    int status;             /* FP32 outcome certainty: FAIL, PASS, UNC */
    double t, u, v;         /* FP64 values */
    double et, eu, ev;      /* bounds on the FP32 error of t, u, v (times c) */
} tri_test;

/* A ray as the FP32 side holds it: value + per-component error bound. */
typedef struct { v3 o, d; ev3 eo, ed; } ray_ev;

static int certain(double margin, double err) { return margin > err ? ST_PASS : (margin < -err ? ST_FAIL : ST_UNC); }

static void mt_test(const or_scene* s, uint32_t tri, const ray_ev* r, double tmin, double tmax, double c, tri_test* out)
{
    v3 a, b, cc;
    tri_verts(s, tri, &a, &b, &cc);
    /* FP64 Moller-Trumbore (Moller & Trumbore, JGT 1997) */
    v3 e1 = sub(b, a), e2 = sub(cc, a);
    v3 p = cross(r->d, e2);
    double det = dot(e1, p);
    v3 sv = sub(r->o, a);
    v3 q = cross(sv, e1);
    double u = 0, v = 0, t = 0;
    out->exact_hit = 0;
    if (det != 0.0) {
        u = dot(sv, p) / det;
        v = dot(r->d, q) / det;
        t = dot(e2, q) / det;
        out->exact_hit = (u >= 0.0 && v >= 0.0 && u + v <= 1.0 && t > tmin && t < tmax);
    }
    out->t = t; out->u = u; out->v = v;

    /* The same steps with FP32 error bounds: edges e1 = fl(v1 - v0), e2 = fl(v2 - v0). */
    ev3 A = ev3_exact(a), B = ev3_exact(b), C = ev3_exact(cc);
    ev3 E1 = ev3_sub(B, A), E2 = ev3_sub(C, A);
    ev3 P = ev3_cross(r->ed, E2);
    ev DET = ev3_dot(E1, P);
    ev3 S = ev3_sub(r->eo, A);
    ev3 Q = ev3_cross(S, E1);
    ev SP = ev3_dot(S, P), DQ = ev3_dot(r->ed, Q), TQ = ev3_dot(E2, Q);
    double edet = c * DET.e, esp = c * SP.e, edq = c * DQ.e, etq = c * TQ.e;

    if (fabs(DET.v) > edet) {
        /* determinant sign certain: interval quotients of the FP32 numerators over the
         * FP32 determinant, widened by the reciprocal (<= 1 ulp) and product roundings */
        double sg = DET.v > 0 ? 1.0 : -1.0;
        double dlo = fabs(DET.v) - edet, dhi = fabs(DET.v) + edet;
        double qlo[3], qhi[3];
        const double num[3] = {sg * SP.v, sg * DQ.v, sg * TQ.v}, en[3] = {esp, edq, etq};
        for (int k = 0; k < 3; ++k) {
            double a = num[k] - en[k], b = num[k] + en[k];
            double lo = fmin(a / dlo, a / dhi), hi = fmax(b / dlo, b / dhi);
            double w = 4.0 * c * U32R;
            qlo[k] = lo - w * fabs(lo);
            qhi[k] = hi + w * fabs(hi);
        }
        /* FP32 evaluates u + v <= 1 on the rounded quotients */
        double slo = (qlo[0] + qlo[1]), shi = (qhi[0] + qhi[1]);
        slo -= c * U32R * fabs(slo); shi += c * U32R * fabs(shi);
        int st[5];
        st[0] = qlo[0] >= 0.0 ? ST_PASS : (qhi[0] < 0.0 ? ST_FAIL : ST_UNC);
        st[1] = qlo[1] >= 0.0 ? ST_PASS : (qhi[1] < 0.0 ? ST_FAIL : ST_UNC);
        st[2] = shi <= 1.0 ? ST_PASS : (slo > 1.0 ? ST_FAIL : ST_UNC);
        st[3] = qlo[2] > tmin ? ST_PASS : (qhi[2] <= tmin ? ST_FAIL : ST_UNC);
        st[4] = isinf(tmax) ? ST_PASS : (qhi[2] < tmax ? ST_PASS : (qlo[2] >= tmax ? ST_FAIL : ST_UNC));
        int status = ST_PASS;
        for (int k = 0; k < 5; ++k) {
            if (st[k] == ST_FAIL) { status = ST_FAIL; break; }
            if (st[k] == ST_UNC) status = ST_UNC;
        }
        out->status = status;
        out->eu = fmax(u - qlo[0], qhi[0] - u);
        out->ev = fmax(v - qlo[1], qhi[1] - v);
        out->et = fmax(t - qlo[2], qhi[2] - t);
    } else {
        /* sign of the determinant not certain: the FP32 quotients are certainly outside
         * [0,1] when a numerator certainly exceeds the determinant in magnitude */
        double dmax = fabs(DET.v) + edet;
        if (fabs(SP.v) - esp > dmax || fabs(DQ.v) - edq > dmax) out->status = ST_FAIL;
        else out->status = ST_UNC;
        out->et = INFINITY; out->eu = INFINITY; out->ev = INFINITY;
    }
    if (out->status == ST_PASS && !out->exact_hit) out->status = ST_UNC; /* cannot happen; stay safe */
}

/* ------------------------------------------------------------------------- */
/* Watertight ray/triangle test (Woop, Benthin and Wald, JCGT 2013) as the    */
/* FP32 side evaluates it: kz = axis of the largest |d| (first on ties),      */
/* kx, ky the next axes cyclically, swapped when d[kz] < 0; Sx = d[kx]/d[kz], */
/* Sy = d[ky]/d[kz], Sz = 1/d[kz]; vertices relative to the origin, sheared:  */
/* X' = X[kx] - Sx X[kz], Y' = X[ky] - Sy X[kz]; edge functions               */
/* U = Cx By - Cy Bx, V = Ax Cy - Ay Cx, W = Bx Ay - By Ax (recomputed in FP64 */
/* when one is exactly zero); a hit needs U, V, W of one sign (not all zero); */
/* det = (U + V) + W, T = (U Sz A[kz] + V Sz B[kz]) + W Sz C[kz], t = T / det */
/* (reciprocal within 1 ulp), u = V / det, v = W / det.  In exact arithmetic  */
/* it decides the same geometric crossing as Moller-Trumbore, so only the     */
/* FP32 certainty (the band) depends on the test.                             */
/* ------------------------------------------------------------------------- */
static int wt_band_perm(const ray_ev* r, int kx, int ky, int kz, v3 a, v3 b, v3 cc, double tmin, double tmax,
                        double c, double* et, double* eu, double* evv)
{
    *et = *eu = *evv = INFINITY;
    ev dz = ev3_comp(r->ed, kz);
    if (fabs(dz.v) <= c * dz.e) return ST_UNC;
    ev Sx = ev_div(ev3_comp(r->ed, kx), dz), Sy = ev_div(ev3_comp(r->ed, ky), dz), Sz = ev_div(ev_x(1.0, 0.0), dz);
    ev3 V0 = ev3_sub(ev3_exact(a), r->eo), V1 = ev3_sub(ev3_exact(b), r->eo), V2 = ev3_sub(ev3_exact(cc), r->eo);
    ev Ax = ev_sub(ev3_comp(V0, kx), ev_mul(Sx, ev3_comp(V0, kz)));
    ev Ay = ev_sub(ev3_comp(V0, ky), ev_mul(Sy, ev3_comp(V0, kz)));
    ev Bx = ev_sub(ev3_comp(V1, kx), ev_mul(Sx, ev3_comp(V1, kz)));
    ev By = ev_sub(ev3_comp(V1, ky), ev_mul(Sy, ev3_comp(V1, kz)));
    ev Cx = ev_sub(ev3_comp(V2, kx), ev_mul(Sx, ev3_comp(V2, kz)));
    ev Cy = ev_sub(ev3_comp(V2, ky), ev_mul(Sy, ev3_comp(V2, kz)));
    ev U = ev_sub(ev_mul(Cx, By), ev_mul(Cy, Bx));
    ev V = ev_sub(ev_mul(Ax, Cy), ev_mul(Ay, Cx));
    ev W = ev_sub(ev_mul(Bx, Ay), ev_mul(By, Ax));
    const ev E[3] = {U, V, W};
    int pos = 0, neg = 0, unk = 0;
    for (int k = 0; k < 3; ++k) {
        if (E[k].v > c * E[k].e) ++pos;
        else if (E[k].v < -c * E[k].e) ++neg;
        else ++unk;
    }
    if (pos > 0 && neg > 0) return ST_FAIL;          /* certainly on both sides of some edge */
    if (unk > 0) return ST_UNC;
    ev det = ev_add(ev_add(U, V), W);
    ev Az = ev_mul(Sz, ev3_comp(V0, kz)), Bz = ev_mul(Sz, ev3_comp(V1, kz)), Cz = ev_mul(Sz, ev3_comp(V2, kz));
    ev T = ev_add(ev_add(ev_mul(U, Az), ev_mul(V, Bz)), ev_mul(W, Cz));
    double edet = c * det.e;
    if (!(fabs(det.v) > edet)) return ST_UNC;
    double sg = det.v > 0 ? 1.0 : -1.0;
    double dlo = fabs(det.v) - edet, dhi = fabs(det.v) + edet;
    const double num[3] = {sg * T.v, sg * V.v, sg * W.v}, en[3] = {c * T.e, c * V.e, c * W.e};
    double qlo[3], qhi[3];
    for (int k = 0; k < 3; ++k) {
        double lo_ = num[k] - en[k], hi_ = num[k] + en[k];
        double lo = fmin(lo_ / dlo, lo_ / dhi), hi = fmax(hi_ / dlo, hi_ / dhi);
        double w = 4.0 * c * U32R;
        qlo[k] = lo - w * fabs(lo);
        qhi[k] = hi + w * fabs(hi);
    }
    int st0 = qlo[0] > tmin ? ST_PASS : (qhi[0] <= tmin ? ST_FAIL : ST_UNC);
    int st1 = isinf(tmax) ? ST_PASS : (qhi[0] < tmax ? ST_PASS : (qlo[0] >= tmax ? ST_FAIL : ST_UNC));
    double t = num[0] / fabs(det.v), u = num[1] / fabs(det.v), v = num[2] / fabs(det.v);
    *et = fmax(t - qlo[0], qhi[0] - t);
    *eu = fmax(u - qlo[1], qhi[1] - u);
    *evv = fmax(v - qlo[2], qhi[2] - v);
    if (st0 == ST_FAIL || st1 == ST_FAIL) return ST_FAIL;
    if (st0 == ST_UNC || st1 == ST_UNC) return ST_UNC;
    return ST_PASS;
}

static void wt_band(const or_scene* s, uint32_t tri, const ray_ev* r, double tmin, double tmax, double c, tri_test* out)
{
    v3 a, b, cc;
    tri_verts(s, tri, &a, &b, &cc);
    const double dv[3] = {r->ed.x.v, r->ed.y.v, r->ed.z.v}, de[3] = {r->ed.x.e, r->ed.y.e, r->ed.z.e};
    int kz = 0;
    if (fabs(dv[1]) > fabs(dv[kz])) kz = 1;
    if (fabs(dv[2]) > fabs(dv[kz])) kz = 2;
    /* axes whose |d| may be the FP32 side's largest (its rounded values can order a near tie differently) */
    int cand[3], nc = 0;
    for (int k = 0; k < 3; ++k)
        if (k == kz || fabs(dv[k]) + de[k] * c >= fabs(dv[kz]) - de[kz] * c) cand[nc++] = k;
    int status = -1;
    double et = 0, eu = 0, evv = 0;
    for (int q = 0; q < nc; ++q) {
        const int z = cand[q];
        int x = (z + 1) % 3, y = (z + 2) % 3;
        /* the swap follows the sign of d[z]; an uncertain sign is covered by evaluating both orders */
        int orders = fabs(dv[z]) > c * de[z] ? 1 : 2;
        for (int o = 0; o < orders; ++o) {
            int sw = (dv[z] < 0.0) ^ (o == 1);
            int kx = sw ? y : x, ky = sw ? x : y;
            double a_, b_, c_;
            int st = wt_band_perm(r, kx, ky, z, a, b, cc, tmin, tmax, c, &a_, &b_, &c_);
            if (status < 0) status = st;
            else if (st != status) status = ST_UNC;
            et = fmax(et, a_); eu = fmax(eu, b_); evv = fmax(evv, c_);
        }
    }
    out->status = status;
    out->et = et; out->eu = eu; out->ev = evv;
    if (out->status == ST_PASS && !out->exact_hit) out->status = ST_UNC;   /* cannot happen; stay safe */
    if (out->status == ST_FAIL && out->exact_hit) out->status = ST_UNC;
}

/* the triangle test of the scene's FP32 side: exact answer + certainty */
static void tri_check(const or_scene* s, uint32_t tri, const ray_ev* r, double tmin, double tmax, double c, tri_test* out)
{
    mt_test(s, tri, r, tmin, tmax, c, out);
    if (s->flags & 1) wt_band(s, tri, r, tmin, tmax, c, out);
}

/* ------------------------------------------------------------------------- */
/* Oracle BVH: binary, median split on the longest centroid axis, <= 4 tris  */
/* per leaf, FP64 boxes.  It only prunes candidate triangles.                 */
/* ------------------------------------------------------------------------- */
typedef struct { double lo[3], hi[3]; int32_t left, right; int32_t first, count; } bnode;

typedef struct or_bvh {
    const or_scene* scene;
    bnode* nodes; int64_t n_nodes, cap;
    uint32_t* tris;
    double* cen;    /* centroids, 3 per triangle of the range, indexed by id - tri0 */
    int64_t tri0;   /* first triangle id of the range */
    double margin;  /* absolute box padding */
    int depth;
} or_bvh;

static void tri_bounds(const or_scene* s, uint32_t t, double lo[3], double hi[3])
{
    v3 a, b, c;
    tri_verts(s, t, &a, &b, &c);
    for (int k = 0; k < 3; ++k) {
        double x = comp(a, k), y = comp(b, k), z = comp(c, k);
        lo[k] = fmin(x, fmin(y, z));
        hi[k] = fmax(x, fmax(y, z));
    }
}

static void select_kth(uint32_t* t, const double* cen, int64_t base, int axis, int64_t lo, int64_t hi, int64_t k)
{
    /* quickselect: afterwards t[lo..k) <= t[k] <= t[k+1..hi) on the centroid axis */
    while (hi - lo > 1) {
        double pv = cen[3 * ((int64_t)t[lo + (hi - lo) / 2] - base) + axis];
        int64_t i = lo, j = hi - 1;
        while (i <= j) {
            while (cen[3 * ((int64_t)t[i] - base) + axis] < pv) ++i;
            while (cen[3 * ((int64_t)t[j] - base) + axis] > pv) --j;
            if (i <= j) { uint32_t tmp = t[i]; t[i] = t[j]; t[j] = tmp; ++i; --j; }
        }
        if (k <= j) hi = j + 1;
        else if (k >= i) lo = i;
        else return;
    }
}

static int32_t build_rec(or_bvh* B, int64_t first, int64_t count, int depth)
{
    if (B->n_nodes == B->cap) {
        B->cap *= 2;
        B->nodes = (bnode*)realloc(B->nodes, (size_t)B->cap * sizeof(bnode));
    }
    int32_t id = (int32_t)B->n_nodes++;
    if (depth > B->depth) B->depth = depth;
    bnode nd;
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < 3; ++k) { nd.lo[k] = INFINITY; nd.hi[k] = -INFINITY; }
    for (int64_t i = first; i < first + count; ++i) {
        double lo[3], hi[3];
        tri_bounds(B->scene, B->tris[i], lo, hi);
        for (int k = 0; k < 3; ++k) {
            nd.lo[k] = fmin(nd.lo[k], lo[k]); nd.hi[k] = fmax(nd.hi[k], hi[k]);
            double cv = B->cen[3 * ((int64_t)B->tris[i] - B->tri0) + k];
            clo[k] = fmin(clo[k], cv); chi[k] = fmax(chi[k], cv);
        }
    }
    for (int k = 0; k < 3; ++k) { nd.lo[k] -= B->margin; nd.hi[k] += B->margin; }
    nd.first = (int32_t)first; nd.count = (int32_t)count; nd.left = nd.right = -1;
    if (count > 4) {
        int axis = 0;
        for (int k = 1; k < 3; ++k) if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
        int64_t mid = first + count / 2;
        select_kth(B->tris, B->cen, B->tri0, axis, first, first + count, mid);
        nd.count = 0;
        B->nodes[id] = nd;
        int32_t l = build_rec(B, first, mid - first, depth + 1);
        int32_t r = build_rec(B, mid, first + count - mid, depth + 1);
        B->nodes[id].left = l; B->nodes[id].right = r;
        return id;
    }
    B->nodes[id] = nd;
    return id;
}

/* BVH over the triangles first .. first + count - 1 of the scene (ids stay the scene's) */
static or_bvh* bvh_build_range(const or_scene* s, int64_t first, int64_t count, double scale)
{
    or_bvh* B = (or_bvh*)calloc(1, sizeof(or_bvh));
    B->scene = s;
    B->cap = 1024;
    B->nodes = (bnode*)malloc((size_t)B->cap * sizeof(bnode));
    B->tris = (uint32_t*)malloc((size_t)(count > 0 ? count : 1) * sizeof(uint32_t));
    B->cen = (double*)malloc((size_t)(count > 0 ? count : 1) * 3 * sizeof(double));
    B->tri0 = first;
    /* pad boxes well beyond FP32 rounding of the GPU box test and of the hit decisions */
    B->margin = 1e-4 * scale;
    for (int64_t i = 0; i < count; ++i) {
        int64_t t = first + i;
        v3 a, b, c;
        tri_verts(s, (uint32_t)t, &a, &b, &c);
        B->tris[i] = (uint32_t)t;
        B->cen[3 * i + 0] = (a.x + b.x + c.x) / 3.0;
        B->cen[3 * i + 1] = (a.y + b.y + c.y) / 3.0;
        B->cen[3 * i + 2] = (a.z + b.z + c.z) / 3.0;
    }
    if (count > 0) build_rec(B, 0, count, 0);
    return B;
}

static double scene_scale(const or_scene* s)
{
    double scale = 1.0;
    for (int64_t i = 0; i < 3 * s->nv; ++i) scale = fmax(scale, fabs((double)s->pos[i]));
    return scale;
}

OR_API or_bvh* or_bvh_build(const or_scene* s) { return bvh_build_range(s, 0, s->nt, scene_scale(s)); }

OR_API void or_bvh_free(or_bvh* B)
{
    if (!B) return;
    free(B->nodes); free(B->tris); free(B->cen); free(B);
}

OR_API int64_t or_bvh_nodes(const or_bvh* B) { return B->n_nodes; }
OR_API int or_bvh_depth(const or_bvh* B) { return B->depth; }

/* slab test in FP64 against a padded box; returns entry distance or +inf */
static double box_enter(const bnode* n, const ray_ev* r, double tmin, double tmax)
{
    double t0 = tmin, t1 = tmax;
    for (int k = 0; k < 3; ++k) {
        double o = comp(r->o, k), d = comp(r->d, k);
        if (d == 0.0) {
            if (o < n->lo[k] || o > n->hi[k]) return INFINITY;
            continue;
        }
        double a = (n->lo[k] - o) / d, b = (n->hi[k] - o) / d;
        if (a > b) { double tmp = a; a = b; b = tmp; }
        t0 = fmax(t0, a); t1 = fmin(t1, b);
        if (t0 > t1) return INFINITY;
    }
    return t0;
}

/* ------------------------------------------------------------------------- */
/* Closest hit and any hit, with the band decision.                           */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint32_t id; double t, u, v; double et, eu, ev;
    int band;
    int64_t n_candidates;
} hit_rec;

typedef struct {
    int have_best; uint32_t best_id; double best_t, best_thi; int best_status;
    tri_test best;
    double pass_lo1, pass_lo2; uint32_t pass_id1;
    double unc_lo;
    int64_t n_cand;
} closest_acc;

static void closest_consider(closest_acc* A, uint32_t tri, const tri_test* tt)
{
    if (tt->status == ST_FAIL && !tt->exact_hit) return;
    A->n_cand++;
    double tlo = tt->t - tt->et;
    if (tt->status == ST_PASS) {
        if (tlo < A->pass_lo1) { A->pass_lo2 = A->pass_lo1; A->pass_lo1 = tlo; A->pass_id1 = tri; }
        else if (tlo < A->pass_lo2) A->pass_lo2 = tlo;
    } else if (tt->status == ST_UNC) {
        if (tlo < A->unc_lo) A->unc_lo = tlo;
    }
    if (tt->exact_hit) {
        if (!A->have_best || tt->t < A->best_t || (tt->t == A->best_t && tri < A->best_id)) {
            A->have_best = 1; A->best_id = tri; A->best_t = tt->t; A->best = *tt;
            A->best_thi = tt->t + tt->et; A->best_status = tt->status;
        }
    }
}

static void closest_finish(const closest_acc* A, hit_rec* out)
{
    out->n_candidates = A->n_cand;
    if (!A->have_best) {
        out->id = NO_HIT; out->t = INFINITY; out->u = out->v = 0;
        out->et = out->eu = out->ev = 0;
        out->band = (A->unc_lo < INFINITY) || (A->pass_lo1 < INFINITY);
        return;
    }
    out->id = A->best_id; out->t = A->best.t; out->u = A->best.u; out->v = A->best.v;
    out->et = A->best.et; out->eu = A->best.eu; out->ev = A->best.ev;
    /* the answer is certain when the best hit is a certain FP32 hit, no uncertain triangle could
     * come before it, and no other certain hit overlaps its FP32 t interval */
    double other_pass = (A->pass_id1 == A->best_id) ? A->pass_lo2 : A->pass_lo1;
    out->band = (A->best_status != ST_PASS) || (A->unc_lo <= A->best_thi) || (other_pass <= A->best_thi);
}

static void acc_init(closest_acc* A)
{
    memset(A, 0, sizeof(*A));
    A->pass_lo1 = A->pass_lo2 = A->unc_lo = INFINITY;
    A->pass_id1 = NO_HIT;
}

static void closest_bvh_acc(const or_bvh* B, const ray_ev* r, double tmin, double tmax, double c, closest_acc* Ap)
{
    closest_acc A = *Ap;
    if (B->n_nodes > 0) {
        int32_t stack[256];
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            const bnode* n = &B->nodes[stack[--sp]];
            double te = box_enter(n, r, tmin - B->margin, tmax);
            if (te == INFINITY) continue;
            /* no triangle entering after the current best (plus padding) can change the answer
             * or the band, except grazing triangles whose FP32 t error exceeds the padding */
            if (A.have_best && te > A.best_thi + B->margin) continue;
            if (n->left < 0) {
                for (int32_t i = 0; i < n->count; ++i) {
                    uint32_t tri = B->tris[n->first + i];
                    tri_test tt;
                    tri_check(B->scene, tri, r, tmin, tmax, c, &tt);
                    closest_consider(&A, tri, &tt);
                }
            } else {
                stack[sp++] = n->right;
                stack[sp++] = n->left;
            }
        }
    }
    *Ap = A;
}

static void closest_bvh(const or_bvh* B, const ray_ev* r, double tmin, double tmax, double c, hit_rec* out)
{
    closest_acc A;
    acc_init(&A);
    closest_bvh_acc(B, r, tmin, tmax, c, &A);
    closest_finish(&A, out);
}

static void closest_brute(const or_scene* s, const ray_ev* r, double tmin, double tmax, double c, hit_rec* out)
{
    closest_acc A;
    acc_init(&A);
    for (int64_t t = 0; t < s->nt; ++t) {
        tri_test tt;
        tri_check(s, (uint32_t)t, r, tmin, tmax, c, &tt);
        closest_consider(&A, (uint32_t)t, &tt);
    }
    closest_finish(&A, out);
}

/* any hit: returns occluded (exact); *band set when no certain occluder exists but an uncertain one does */
static int any_bvh(const or_scene* s, const or_bvh* B, const ray_ev* r, double tmin, double tmax, double c, int* band, uint32_t* who)
{
    int occluded = 0, unc = 0;
    *who = NO_HIT;
    if (B == NULL) {
        for (int64_t t = 0; t < s->nt; ++t) {
            tri_test tt;
            tri_check(s, (uint32_t)t, r, tmin, tmax, c, &tt);
            if (tt.exact_hit) { occluded = 1; if (*who == NO_HIT) *who = (uint32_t)t; }
            if (tt.status == ST_PASS) { *band = 0; return 1; }
            if (tt.status == ST_UNC) unc = 1;
        }
        *band = unc;
        return occluded;
    }
    if (B->n_nodes == 0) { *band = 0; return 0; }
    int32_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const bnode* n = &B->nodes[stack[--sp]];
        if (box_enter(n, r, tmin - B->margin, tmax + B->margin) == INFINITY) continue;
        if (n->left < 0) {
            for (int32_t i = 0; i < n->count; ++i) {
                uint32_t tri = B->tris[n->first + i];
                tri_test tt;
                tri_check(s, tri, r, tmin, tmax, c, &tt);
                if (tt.exact_hit) { occluded = 1; if (*who == NO_HIT) *who = tri; }
                if (tt.status == ST_PASS) { *band = 0; *who = tri; return 1; }
                if (tt.status == ST_UNC) unc = 1;
            }
        } else {
            stack[sp++] = n->right;
            stack[sp++] = n->left;
        }
    }
    *band = unc;
    return occluded;
}

/* ------------------------------------------------------------------------- */
/* Two-level scenes (Sec. IV-B, "Ray-traced shadows": one acceleration       */
/* structure per mesh, instanced with a transform under a top level).        */
/* Instance i holds the contiguous triangles first_i .. first_i + count_i - 1 */
/* of the rest-frame scene and a world-to-object map x' = M x + m (FP32).    */
/* A world ray is mapped into each instance as o' = M o + m, d' = M d (the   */
/* FP32 side evaluates every component as ((M0 a0 + M1 a1) + M2 a2) [+ m])   */
/* and tested there; t is the parameter along the mapped ray.  The answer is */
/* the closest (resp. any) hit over all instances, ties to the smaller id.   */
/* ------------------------------------------------------------------------- */
typedef struct or_inst {
    const or_scene* rest;
    int64_t n;
    uint32_t* range;     /* first, count per instance */
    float* w2o;          /* 12 per instance, row-major [M | m] */
    bnode* wbox;         /* padded world box of each instance (only lo/hi used) */
    or_bvh** bvh;        /* per-instance BVH over its rest triangles */
    double margin;
} or_inst;

/* x' = M x + m in FP32 for the rigid map x = R x' + t given as [R | t]: M = R^T, m = -(R^T t), each
 * component of R^T t evaluated as ((R0k t0 + R1k t1) + R2k t2) */
OR_API void or_w2o_f32(const float* o2w, int64_t n, float* w2o)
{
    for (int64_t i = 0; i < n; ++i) {
        const float* X = o2w + 12 * i;
        float* W = w2o + 12 * i;
        for (int k = 0; k < 3; ++k) {
            for (int j = 0; j < 3; ++j) W[4 * k + j] = X[4 * j + k];
            float a = X[k] * X[3];
            float b = X[4 + k] * X[7];
            float c = X[8 + k] * X[11];
            W[4 * k + 3] = -((a + b) + c);
        }
    }
}

static ev3 xform_pt(const float* W, ev3 p, int affine)
{
    ev3 r;
    ev* out[3] = {&r.x, &r.y, &r.z};
    for (int k = 0; k < 3; ++k) {
        ev3 row = {{W[4 * k], 0.0}, {W[4 * k + 1], 0.0}, {W[4 * k + 2], 0.0}};
        ev v = ev3_dot(row, p);
        if (affine) v = ev_add(v, ev_x(W[4 * k + 3], 0.0));
        *out[k] = v;
    }
    return r;
}

static ray_ev xform_ray(const float* W, const ray_ev* r)
{
    ray_ev q;
    q.eo = xform_pt(W, r->eo, 1);
    q.ed = xform_pt(W, r->ed, 0);
    /* the values are the FP64 images of the world ray's values */
    ev3 o = xform_pt(W, ev3_exact(r->o), 1), d = xform_pt(W, ev3_exact(r->d), 0);
    q.o = mk(o.x.v, o.y.v, o.z.v);
    q.d = mk(d.x.v, d.y.v, d.z.v);
    return q;
}

/* world box: the corners of the instance's rest box mapped by the exact inverse of x' = M x + m */
static void inst_world_box(const float* W, const double lo[3], const double hi[3], double margin, bnode* out)
{
    double M[3][3], Mi[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[a][b] = W[4 * a + b];
    double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                 M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    Mi[0][0] = (M[1][1] * M[2][2] - M[1][2] * M[2][1]) / det;
    Mi[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / det;
    Mi[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) / det;
    Mi[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) / det;
    Mi[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / det;
    Mi[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / det;
    Mi[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) / det;
    Mi[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / det;
    Mi[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / det;
    for (int k = 0; k < 3; ++k) { out->lo[k] = INFINITY; out->hi[k] = -INFINITY; }
    for (int corner = 0; corner < 8; ++corner) {
        double x[3];
        for (int k = 0; k < 3; ++k) x[k] = ((corner >> k) & 1 ? hi[k] : lo[k]) - W[4 * k + 3];
        for (int a = 0; a < 3; ++a) {
            double p = Mi[a][0] * x[0] + Mi[a][1] * x[1] + Mi[a][2] * x[2];
            out->lo[a] = fmin(out->lo[a], p);
            out->hi[a] = fmax(out->hi[a], p);
        }
    }
    for (int k = 0; k < 3; ++k) { out->lo[k] -= margin; out->hi[k] += margin; }
    out->left = out->right = -1;
    out->first = out->count = 0;
}

OR_API or_inst* or_inst_create(const or_scene* rest, int64_t n, const uint32_t* range, const float* w2o, int use_bvh)
{
    or_inst* I = (or_inst*)calloc(1, sizeof(or_inst));
    I->rest = rest;
    I->n = n;
    I->range = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * 2 * sizeof(uint32_t));
    I->w2o = (float*)malloc((size_t)(n > 0 ? n : 1) * 12 * sizeof(float));
    I->wbox = (bnode*)malloc((size_t)(n > 0 ? n : 1) * sizeof(bnode));
    I->bvh = (or_bvh**)calloc((size_t)(n > 0 ? n : 1), sizeof(or_bvh*));
    memcpy(I->range, range, (size_t)n * 2 * sizeof(uint32_t));
    memcpy(I->w2o, w2o, (size_t)n * 12 * sizeof(float));
    double scale = scene_scale(rest);
    I->margin = 1e-4 * scale;
    for (int64_t i = 0; i < n; ++i) {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (uint32_t t = range[2 * i]; t < range[2 * i] + range[2 * i + 1]; ++t) {
            double tl[3], th[3];
            tri_bounds(rest, t, tl, th);
            for (int k = 0; k < 3; ++k) { lo[k] = fmin(lo[k], tl[k]); hi[k] = fmax(hi[k], th[k]); }
        }
        inst_world_box(I->w2o + 12 * i, lo, hi, I->margin, &I->wbox[i]);
        if (use_bvh) I->bvh[i] = bvh_build_range(rest, range[2 * i], range[2 * i + 1], scale);
    }
    return I;
}

OR_API void or_inst_free(or_inst* I)
{
    if (!I) return;
    for (int64_t i = 0; i < I->n; ++i) or_bvh_free(I->bvh[i]);
    free(I->bvh); free(I->wbox); free(I->w2o); free(I->range); free(I);
}

static void closest_inst(const or_inst* I, int use_bvh, const ray_ev* r, double tmin, double tmax, double c,
                         hit_rec* out)
{
    closest_acc A;
    acc_init(&A);
    for (int64_t i = 0; i < I->n; ++i) {
        double te = box_enter(&I->wbox[i], r, tmin - I->margin, tmax);
        if (te == INFINITY) continue;
        if (A.have_best && te > A.best_thi + I->margin) continue;
        ray_ev q = xform_ray(I->w2o + 12 * i, r);
        if (use_bvh && I->bvh[i]) {
            closest_bvh_acc(I->bvh[i], &q, tmin, tmax, c, &A);
        } else {
            for (uint32_t t = I->range[2 * i]; t < I->range[2 * i] + I->range[2 * i + 1]; ++t) {
                tri_test tt;
                tri_check(I->rest, t, &q, tmin, tmax, c, &tt);
                closest_consider(&A, t, &tt);
            }
        }
    }
    closest_finish(&A, out);
}

static int any_inst(const or_inst* I, int use_bvh, const ray_ev* r, double tmin, double tmax, double c, int* band)
{
    int occluded = 0, unc = 0;
    for (int64_t i = 0; i < I->n; ++i) {
        if (box_enter(&I->wbox[i], r, tmin - I->margin, tmax + I->margin) == INFINITY) continue;
        ray_ev q = xform_ray(I->w2o + 12 * i, r);
        int b = 0, occ = 0;
        uint32_t who;
        if (use_bvh && I->bvh[i]) {
            occ = any_bvh(I->rest, I->bvh[i], &q, tmin, tmax, c, &b, &who);
        } else {
            for (uint32_t t = I->range[2 * i]; t < I->range[2 * i] + I->range[2 * i + 1]; ++t) {
                tri_test tt;
                tri_check(I->rest, t, &q, tmin, tmax, c, &tt);
                if (tt.exact_hit) occ = 1;
                if (tt.status == ST_PASS) { occ = 1; b = 0; break; }
                if (tt.status == ST_UNC) b = 1;
            }
        }
        if (occ && !b) { *band = 0; return 1; }   /* a certain occluder */
        occluded |= occ;
        unc |= b;
    }
    *band = unc;
    return occluded;
}

/* Hit queries of a scene: through its instances when it has them, else over its own triangles with the
 * BVH B (NULL = brute force; for instanced scenes B only selects per-instance BVHs vs brute force). */
static void closest_q(const or_scene* s, const void* B, const ray_ev* r, double tmin, double tmax, double c,
                      hit_rec* out)
{
    if (s->inst) closest_inst(s->inst, B != NULL, r, tmin, tmax, c, out);
    else if (B) closest_bvh((const or_bvh*)B, r, tmin, tmax, c, out);
    else closest_brute(s, r, tmin, tmax, c, out);
}

static int any_q(const or_scene* s, const void* B, const ray_ev* r, double tmin, double tmax, double c, int* band)
{
    uint32_t who;
    if (s->inst) return any_inst(s->inst, B != NULL, r, tmin, tmax, c, band);
    return any_bvh(s, (const or_bvh*)B, r, tmin, tmax, c, band, &who);
}

static ray_ev exact_ray(v3 o, v3 d)
{
    ray_ev r;
    r.o = o; r.d = d; r.eo = ev3_exact(o); r.ed = ev3_exact(d);
    return r;
}

/* Single-ray queries with FP32-exact inputs (e.g. camera rays); bvh may be NULL (brute force). */
OR_API void or_closest(const or_scene* s, const or_bvh* B, const float o[3], const float d[3],
                       double tmin, double tmax, double c, uint32_t* id, double tuv[3], double err[3],
                       int* band, int64_t* n_cand)
{
    ray_ev r = exact_ray(from_f(o), from_f(d));
    hit_rec h;
    closest_q(s, B, &r, tmin, tmax, c, &h);
    *id = h.id; tuv[0] = h.t; tuv[1] = h.u; tuv[2] = h.v;
    err[0] = h.et; err[1] = h.eu; err[2] = h.ev;
    *band = h.band;
    if (n_cand) *n_cand = h.n_candidates;
}

/* Segment query in FP64: occluded iff some triangle is hit at tmin < t < tmax. */
OR_API int or_any(const or_scene* s, const or_bvh* B, const double o[3], const double d[3],
                  double tmin, double tmax, double c, int* band)
{
    v3 O = mk(o[0], o[1], o[2]), D = mk(d[0], d[1], d[2]);
    ray_ev r;
    r.o = O; r.d = D; r.eo = ev3_rounded(O); r.ed = ev3_rounded(D);
    return any_q(s, B, &r, tmin, tmax, c, band);
}

/* ------------------------------------------------------------------------- */
/* Cook-Torrance / GGX BRDF (Sec. IV-B equation) + Lambert diffuse.           */
/* alpha = roughness^2; k = (roughness+1)^2 / 8; F0 = mix(0.04, albedo, m).   */
/* ------------------------------------------------------------------------- */
static const double PI = 3.14159265358979323846;

/* Trowbridge-Reitz GGX normal distribution; the denominator is written as
 * a2 (n.h)^2 + |n x h|^2, equal to 1 + (a2 - 1)(n.h)^2 for unit n and h. */
static double ggx_D(v3 n, v3 h, double alpha)
{
    double a2 = alpha * alpha, ndh = dot(n, h);
    v3 nxh = cross(n, h);
    double den = a2 * ndh * ndh + dot(nxh, nxh);
    return a2 / (PI * den * den);
}

/* Schlick-GGX masking for one direction: x / (x (1 - k) + k) */
static double schlick_g1(double x, double k) { return x / (x * (1.0 - k) + k); }

/* Schlick Fresnel: F0 + (1 - F0) (1 - cos)^5 */
static double schlick_f(double f0, double cos_hv) { return f0 + (1.0 - f0) * pow(1.0 - cos_hv, 5.0); }

OR_API double or_ggx_D(const double n_[3], const double h_[3], double alpha)
{
    return ggx_D(mk(n_[0], n_[1], n_[2]), mk(h_[0], h_[1], h_[2]), alpha);
}
OR_API double or_schlick_g1(double x, double k) { return schlick_g1(x, k); }
OR_API double or_schlick_f(double f0, double c) { return schlick_f(f0, c); }

/* f = (1 - F)(1 - m) albedo / pi + D F G1(n.wo) G1(n.wi) / (4 (n.wo)(n.wi)), zero unless both cosines > 0 */
OR_API void or_brdf_k(const double n_[3], const double wo_[3], const double wi_[3], const double albedo[3],
                      double rough, double metal, double kgeo, double out[3])
{
    v3 n = mk(n_[0], n_[1], n_[2]), wo = mk(wo_[0], wo_[1], wo_[2]), wi = mk(wi_[0], wi_[1], wi_[2]);
    double ndo = dot(n, wo), ndi = dot(n, wi);
    out[0] = out[1] = out[2] = 0.0;
    if (!(ndo > 0.0) || !(ndi > 0.0)) return;
    v3 h = nrm(add(wo, wi));
    double D = ggx_D(n, h, rough * rough);
    double G = schlick_g1(ndo, kgeo) * schlick_g1(ndi, kgeo);
    double hdo = dot(h, wo);
    for (int ch = 0; ch < 3; ++ch) {
        double f0 = 0.04 * (1.0 - metal) + albedo[ch] * metal;
        double F = schlick_f(f0, hdo);
        double spec = D * F * G / (4.0 * ndo * ndi);
        double diff = (1.0 - F) * (1.0 - metal) * albedo[ch] / PI;
        out[ch] = diff + spec;
    }
}

OR_API void or_brdf(const double n[3], const double wo[3], const double wi[3], const double albedo[3],
                    double rough, double metal, double out[3])
{
    double k = (rough + 1.0) * (rough + 1.0) / 8.0;
    or_brdf_k(n, wo, wi, albedo, rough, metal, k, out);
}

static void brdf_v(v3 n, v3 wo, v3 wi, const float* mat, double out[3])
{
    double nn[3] = {n.x, n.y, n.z}, o[3] = {wo.x, wo.y, wo.z}, i[3] = {wi.x, wi.y, wi.z};
    double alb[3] = {mat[0], mat[1], mat[2]};
    or_brdf(nn, o, i, alb, (double)mat[3], (double)mat[4], out);
}

/* ------------------------------------------------------------------------- */
/* Surface point of a primary hit (FP64): barycentric point, two-sided       */
/* geometric normal facing the viewer, shadow-ray origin offset, and the     */
/* shading normal: with vertex normals their barycentric interpolation,      */
/* normalised and turned to the geometric normal's side; else the geometric  */
/* normal.  Shading uses ns; the shadow origin and cast test use n.           */
/* ------------------------------------------------------------------------- */
typedef struct { v3 p, n, wo, os, ns; } surface;

static void make_surface(const or_scene* s, uint32_t tri, double u, double v, v3 dir, surface* S)
{
    v3 a, b, c;
    tri_verts(s, tri, &a, &b, &c);
    S->p = add(add(scl(a, 1.0 - u - v), scl(b, u)), scl(c, v));
    v3 ng = nrm(cross(sub(b, a), sub(c, a)));
    if (dot(ng, dir) > 0.0) ng = scl(ng, -1.0);
    S->n = ng;
    S->wo = nrm(scl(dir, -1.0));
    double off = ldexp(fmax(1.0, amax(S->p)), -18);
    S->os = add(S->p, scl(S->n, off));
    S->ns = ng;
    if (s->nrm) {
        const uint32_t* ix = s->idx + 3 * (int64_t)tri;
        v3 na = from_f(s->nrm + 3 * (int64_t)ix[0]), nb = from_f(s->nrm + 3 * (int64_t)ix[1]);
        v3 nc = from_f(s->nrm + 3 * (int64_t)ix[2]);
        v3 ns = nrm(add(add(scl(na, 1.0 - u - v), scl(nb, u)), scl(nc, v)));
        if (dot(ns, ng) < 0.0) ns = scl(ns, -1.0);
        S->ns = ns;
    }
}

/* Shadow segment from the surface origin to a target point; the FP32 side holds the origin
 * rounded to FP32 and the direction as fl(target - fl(origin)), target error et per component. */
static int shadow_test(const or_scene* s, const or_bvh* B, const surface* S, v3 target, double target_err,
                       double c, int* cast, int* band)
{
    v3 d = sub(target, S->os);
    ray_ev r;
    r.o = S->os; r.d = d;
    r.eo = ev3_rounded(S->os);
    ev3 T = {{target.x, target_err}, {target.y, target_err}, {target.z, target_err}};
    r.ed = ev3_sub(T, r.eo);
    /* cast iff n . d > 0 (light on the front side); FP32 evaluates it from rounded n and d */
    ev3 N = ev3_rounded(S->n);
    ev nd = ev3_dot(N, r.ed);
    *band = 0;
    *cast = nd.v > 0.0;
    if (fabs(nd.v) <= c * nd.e) *band = 1;
    if (!*cast) return 0;
    int b2 = 0;
    int occ = any_q(s, B, &r, 0.0, 1.0, c, &b2);
    if (b2) *band = 1;
    return occ;
}

/* ------------------------------------------------------------------------- */
/* Point-light render of a list of samples.                                   */
/* ------------------------------------------------------------------------- */
OR_API void or_render_point(const or_scene* s, const or_bvh* B, const or_camera* cam,
                            const float* lights, int n_lights, double c,
                            const int64_t* samples, int64_t n,
                            uint32_t* hit_id, double* tuv, double* tuv_err, uint8_t* band_primary,
                            uint32_t* mask, uint32_t* band_shadow, double* rgb, uint32_t* cast_mask)
{
    cam_basis cb;
    camera_basis(cam, &cb);
    for (int64_t q = 0; q < n; ++q) {
        float of[3], df[3];
        gen_ray(cam, &cb, samples[q], of, df);
        ray_ev r = exact_ray(from_f(of), from_f(df));
        hit_rec h;
        closest_q(s, B, &r, 0.0, INFINITY, c, &h);
        hit_id[q] = h.id;
        tuv[3 * q + 0] = h.t; tuv[3 * q + 1] = h.u; tuv[3 * q + 2] = h.v;
        tuv_err[3 * q + 0] = h.et; tuv_err[3 * q + 1] = h.eu; tuv_err[3 * q + 2] = h.ev;
        band_primary[q] = (uint8_t)h.band;
        mask[q] = 0; band_shadow[q] = 0; cast_mask[q] = 0;
        rgb[3 * q + 0] = rgb[3 * q + 1] = rgb[3 * q + 2] = 0.0;
        if (h.id == NO_HIT) continue;
        surface S;
        make_surface(s, h.id, h.u, h.v, r.d, &S);
        const float* mat = s->mats + 5 * (int64_t)s->tri_mat[h.id];
        for (int l = 0; l < n_lights; ++l) {
            const float* L = lights + 6 * l;
            v3 lp = from_f(L);
            int cast, band;
            int occ = shadow_test(s, B, &S, lp, 0.0, c, &cast, &band);
            if (band) band_shadow[q] |= 1u << l;
            if (cast) cast_mask[q] |= 1u << l;
            if (!cast || occ) continue;
            mask[q] |= 1u << l;
            v3 tl = sub(lp, S.p);
            double d2 = dot(tl, tl);
            v3 wi = nrm(tl);
            double f[3];
            brdf_v(S.ns, S.wo, wi, mat, f);
            double cosi = fmax(dot(S.ns, wi), 0.0);
            for (int ch = 0; ch < 3; ++ch) rgb[3 * q + ch] += f[ch] * (double)L[3 + ch] * cosi / d2;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Rectangular area light: visibility estimate and unshadowed radiance.      */
/* rect = centre[3], edge_u[3], edge_v[3], radiance[3].  Light samples        */
/* y_k = c + (xi1 - 1/2) e_u + (xi2 - 1/2) e_v, xi from Philox with counter  */
/* (pixel, k, 1 + stream, 0).  V = mean over k of [n.d > 0, light faces the  */
/* point, segment unoccluded].  Radiance = unshadowed centre-point radiance  */
/* (L_e A cos_L at the centre) times V.                                       */
/* ------------------------------------------------------------------------- */
typedef struct { v3 C, EU, EV, nL; double area, terr; } rect_geo;

static void rect_setup(const float* rect, rect_geo* R)
{
    R->C = from_f(rect); R->EU = from_f(rect + 3); R->EV = from_f(rect + 6);
    v3 nl_raw = cross(R->EU, R->EV);
    R->area = len(nl_raw);
    R->nL = nrm(nl_raw);
    R->terr = 3.0 * U32R * (amax(R->C) + 0.5 * amax(R->EU) + 0.5 * amax(R->EV));
}

/* N light samples at one surface point; returns the visible count, adds band samples to *band_count */
static int rect_visibility(const or_scene* s, const or_bvh* B, const surface* S, const rect_geo* R,
                           uint32_t pixel, int N, uint32_t stream, uint32_t seed, uint32_t frame, double c,
                           int* band_count, int* cast_count)
{
    int vis = 0;
    for (int k = 0; k < N; ++k) {
        uint32_t ctr[4] = {pixel, (uint32_t)k, 1u + stream, 0u}, key[2] = {seed, frame}, rr[4];
        or_philox4x32_10(ctr, key, rr);
        v3 y = add(add(R->C, scl(R->EU, unit24(rr[0]) - 0.5)), scl(R->EV, unit24(rr[1]) - 0.5));
        int cast, band;
        int occ = shadow_test(s, B, S, y, R->terr, c, &cast, &band);
        /* the light emits on the side its normal e_u x e_v points to */
        v3 d = sub(y, S->os);
        double ed = 4.0 * U32R * amax(d);
        ev3 D = {{d.x, ed}, {d.y, ed}, {d.z, ed}};
        ev facing = ev3_dot(ev3_rounded(R->nL), D);
        int faces = facing.v < 0.0;
        if (fabs(facing.v) <= c * facing.e) band = 1;
        if (band) (*band_count)++;
        if (cast && cast_count) (*cast_count)++;
        if (cast && faces && !occ) vis++;
    }
    return vis;
}

/* Visibility of the rect light from an explicit surface point p with unit normal n
 * (shadow origin offset as for camera hits); Philox counter (pixel, k, 1 + stream, 0). */
OR_API int or_rect_vis_point(const or_scene* s, const or_bvh* B, const double p[3], const double n[3],
                             const float* rect, int N, uint32_t stream, uint32_t pixel, uint32_t seed,
                             uint32_t frame, double c, int* band_count)
{
    surface S;
    S.p = mk(p[0], p[1], p[2]);
    S.n = nrm(mk(n[0], n[1], n[2]));
    S.wo = S.n;
    S.ns = S.n;
    double off = ldexp(fmax(1.0, amax(S.p)), -18);
    S.os = add(S.p, scl(S.n, off));
    rect_geo R;
    rect_setup(rect, &R);
    *band_count = 0;
    return rect_visibility(s, B, &S, &R, pixel, N, stream, seed, frame, c, band_count, NULL);
}

OR_API void or_render_rect(const or_scene* s, const or_bvh* B, const or_camera* cam,
                           const float* rect, int n_light_samples, uint32_t stream, double c,
                           const int64_t* pixels, int64_t n,
                           uint32_t* hit_id, uint8_t* band_primary,
                           int32_t* vis_count, int32_t* band_count, int32_t* cast_count, double* rgb_unshadowed)
{
    cam_basis cb;
    camera_basis(cam, &cb);
    rect_geo R;
    rect_setup(rect, &R);
    for (int64_t q = 0; q < n; ++q) {
        int64_t pix = pixels[q];
        float of[3], df[3];
        gen_ray(cam, &cb, pix, of, df);   /* 1 sample per pixel */
        ray_ev r = exact_ray(from_f(of), from_f(df));
        hit_rec h;
        closest_q(s, B, &r, 0.0, INFINITY, c, &h);
        hit_id[q] = h.id;
        band_primary[q] = (uint8_t)h.band;
        vis_count[q] = 0; band_count[q] = 0; cast_count[q] = 0;
        rgb_unshadowed[3 * q] = rgb_unshadowed[3 * q + 1] = rgb_unshadowed[3 * q + 2] = 0.0;
        if (h.id == NO_HIT) continue;
        surface S;
        make_surface(s, h.id, h.u, h.v, r.d, &S);
        int bc = 0, cc = 0;
        vis_count[q] = rect_visibility(s, B, &S, &R, (uint32_t)pix, n_light_samples, stream,
                                       cam->seed, cam->frame, c, &bc, &cc);
        band_count[q] = bc;
        cast_count[q] = cc;
        /* unshadowed centre-point radiance: the light seen as a point source of intensity L_e A cos_L */
        const float* mat = s->mats + 5 * (int64_t)s->tri_mat[h.id];
        v3 tl = sub(R.C, S.p);
        double d2 = dot(tl, tl);
        v3 wi = nrm(tl);
        double cosl = fmax(-dot(R.nL, wi), 0.0);
        double cosi = fmax(dot(S.ns, wi), 0.0);
        double f[3];
        brdf_v(S.ns, S.wo, wi, mat, f);
        for (int ch = 0; ch < 3; ++ch)
            rgb_unshadowed[3 * q + ch] = f[ch] * (double)rect[9 + ch] * R.area * cosl * cosi / d2;
    }
}

/* ------------------------------------------------------------------------- */
/* Instrumented any-hit traversal of a 4-wide BVH given in the library's      */
/* exported layout (per node 32 words: lo_x[4] hi_x[4] lo_y[4] hi_y[4]        */
/* lo_z[4] hi_z[4] child[4] meta[4]; child word: 0xFFFFFFFF empty, bit 31 =   */
/* leaf with count - 1 in bits 28..30 and first slot in bits 0..27, else an   */
/* internal node; `order` maps a leaf slot to the original triangle id).      */
/* The work a ray's own traversal does (Sec. IV-B: an acceleration structure  */
/* answers a ray query by visiting few nodes): from the root, visit a node =  */
/* test its four child boxes against the segment 0 <= t <= 1; continue with  */
/* the nearest entered child and stack the others (farthest first); at a leaf */
/* test its triangles in slot order and stop at the first crossing with       */
/* 0 < t < 1.  Everything in FP64.  Counts node visits and triangle tests.    */
/* ------------------------------------------------------------------------- */
static float word_f(uint32_t w) { float f; memcpy(&f, &w, 4); return f; }

static int count_any_bvh4(const or_scene* s, const uint32_t* nodes, const uint32_t* order, v3 o, v3 d,
                          int64_t* n_nodes, int64_t* n_tris)
{
    uint32_t stack[256];
    int sp = 0;
    uint32_t cur = 0;
    const double O[3] = {o.x, o.y, o.z}, D[3] = {d.x, d.y, d.z};
    for (;;) {
        if (cur == 0xFFFFFFFFu) {
            if (sp == 0) return 0;
            cur = stack[--sp];
            continue;
        }
        if (!(cur & 0x80000000u)) {
            const uint32_t* nd = nodes + 32 * (int64_t)cur;
            (*n_nodes)++;
            double tn[4];
            uint32_t cw[4];
            int nh = 0;
            for (int c = 0; c < 4; ++c) {
                uint32_t w = nd[24 + c];
                if (w == 0xFFFFFFFFu) continue;
                double t0 = 0.0, t1 = 1.0;
                int hit = 1;
                for (int a = 0; a < 3 && hit; ++a) {
                    double lo = word_f(nd[8 * a + c]), hi = word_f(nd[8 * a + 4 + c]);
                    if (D[a] == 0.0) {
                        if (O[a] < lo || O[a] > hi) hit = 0;
                        continue;
                    }
                    double ta = (lo - O[a]) / D[a], tb = (hi - O[a]) / D[a];
                    if (ta > tb) { double x = ta; ta = tb; tb = x; }
                    t0 = fmax(t0, ta);
                    t1 = fmin(t1, tb);
                    if (t0 > t1) hit = 0;
                }
                if (!hit) continue;
                /* insertion by entry distance, earlier slots first on ties */
                int k = nh++;
                while (k > 0 && tn[k - 1] > t0) { tn[k] = tn[k - 1]; cw[k] = cw[k - 1]; --k; }
                tn[k] = t0; cw[k] = w;
            }
            for (int k = nh - 1; k >= 1; --k) stack[sp++] = cw[k];
            cur = nh > 0 ? cw[0] : 0xFFFFFFFFu;
            continue;
        }
        uint32_t first = cur & 0x0FFFFFFFu, cnt = ((cur >> 28) & 7u) + 1u;
        for (uint32_t i = 0; i < cnt; ++i) {
            v3 a, b, c;
            tri_verts(s, order[first + i], &a, &b, &c);
            (*n_tris)++;
            v3 e1 = sub(b, a), e2 = sub(c, a), pv = cross(d, e2);
            double det = dot(e1, pv);
            if (det == 0.0) continue;
            v3 sv = sub(o, a), qv = cross(sv, e1);
            double u = dot(sv, pv) / det, v = dot(d, qv) / det, t = dot(e2, qv) / det;
            if (u >= 0.0 && v >= 0.0 && u + v <= 1.0 && t > 0.0 && t < 1.0) return 1;
        }
        cur = 0xFFFFFFFFu;
    }
}

/* Explicit segments o + t d, 0 < t < 1 (n x 3 doubles each): occluded flag per segment and, added to out[0] and
 * out[1], the node visits and triangle tests of the instrumented traversal. */
OR_API void or_count_any(const or_scene* s, const uint32_t* nodes, const uint32_t* order, const double* o,
                         const double* d, int64_t n, uint8_t* occluded, int64_t out[2])
{
    for (int64_t q = 0; q < n; ++q)
        occluded[q] = (uint8_t)count_any_bvh4(s, nodes, order, mk(o[3 * q], o[3 * q + 1], o[3 * q + 2]),
                                              mk(d[3 * q], d[3 * q + 1], d[3 * q + 2]), &out[0], &out[1]);
}

/* Rect-light shadow rays of the given pixels (1 camera sample each, as or_render_rect), traced through the
 * exported BVH by the instrumented traversal: adds to out[0] the rays cast (n . d > 0 and the light's
 * emitting side faces the point), out[1] node visits, out[2] triangle tests. */
OR_API void or_count_rect(const or_scene* s, const or_bvh* B, const uint32_t* nodes, const uint32_t* order,
                          const or_camera* cam, const float* rect, int n_light_samples, uint32_t stream,
                          const int64_t* pixels, int64_t n, int64_t out[3])
{
    cam_basis cb;
    camera_basis(cam, &cb);
    rect_geo R;
    rect_setup(rect, &R);
    for (int64_t q = 0; q < n; ++q) {
        int64_t pix = pixels[q];
        float of[3], df[3];
        gen_ray(cam, &cb, pix, of, df);
        ray_ev r = exact_ray(from_f(of), from_f(df));
        hit_rec h;
        closest_q(s, B, &r, 0.0, INFINITY, 4.0, &h);
        if (h.id == NO_HIT) continue;
        surface S;
        make_surface(s, h.id, h.u, h.v, r.d, &S);
        for (int k = 0; k < n_light_samples; ++k) {
            uint32_t ctr[4] = {(uint32_t)pix, (uint32_t)k, 1u + stream, 0u}, key[2] = {cam->seed, cam->frame}, rr[4];
            or_philox4x32_10(ctr, key, rr);
            v3 y = add(add(R.C, scl(R.EU, unit24(rr[0]) - 0.5)), scl(R.EV, unit24(rr[1]) - 0.5));
            v3 d = sub(y, S.os);
            if (!(dot(S.n, d) > 0.0) || !(dot(R.nL, d) < 0.0)) continue;
            out[0]++;
            count_any_bvh4(s, nodes, order, S.os, d, &out[1], &out[2]);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* FP32 mirrors: supersampling resolve and rigid vertex transforms.          */
/* ------------------------------------------------------------------------- */
/* out[p] = ((s0 + s1) + (s2 + s3)) * 0.25 per channel; n_per = 4; or copy when n_per = 1 */
OR_API void or_resolve_f32(const float* samples, int64_t n_pixels, int n_per, float* out)
{
    for (int64_t p = 0; p < n_pixels; ++p) {
        for (int ch = 0; ch < 4; ++ch) {
            if (n_per == 1) { out[4 * p + ch] = samples[4 * p + ch]; continue; }
            const float* s = samples + (int64_t)16 * p + ch;
            float a = s[0] + s[4];
            float b = s[8] + s[12];
            out[4 * p + ch] = (a + b) * 0.25f;
        }
    }
}

/* rest (nv x 3) -> out for the vertex ranges of the given bodies:
 * x' = ((R00 x + R01 y) + R02 z) + t0, etc., with M = [R | t] row-major 3x4 */
OR_API void or_transform_f32(const float* rest, const uint32_t* body_vrange, const uint32_t* body_ids,
                             const float* xf, int64_t n_bodies, float* out)
{
    for (int64_t b = 0; b < n_bodies; ++b) {
        const float* M = xf + 12 * b;
        uint32_t first = body_vrange[2 * (int64_t)body_ids[b]], count = body_vrange[2 * (int64_t)body_ids[b] + 1];
        for (uint32_t i = first; i < first + count; ++i) {
            const float* p = rest + 3 * (int64_t)i;
            for (int r = 0; r < 3; ++r) {
                float a = M[4 * r + 0] * p[0];
                float bb = M[4 * r + 1] * p[1];
                float cc = M[4 * r + 2] * p[2];
                out[3 * (int64_t)i + r] = ((a + bb) + cc) + M[4 * r + 3];
            }
        }
    }
}

/* rest normals (nv x 3) -> out for the vertex ranges of the given bodies: n' = ((R00 x + R01 y) + R02 z), etc. */
OR_API void or_rotate_f32(const float* rest, const uint32_t* body_vrange, const uint32_t* body_ids,
                          const float* xf, int64_t n_bodies, float* out)
{
    for (int64_t b = 0; b < n_bodies; ++b) {
        const float* M = xf + 12 * b;
        uint32_t first = body_vrange[2 * (int64_t)body_ids[b]], count = body_vrange[2 * (int64_t)body_ids[b] + 1];
        for (uint32_t i = first; i < first + count; ++i) {
            const float* p = rest + 3 * (int64_t)i;
            for (int r = 0; r < 3; ++r) {
                float a = M[4 * r + 0] * p[0];
                float bb = M[4 * r + 1] * p[1];
                float cc = M[4 * r + 2] * p[2];
                out[3 * (int64_t)i + r] = (a + bb) + cc;
            }
        }
    }
}

/* Per-triangle classification of an FP32-exact ray: out = {exact_hit, status, t, u, v, et, eu, ev}. */
OR_API void or_tri_test(const or_scene* s, uint32_t tri, const float o[3], const float d[3],
                        double tmin, double tmax, double c, double out[8])
{
    ray_ev r = exact_ray(from_f(o), from_f(d));
    tri_test tt;
    tri_check(s, tri, &r, tmin, tmax, c, &tt);
    out[0] = tt.exact_hit; out[1] = tt.status; out[2] = tt.t; out[3] = tt.u; out[4] = tt.v;
    out[5] = tt.et; out[6] = tt.eu; out[7] = tt.ev;
}
