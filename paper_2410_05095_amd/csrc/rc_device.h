// Device helpers shared by the kernels: counter-based RNG, camera rays, the FP64 surface
// reconstruction of a hit, and the GGX BRDF.
#pragma once

#include "rc_internal.h"

// Philox4x32-10 (Salmon et al., SC'11): ten multiply/xor rounds with Weyl key bumps.
__device__ inline void rc_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                 uint32_t out[4])
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ inline float rc_unit24(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

// Camera ray of sample k of pixel `pixel`, in FP32 with the operation order fixed
// (the library is compiled without contraction; division and sqrt are correctly rounded).
__device__ inline void rc_camera_ray(const DevCamera& c, uint32_t pixel, uint32_t k, float o[3], float d[3])
{
    float ox = 0.5f, oy = 0.5f;
    if (c.ssaa > 1) {
        uint32_t r[4];
        rc_philox(pixel, k, 0u, 0u, c.seed, c.frame, r);
        ox = ((float)(k & 1u) + rc_unit24(r[0])) * 0.5f;
        oy = ((float)(k >> 1) + rc_unit24(r[1])) * 0.5f;
    }
    uint32_t i = pixel % (uint32_t)c.width, j = pixel / (uint32_t)c.width;
    float px = (2.0f * ((float)i + ox)) / (float)c.width;
    px = (px - 1.0f) * c.x_scale;
    float py = (2.0f * ((float)j + oy)) / (float)c.height;
    py = (1.0f - py) * c.tan_half;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float t0 = px * c.r[a];
        float t1 = py * c.u[a];
        d[a] = (t0 + t1) + c.f[a];
        o[a] = c.eye[a];
    }
    float n2 = d[0] * d[0] + d[1] * d[1];
    n2 = n2 + d[2] * d[2];
    float len = sqrtf(n2);
    d[0] = d[0] / len; d[1] = d[1] / len; d[2] = d[2] / len;
}

struct D3 { double x, y, z; };
__device__ inline D3 d3(double x, double y, double z) { D3 r = {x, y, z}; return r; }
__device__ inline D3 d3add(D3 a, D3 b) { return d3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ inline D3 d3sub(D3 a, D3 b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline D3 d3scl(D3 a, double s) { return d3(a.x * s, a.y * s, a.z * s); }
__device__ inline double d3dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline D3 d3cross(D3 a, D3 b)
{
    return d3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ inline D3 d3nrm(D3 a) { return d3scl(a, 1.0 / sqrt(d3dot(a, a))); }

struct Surface {
    D3 p;   // hit point
    D3 n;   // unit geometric normal facing the viewer
    D3 wo;  // unit direction towards the viewer
    D3 ns;  // unit shading normal: interpolated vertex normal on the viewer's side, or n
};

// FP64 reconstruction of a camera hit from the FP32 ray and the FP32 triangle: barycentric
// point of the Moller-Trumbore solution, two-sided geometric normal.
__device__ inline Surface rc_surface(const DevScene& sc, const DevCamera& cam, uint32_t pixel, uint32_t k,
                                     uint32_t tri)
{
    float of[3], df[3];
    rc_camera_ray(cam, pixel, k, of, df);
    const uint32_t* ix = sc.idx + 3 * (size_t)tri;
    const float* pa = sc.pos + 3 * (size_t)ix[0];
    const float* pb = sc.pos + 3 * (size_t)ix[1];
    const float* pc = sc.pos + 3 * (size_t)ix[2];
    D3 a = d3(pa[0], pa[1], pa[2]), b = d3(pb[0], pb[1], pb[2]), c = d3(pc[0], pc[1], pc[2]);
    D3 o = d3(of[0], of[1], of[2]), d = d3(df[0], df[1], df[2]);
    D3 e1 = d3sub(b, a), e2 = d3sub(c, a);
    D3 pv = d3cross(d, e2);
    double det = d3dot(e1, pv);
    D3 s = d3sub(o, a);
    double u = d3dot(s, pv) / det;
    D3 q = d3cross(s, e1);
    double v = d3dot(d, q) / det;
    Surface S;
    S.p = d3add(d3add(d3scl(a, 1.0 - u - v), d3scl(b, u)), d3scl(c, v));
    D3 ng = d3nrm(d3cross(e1, e2));
    if (d3dot(ng, d) > 0.0) ng = d3scl(ng, -1.0);
    S.n = ng;
    S.wo = d3nrm(d3scl(d, -1.0));
    S.ns = ng;
    if (sc.nrm) {
        const float* na = sc.nrm + 3 * (size_t)ix[0];
        const float* nb = sc.nrm + 3 * (size_t)ix[1];
        const float* nc = sc.nrm + 3 * (size_t)ix[2];
        D3 ns = d3add(d3add(d3scl(d3(na[0], na[1], na[2]), 1.0 - u - v), d3scl(d3(nb[0], nb[1], nb[2]), u)),
                      d3scl(d3(nc[0], nc[1], nc[2]), v));
        ns = d3nrm(ns);
        if (d3dot(ns, ng) < 0.0) ns = d3scl(ns, -1.0);
        S.ns = ns;
    }
    return S;
}

// Shadow-ray origin: offset along the normal by 2^-18 max(1, |p|_inf).
__device__ inline D3 rc_shadow_origin(const Surface& S)
{
    double m = fmax(fabs(S.p.x), fmax(fabs(S.p.y), fabs(S.p.z)));
    double off = ldexp(fmax(1.0, m), -18);
    return d3add(S.p, d3scl(S.n, off));
}

// Cook-Torrance (GGX D, Schlick F, Schlick-GGX G with k = (r+1)^2/8) plus Lambert diffuse,
// evaluated in FP64; mat = albedo rgb, roughness, metallic.  Zero unless n.wo > 0 and n.wi > 0.
__device__ inline void rc_brdf(D3 n, D3 wo, D3 wi, const float* mat, double f[3])
{
    f[0] = f[1] = f[2] = 0.0;
    double ndo = d3dot(n, wo), ndi = d3dot(n, wi);
    if (!(ndo > 0.0) || !(ndi > 0.0)) return;
    const double PI = 3.14159265358979323846;
    D3 h = d3nrm(d3add(wo, wi));
    double r = (double)mat[3], m = (double)mat[4];
    double alpha = r * r, a2 = alpha * alpha;
    double ndh = d3dot(n, h);
    D3 nxh = d3cross(n, h);
    double den = a2 * ndh * ndh + d3dot(nxh, nxh);
    double D = a2 / (PI * den * den);
    double k = (r + 1.0) * (r + 1.0) / 8.0;
    double G = (ndo / (ndo * (1.0 - k) + k)) * (ndi / (ndi * (1.0 - k) + k));
    double hdo = d3dot(h, wo);
    double x = 1.0 - hdo;
    double x2 = x * x;
    double fw = x2 * x2 * x;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        double alb = (double)mat[ch];
        double f0 = 0.04 * (1.0 - m) + alb * m;
        double F = f0 + (1.0 - f0) * fw;
        double spec = D * F * G / (4.0 * ndo * ndi);
        double diff = (1.0 - F) * (1.0 - m) * alb / PI;
        f[ch] = diff + spec;
    }
}

// Tiled sample order: 64 consecutive work items cover an 8x8 (1 spp) or 4x4-pixel (2x2 spp) tile.
__device__ inline bool rc_item_to_sample(const DevCamera& c, uint32_t item, uint32_t& pixel, uint32_t& k)
{
    uint32_t spp = (uint32_t)(c.ssaa * c.ssaa);
    uint32_t tw = spp == 1 ? 8u : 4u;
    uint32_t tiles_x = ((uint32_t)c.width + tw - 1) / tw;
    uint32_t tile = item >> 6, within = item & 63u;
    uint32_t pit = within / spp;
    k = within % spp;
    uint32_t i = (tile % tiles_x) * tw + pit % tw;
    uint32_t j = (tile / tiles_x) * tw + pit / tw;
    if (i >= (uint32_t)c.width || j >= (uint32_t)c.height) return false;
    pixel = j * (uint32_t)c.width + i;
    return true;
}

__host__ __device__ inline uint32_t rc_n_items(int width, int height, int ssaa)
{
    uint32_t spp = (uint32_t)(ssaa * ssaa);
    uint32_t tw = spp == 1 ? 8u : 4u;
    uint32_t tx = ((uint32_t)width + tw - 1) / tw, ty = ((uint32_t)height + tw - 1) / tw;
    return tx * ty * 64u;
}
