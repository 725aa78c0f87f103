// Display post pass of a rendered frame (the paper's main-pass tone mapping and gamma correction and its
// FXAA post-processing pass, Sec. IV-B): Reinhard tone map + sRGB8 encoding, then FXAA on the 8-bit image.
// The exact definition (integer luma, integer edge decisions, FP32 blend in a fixed order) is stated with
// rc_postprocess in include/raycast.h; both kernels are HBM-bound image passes.
#include "rc_internal.h"

#include <mutex>

namespace {

constexpr int EDGE_MIN = 2048;   // minimum local luma range (luma scale 0..65280)
constexpr int EDGE_REL_SHIFT = 3;
constexpr int SEARCH = 12;

__device__ inline uint8_t srgb8(float r)
{
    const double v = (double)r;
    const double s = v <= 0.0031308 ? 12.92 * v : 1.055 * pow(fmax(v, 0.0), 1.0 / 2.4) - 0.055;
    return (uint8_t)fmin(fmax(floor(s * 255.0 + 0.5), 0.0), 255.0);
}

__global__ __launch_bounds__(256) void k_tonemap(const float4* rgba, uint32_t n, uchar4* out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 c = rgba[i];
    float v[3] = {fmaxf(c.x, 0.0f), fmaxf(c.y, 0.0f), fmaxf(c.z, 0.0f)};
    uint8_t q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) q[k] = srgb8(v[k] / (1.0f + v[k]));
    const double a = fmin(fmax((double)c.w, 0.0), 1.0);
    out[i] = make_uchar4(q[0], q[1], q[2], (uint8_t)floor(a * 255.0 + 0.5));
}

__device__ inline int luma_at(const uchar4* img, int W, int H, int x, int y)
{
    x = min(max(x, 0), W - 1);
    y = min(max(y, 0), H - 1);
    const uchar4 p = img[(size_t)y * W + x];
    return 77 * (int)p.x + 150 * (int)p.y + 29 * (int)p.z;
}

__global__ __launch_bounds__(256) void k_fxaa(const uchar4* in, int W, int H, uchar4* out)
{
    const int x = blockIdx.x * 16 + (threadIdx.x & 15), y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= W || y >= H) return;
    const uchar4 p = in[(size_t)y * W + x];
    const int Lc = luma_at(in, W, H, x, y);
    const int Ln = luma_at(in, W, H, x, y - 1), Ls = luma_at(in, W, H, x, y + 1);
    const int Lw = luma_at(in, W, H, x - 1, y), Le = luma_at(in, W, H, x + 1, y);
    const int lmax = max(max(max(Lc, Ln), max(Ls, Lw)), Le);
    const int lmin = min(min(min(Lc, Ln), min(Ls, Lw)), Le);
    const int rng = lmax - lmin;
    if (!(rng >= EDGE_MIN && (rng << EDGE_REL_SHIFT) >= lmax)) {
        out[(size_t)y * W + x] = p;
        return;
    }
    const int Lnw = luma_at(in, W, H, x - 1, y - 1), Lne = luma_at(in, W, H, x + 1, y - 1);
    const int Lsw = luma_at(in, W, H, x - 1, y + 1), Lse = luma_at(in, W, H, x + 1, y + 1);
    // second differences across rows (large at an edge running along x) and across columns
    const int d_rows = abs(Lnw - 2 * Lw + Lsw) + 2 * abs(Ln - 2 * Lc + Ls) + abs(Lne - 2 * Le + Lse);
    const int d_cols = abs(Lnw - 2 * Ln + Lne) + 2 * abs(Lw - 2 * Lc + Le) + abs(Lsw - 2 * Ls + Lse);
    const bool horiz = d_rows >= d_cols;
    const int L1 = horiz ? Ln : Lw, L2 = horiz ? Ls : Le;
    const int g1 = abs(L1 - Lc), g2 = abs(L2 - Lc);
    const bool first = g1 >= g2;
    const int grad = max(g1, g2);
    const int S2 = Lc + (first ? L1 : L2);    // twice the mean luma of the pair straddling the edge
    const int sx = horiz ? 0 : (first ? -1 : 1), sy = horiz ? (first ? -1 : 1) : 0;
    const int ax = horiz ? 1 : 0, ay = horiz ? 0 : 1;
    int dist[2] = {SEARCH + 1, SEARCH + 1}, mend[2] = {0, 0};
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int sgn = side == 0 ? 1 : -1;
        for (int i = 1; i <= SEARCH; ++i) {
            const int px = x + sgn * i * ax, py = y + sgn * i * ay;
            const int m = luma_at(in, W, H, px, py) + luma_at(in, W, H, px + sx, py + sy);
            if (2 * abs(m - S2) >= grad) {
                dist[side] = i;
                mend[side] = m;
                break;
            }
        }
    }
    const bool near_pos = dist[0] < dist[1];
    const int dmin = min(dist[0], dist[1]);
    const int me = near_pos ? mend[0] : mend[1];
    const bool found = (near_pos ? dist[0] : dist[1]) <= SEARCH;
    const bool blend_edge = found && ((me - S2 < 0) != (2 * Lc - S2 < 0));
    const float off_edge = blend_edge ? 0.5f - (float)dmin / (float)(dist[0] + dist[1]) : 0.0f;
    const int a12 = 2 * (Ln + Ls + Le + Lw) + (Lne + Lnw + Lse + Lsw);
    const float num = (float)abs(a12 - 12 * Lc), den = (float)max(12 * rng, 1);
    const float s1 = fminf(num / den, 1.0f);
    float t = -2.0f * s1;
    t = t + 3.0f;
    t = t * s1;
    t = t * s1;
    const float sub = (t * t) * 0.75f;
    const float w = fmaxf(off_edge, sub);
    const int qx = min(max(x + sx, 0), W - 1), qy = min(max(y + sy, 0), H - 1);
    const uchar4 q = in[(size_t)qy * W + qx];
    const float a[3] = {(float)p.x, (float)p.y, (float)p.z}, b[3] = {(float)q.x, (float)q.y, (float)q.z};
    uint8_t r[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float d = b[k] - a[k];
        const float wd = w * d;
        const float v = a[k] + wd;
        r[k] = (uint8_t)fminf(fmaxf(floorf(v + 0.5f), 0.0f), 255.0f);
    }
    out[(size_t)y * W + x] = make_uchar4(r[0], r[1], r[2], p.w);
}

}  // namespace

void rc_launch_postprocess(const float* rgba, uint32_t w, uint32_t h, bool fxaa, uint8_t* scratch, uint8_t* out,
                           hipStream_t st)
{
    const uint32_t n = w * h;
    uchar4* tm = reinterpret_cast<uchar4*>(fxaa ? scratch : out);
    hipLaunchKernelGGL(k_tonemap, dim3((n + 255) / 256), dim3(256), 0, st, reinterpret_cast<const float4*>(rgba), n,
                       tm);
    if (fxaa)
        hipLaunchKernelGGL(k_fxaa, dim3((w + 15) / 16, (h + 15) / 16), dim3(256), 0, st, tm, (int)w, (int)h,
                           reinterpret_cast<uchar4*>(out));
}

// Fixed scratch of rc_postprocess_noalloc: the tone-mapped 8-bit image that FXAA reads, for images of at most
// RC_POST_SCRATCH_PIXELS pixels (16 MiB).  Each GPU the library runs on holds its own copy until the
// process ends.  In host code this name is only a stand-in for the symbol: kernels receive the device address
// that rc_post_scratch_init obtained for the current device.
static __device__ __align__(256) uchar4 scratch[RC_POST_SCRATCH_PIXELS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
uint8_t* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t rc_post_scratch_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return hipSuccess;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    e = hipSetDevice(device);
    if (e != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess && ptr) g_scratch_ptr[device] = static_cast<uint8_t*>(ptr);
    else if (e == hipSuccess) e = hipErrorInvalidSymbol;
    hipError_t e2 = hipSetDevice(prev);
    return e != hipSuccess ? e : e2;
}

uint8_t* rc_post_scratch(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch_ptr[device];
}
