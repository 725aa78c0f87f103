// U-Net shadow-denoiser kernels for gfx950: BF16 storage, FP32 accumulation.
//
// 3x3 convolutions are implicit GEMMs on the matrix cores (v_mfma_f32_16x16x32_bf16):
//   forward      out[p][co] = sum_{tap,ci} in[p + off(tap)][ci] * W[co][tap][ci]     (M = pixels, N = Cout)
//   input grad   gin[p][ci] = sum_{tap,co} g[p - off(tap)][co] * W[co][tap][ci]      = the forward kernel
//                with the flipped, transposed weights Wf[ci][8 - tap][co]
//   weight grad  dW[co][tap][ci] = sum_p g[p][co] * in[p + off(tap)][ci]            (K = pixels, split over
//                chunks; the per-chunk partials are summed in chunk order, so the result is deterministic)
// Tensors are NHWC; every reduction (bias, head, loss) is a fixed-order two-stage sum.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "rc_unet.h"

#ifndef RC_CONV_ROWS
#define RC_CONV_ROWS 8   // output rows per wave of the row-blocked convolution
#endif
// minimum waves per SIMD the compiler keeps the convolution kernels to (their register budget)
#ifndef RC_OCC_E1A
#define RC_OCC_E1A 4
#endif
#ifndef RC_OCC_ROWS
#define RC_OCC_ROWS 2
#endif
#ifndef RC_OCC_416
#define RC_OCC_416 3
#endif
#ifndef RC_OCC_816
#define RC_OCC_816 2
#endif

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ inline uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline bf16x8 load8(const uint16_t* p) { return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p)); }

__device__ inline void unpack8(uint4 v, float f[8])
{
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        f[2 * e] = __uint_as_float(w[e] << 16);
        f[2 * e + 1] = __uint_as_float(w[e] & 0xFFFF0000u);
    }
}
__device__ inline uint4 pack8(const float f[8])
{
    uint32_t w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = (uint32_t)f2bf(f[2 * e]) | ((uint32_t)f2bf(f[2 * e + 1]) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// 2x2 average pool of four 8-channel groups: a = (2y, 2x), b = (2y, 2x + 1), c = (2y + 1, 2x),
// d = (2y + 1, 2x + 1), as ((a + b) + (c + d)) / 4 rounded to BF16
__device__ inline uint4 pool4(uint4 a, uint4 b, uint4 c, uint4 d)
{
    float fa[8], fb[8], fc[8], fd[8], r[8];
    unpack8(a, fa); unpack8(b, fb); unpack8(c, fc); unpack8(d, fd);
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = ((fa[e] + fb[e]) + (fc[e] + fd[e])) * 0.25f;
    return pack8(r);
}

// the 1x1 head on one pixel's 32 BF16 channels (FP32, channels in order, weights rounded to BF16), then the
// sigmoid
__device__ inline float head_value(const float f[32], const float* wh, const float* bh)
{
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 32; ++c) s = fmaf(f[c], bf2f(f2bf(wh[c])), s);
    s += bh[0];
    return 1.0f / (1.0f + expf(-s));
}

// ---------------------------------------------------------------- 3x3 convolution
// Each wave computes 32 pixels (two 16-row MFMA tiles) x 16*NT output channels; a block has 4 waves.
template <int NT>
__global__ __launch_bounds__(256) void k_conv3x3(ConvArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int P = a.N * a.H * a.W;
    const int p0 = (blockIdx.x * 4 + wave) * 32;
    if (p0 >= P) return;
    const int K = 9 * a.Cin;
    const int r = lane & 15, g = lane >> 4;
    int ny[2], yy[2], xx[2];
    bool pv[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        int p = p0 + 16 * mt + r;
        pv[mt] = p < P;
        int q = pv[mt] ? p : 0;
        xx[mt] = q % a.W;
        int t = q / a.W;
        yy[mt] = t % a.H;
        ny[mt] = t / a.H;
    }
    f32x4 acc[2][NT];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = {};
    for (int k0 = 0; k0 < K; k0 += 32) {
        const int kk = k0 + 8 * g;
        const bool kv = kk < K;
        const int tap = kv ? kk / a.Cin : 0;
        const int ci = kk - tap * a.Cin;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        bf16x8 A[2], B[NT];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            int y = yy[mt] + dy, x = xx[mt] + dx;
            bool ok = pv[mt] && kv && y >= 0 && y < a.H && x >= 0 && x < a.W;
            A[mt] = ok ? load8(a.in + ((size_t)(ny[mt] * a.H + y) * a.W + x) * a.Cin + ci) : zero;
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            int co = 16 * nt + r;
            B[nt] = (kv && co < a.Cout) ? load8(a.wt + (size_t)co * K + kk) : zero;
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], B[nt], acc[mt][nt], 0, 0, 0);
    }
    // D layout: lane holds column (channel) 16 nt + (lane & 15), rows (pixels) 4 (lane >> 4) + i
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            int co = 16 * nt + r;
            if (co >= a.Cout) continue;
            float b = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int p = p0 + 16 * mt + 4 * g + i;
                if (p >= P) continue;
                float v = acc[mt][nt][i] + b;
                if (a.relu) v = fmaxf(v, 0.0f);
                size_t o = (size_t)p * a.Cout + co;
                if (a.mask && !(bf2f(a.mask[o]) > 0.0f)) v = 0.0f;
                a.out[o] = f2bf(v);
            }
        }
}

// Tile of workgroup b among n: workgroups are dispatched to the 8 XCDs round-robin (b % 8), so XCD g is
// given the contiguous range of tiles [g q + min(g, r), ...) with q = n / 8, r = n % 8.  Tiles that share
// halo rows then run on the same XCD and meet in its L2.
__device__ inline int xcd_tile(int b, int n)
{
    const int g = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
    return g * q + min(g, r) + k;
}

// One 16-byte group of a convolution's input halo: pixel (y, x) of image n, channels [ci, ci + 8), zero
// outside the image.  The address is formed from the clamped position, so the load is always in bounds and
// needs no branch, and the value is replaced by zero afterwards; a tile's loads can then all be in flight at
// once.  With a second source, channels below Ca come from the 2x nearest-upsampled `in`, the rest from in2.
__device__ inline const uint16_t* group_ptr(const ConvArgs& a, int n, int y, int x, int ci)
{
    if (a.in2 == nullptr) return a.in + ((size_t)(n * a.H + y) * a.W + x) * a.Cin + ci;
    const bool up = ci < a.Ca;
    const size_t ou = ((size_t)(n * (a.H >> 1) + (y >> 1)) * (a.W >> 1) + (x >> 1)) * a.Ca + ci;
    const size_t os = ((size_t)(n * a.H + y) * a.W + x) * (a.Cin - a.Ca) + (ci - a.Ca);
    return (up ? a.in : a.in2) + (up ? ou : os);
}
__device__ inline uint4 halo_group(const ConvArgs& a, int n, int y, int x, int ci)
{
    const bool inb = (unsigned)y < (unsigned)a.H && (unsigned)x < (unsigned)a.W;
    const int yc = min(max(y, 0), a.H - 1), xc = min(max(x, 0), a.W - 1);
    const uint4 v = *reinterpret_cast<const uint4*>(group_ptr(a, n, yc, xc, ci));
    return inb ? v : make_uint4(0u, 0u, 0u, 0u);
}

// 16 zero bytes in device memory: the source of halo groups outside the image for loads that write LDS
// directly
__device__ __align__(16) const uint4 g_zero_group = {0u, 0u, 0u, 0u};

// ---------------------------------------------------------------- 3x3 convolution, LDS-tiled
// Workgroup of 4 waves; output tile = 4 rows x TW = 16 MT columns of one image, wave w computes row w:
// MT 16-pixel M-tiles x NT 16-channel N-tiles.  For each chunk of CC input channels the input halo (6 rows
// x TW + 2 columns) is staged in LDS, zero outside the image, and the 9 taps read their shifted pixels
// from there (each input value is fetched from memory once per tile instead of once per tap).  With SW the
// chunk's weights are staged in LDS too, in MFMA fragment order, and read back with one conflict-free
// 16-byte LDS read per lane and N-tile: the 4 waves then fetch them from memory once per workgroup instead
// of once each per K-step, which pays from 4 N-tiles on; otherwise each wave streams its weight fragments
// through L1 one K-step ahead.  With a second source the halo loader reads channels [0, Ca) from the 2x
// nearest-upsampled low-resolution tensor and the rest from the skip tensor, so the decoder's upsample +
// concat is never materialised.
template <int MT, int NT, int CC, bool SW>
struct ConvLds {
    static constexpr int TW = 16 * MT, HW = TW + 2, HR = 6;
    static constexpr int PST = CC + 8;                         // LDS pixel stride in bf16 (bank padding)
    static constexpr int KS = (9 * CC + 31) / 32;              // K-steps of one chunk (zero-padded)
    static constexpr int HALO_U4 = (HR * HW * PST * 2 + 15) / 16;
    static constexpr int W_U4 = SW ? KS * NT * 64 : 0;         // weight fragments of one chunk
    static constexpr size_t bytes()
    {
        const size_t in = (size_t)(HALO_U4 + W_U4) * 16, out = (size_t)4 * TW * (16 * NT + 8) * 2;
        return in > out ? in : out;
    }
};

template <int MT, int NT, int CC, bool SW, int OCC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC))) void k_conv_lds(ConvArgs a)
{
    extern __shared__ uint4 conv_lds[];
    using L = ConvLds<MT, NT, CC, SW>;
    constexpr int TW = L::TW, HW = L::HW, HR = L::HR, PST = L::PST, KS = L::KS;
    uint16_t* lds = reinterpret_cast<uint16_t*>(conv_lds);
    uint4* wfrag = conv_lds + L::HALO_U4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles_x = (a.W + TW - 1) / TW, tiles_y = (a.H + 3) / 4;
    int tt = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tt % tiles_x;
    tt /= tiles_x;
    const int ty = tt % tiles_y, n = tt / tiles_y;
    const int x0 = tx * TW, y0 = ty * 4;
    const int r = lane & 15, g = lane >> 4;
    const int K = 9 * a.Cin;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = {};
    constexpr int GROUPS = CC / 8;
    constexpr int HALO_ITEMS = HR * HW * GROUPS;
    // item i of a chunk's halo: pixel i / GROUPS of the (HR x HW) halo, channel group i % GROUPS; item f of its
    // staged weights: lane f % 64 of fragment (K-step, N-tile) f / 64 (output channel 16 nt + (l & 15), the
    // 8 K values from 32 ks + 8 (l >> 4) on, tap = K / CC, input channel c0 + K % CC, zero from 9 CC on).
    // Every thread holds PF halo items and WPF weight items in registers: all of its loads are issued before
    // the first is waited for (loaded one by one, each load's latency would be paid in turn).
    constexpr int PF = (HALO_ITEMS + 255) / 256;
    constexpr int WPF = SW ? (L::W_U4 + 255) / 256 : 0;
    auto halo_item = [&](int c0, int i) -> uint4 {
        const int pix = i / GROUPS;
        return halo_group(a, n, y0 - 1 + pix / HW, x0 - 1 + pix % HW, c0 + 8 * (i % GROUPS));
    };
    auto w_item = [&](int c0, int f) -> uint4 {
        const int l = f & 63, q = f >> 6, nt = q % NT, ks = q / NT;
        const int co = 16 * nt + (l & 15), kk = 32 * ks + 8 * (l >> 4);
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (kk < 9 * CC && co < a.Cout) {
            const int tap = kk / CC, cl = kk - tap * CC;
            v = *reinterpret_cast<const uint4*>(a.wt + (size_t)co * K + tap * a.Cin + c0 + cl);
        }
        return v;
    };
    uint4 pf[PF];
    uint4 wpf[WPF > 0 ? WPF : 1];
    auto fetch = [&](int c0) {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int i = (int)threadIdx.x + 256 * k;
            pf[k] = (HALO_ITEMS % 256 == 0 || i < HALO_ITEMS) ? halo_item(c0, i) : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int k = 0; k < WPF; ++k) {
            const int f = (int)threadIdx.x + 256 * k;
            wpf[k] = (L::W_U4 % 256 == 0 || f < L::W_U4) ? w_item(c0, f) : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    for (int c0 = 0; c0 < a.Cin; c0 += CC) {
        fetch(c0);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int i = (int)threadIdx.x + 256 * k;
            if (HALO_ITEMS % 256 == 0 || i < HALO_ITEMS)
                *reinterpret_cast<uint4*>(lds + (i / GROUPS) * PST + 8 * (i % GROUPS)) = pf[k];
        }
#pragma unroll
        for (int k = 0; k < WPF; ++k) {
            const int f = (int)threadIdx.x + 256 * k;
            if (L::W_U4 % 256 == 0 || f < L::W_U4) wfrag[f] = wpf[k];
        }
        __syncthreads();
        // streamed weights: fragments of K-step ks loaded while the MFMAs of the step before run
        auto load_b = [&](int ks, bf16x8* Bd) {
            const int kk = 32 * ks + 8 * g;
            const bool kv = kk < 9 * CC;
            const int tap = kv ? kk / CC : 0;
            const int cl = kk - tap * CC;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int co = 16 * nt + r;
                Bd[nt] = (kv && co < a.Cout) ? load8(a.wt + (size_t)co * K + tap * a.Cin + c0 + cl) : zero;
            }
        };
        bf16x8 B[NT], Bn[NT];
        if constexpr (!SW) load_b(0, B);
        for (int ks = 0; ks < KS; ++ks) {
            if constexpr (SW) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) B[nt] = __builtin_bit_cast(bf16x8, wfrag[(ks * NT + nt) * 64 + lane]);
            } else if (ks + 1 < KS) {
                load_b(ks + 1, Bn);
            }
            const int kk = 32 * ks + 8 * g;
            const bool kv = kk < 9 * CC;
            const int tap = kv ? kk / CC : 0;
            const int cl = kk - tap * CC;
            const int dy = tap / 3, dx = tap % 3;
            bf16x8 A[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                A[mt] = kv ? __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                                 lds + ((wave + dy) * HW + 16 * mt + r + dx) * PST + cl))
                           : zero;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], B[nt], acc[mt][nt], 0, 0, 0);
            if constexpr (!SW) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) B[nt] = Bn[nt];
            }
        }
    }
    // Epilogue through LDS: each wave writes its 16 MT pixels x 16 NT channels (bias, ReLU applied) as
    // bf16 rows of a [pixel][channel] tile, then the tile leaves in 16-byte chunks, consecutive pixels of
    // one image row being contiguous in NHWC.
    constexpr int TC = 16 * NT;                 // channels of the tile
    constexpr int TS = TC + 8;                  // tile row stride (padding spreads the 4 row groups over the banks)
    constexpr int TPX = 16 * MT;                // pixels per wave
    __syncthreads();                            // every wave is done with the halo
    uint16_t* tile = lds + (size_t)wave * TPX * TS;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int co = 16 * nt + r;
        const float b = (a.bias && co < a.Cout) ? a.bias[co] : 0.0f;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = acc[mt][nt][i] + b;
                if (a.relu) v = fmaxf(v, 0.0f);
                tile[(16 * mt + 4 * g + i) * TS + co] = f2bf(v);
            }
    }
    __syncthreads();
    if (a.pool_out) {
        // 2x2 average pool of the tile (rows 0-1 and 2-3 of the 4 waves; tile origin and H, W even)
        const int Hp = a.H / 2, Wp = a.W / 2, c8p = a.Cout / 8;
        for (int q = threadIdx.x; q < 2 * (TPX / 2) * c8p; q += 256) {
            const int pp = q / c8p, c8 = q - pp * c8p;
            const int po = pp / (TPX / 2), px2 = pp % (TPX / 2);
            const int y = y0 + 2 * po, x = x0 + 2 * px2;
            if (x >= a.W || y >= a.H) continue;
            const uint16_t* t0 = lds + (size_t)(2 * po) * TPX * TS + (2 * px2) * TS + 8 * c8;
            const uint4 v = pool4(*reinterpret_cast<const uint4*>(t0), *reinterpret_cast<const uint4*>(t0 + TS),
                                  *reinterpret_cast<const uint4*>(t0 + TPX * TS),
                                  *reinterpret_cast<const uint4*>(t0 + TPX * TS + TS));
            *reinterpret_cast<uint4*>(a.pool_out + ((size_t)(n * Hp + y / 2) * Wp + x / 2) * a.Cout + 8 * c8) = v;
        }
    }
    const int y = y0 + wave;
    if (y >= a.H) return;
    const int c8n = a.Cout / 8;
    for (int q = lane; q < TPX * c8n; q += 64) {
        const int px = q / c8n, c8 = q - px * c8n;
        const int x = x0 + px;
        if (x >= a.W) continue;
        uint4 v = *reinterpret_cast<const uint4*>(tile + px * TS + 8 * c8);
        const size_t o = ((size_t)(n * a.H + y) * a.W + x) * a.Cout + 8 * c8;
        if (a.mask) {
            float f[8], mk[8];
            unpack8(v, f);
            unpack8(*reinterpret_cast<const uint4*>(a.mask + o), mk);
#pragma unroll
            for (int e = 0; e < 8; ++e) f[e] = mk[e] > 0.0f ? f[e] : 0.0f;
            v = pack8(f);
        }
        *reinterpret_cast<uint4*>(a.out + o) = v;
    }
}

// ---------------------------------------------------------------- 3x3 convolution, row-blocked
// For up to 32 output channels (NT <= 2) and Cin a multiple of 32.  With one row per wave (k_conv_lds) an
// A fragment read from LDS feeds only NT MFMAs, so these layers wait on LDS reads.  Here each wave owns R
// output rows x 16 pixels and walks the R + 2 halo rows: the fragment of halo row h and horizontal tap dx is
// read once and serves the vertical taps dy = 0, 1, 2 of output rows h - dy (up to 3 NT MFMAs per read).
// Workgroup: 4 waves side by side (tile R rows x 64 columns); the chunk's weights, 9 taps x NT fragments,
// stay in registers.  Each output row still sums its taps in the order tap = 3 dy + dx within a chunk, as
// k_conv_lds does with 32-channel chunks.
//
// Per chunk of 32 input channels the (R + 2) x 66-pixel halo is staged in LDS, 64 bytes per pixel with no
// padding: the four 16-byte channel groups of halo pixel hx sit in the slots g ^ ((hx >> 1) & 3), so that
// the A-fragment reads (16 consecutive pixels x 4 groups) hit distinct banks in every group of 8 lanes.
// The 64 interior pixels of a halo row are read from memory straight into LDS (global_load_lds_dwordx4: one
// instruction per wave and row, lane l landing at the wave's base + 16 l, so lane l fetches the channel
// group that the swizzle puts in its slot; pixels outside the image read g_zero_group); the two edge
// pixels of each row pass through registers.  No halo data occupies vector registers.
template <int R, int NT>
struct ConvRows {
    static constexpr int TW = 64, HW = TW + 2, HR = R + 2, CC = 32, PIX_BYTES = CC * 2;
    static constexpr int W_OFF = HR * HW * PIX_BYTES;   // then the chunk's 9 NT weight fragments, 1 KB each
    static constexpr size_t bytes()
    {
        const size_t in = (size_t)W_OFF + 9 * NT * 1024, out = (size_t)4 * R * 16 * (16 * NT + 8) * 2;
        return in > out ? in : out;
    }
};

__device__ inline int rows_slot_offset(int hx, int g) { return (g ^ ((hx >> 1) & 3)) << 4; }

// the 9 NT weight fragments of chunk c0 straight into LDS at `dst` (fragment f = NT tap + nt, 1 KB each; wave w
// issues every 4th); lane (r, g) of fragment (tap, nt) holds output channel 16 nt + r, input channels
// c0 + 8 g .. + 8 of that tap, zero beyond Cout
template <int NT>
__device__ __attribute__((always_inline)) inline void rows_weights_to_lds(const ConvArgs& a, int c0, char* dst, int wave,
                                                                          int r, int g)
{
    const int K = 9 * a.Cin;
    for (int f = wave; f < 9 * NT; f += 4) {
        const int tap = f / NT, co = 16 * (f % NT) + r;
        const void* src = co < a.Cout ? (const void*)(a.wt + (size_t)co * K + tap * a.Cin + c0 + 8 * g)
                                      : (const void*)&g_zero_group;
        __builtin_amdgcn_global_load_lds(src, dst + f * 1024, 16, 0, 0);
    }
}

template <int R, int NT, int OCC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC))) void k_conv_rows(ConvArgs a)
{
    extern __shared__ uint4 conv_lds[];
    using L = ConvRows<R, NT>;
    constexpr int TW = L::TW, HW = L::HW, HR = L::HR, CC = L::CC, PB = L::PIX_BYTES;
    static_assert(8 * HR <= 256, "edge items beyond one per thread");
    uint16_t* lds = reinterpret_cast<uint16_t*>(conv_lds);
    char* ldsb = reinterpret_cast<char*>(conv_lds);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles_x = (a.W + TW - 1) / TW, tiles_y = (a.H + R - 1) / R;
    int tt = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tt % tiles_x;
    tt /= tiles_x;
    const int ty = tt % tiles_y, n = tt / tiles_y;
    const int x0 = tx * TW, y0 = ty * R;
    const int r = lane & 15, g = lane >> 4;
    const int K = 9 * a.Cin;
    // this lane's interior halo group: pixel hx = 1 + 16 wave + (lane >> 2) of every halo row, LDS slot lane & 3
    const int d_hx = 1 + 16 * wave + (lane >> 2);
    const int d_x = x0 - 1 + d_hx;
    const int d_g = (lane & 3) ^ ((d_hx >> 1) & 3);
    // this thread's edge group (threads below 8 HR): halo row t >> 3, pixel 0 or HW - 1, group t & 3
    const int t = threadIdx.x;
    const int e_hy = t >> 3, e_hx = ((t >> 2) & 1) ? HW - 1 : 0, e_g = t & 3;
    const int e_off = (e_hy * HW + e_hx) * PB + rows_slot_offset(e_hx, e_g);
    // byte offsets of this lane's A fragment (pixel 16 wave + r + dx, group g) within a halo row
    int a_off[3];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        const int hx = 16 * wave + r + dx;
        a_off[dx] = hx * PB + rows_slot_offset(hx, g);
    }
    f32x4 acc[R][NT];
#pragma unroll
    for (int o = 0; o < R; ++o)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[o][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = {};
    for (int c0 = 0; c0 < a.Cin; c0 += CC) {
        __syncthreads();   // every wave is done with the previous chunk's halo and weights
        // weight fragment f = NT tap + nt, read once per workgroup straight into LDS: lane l holds output
        // channel 16 nt + (l & 15), input channels c0 + 8 (l >> 4) .. + 8 of that tap
        rows_weights_to_lds<NT>(a, c0, ldsb + L::W_OFF, wave, r, g);
#pragma unroll
        for (int hy = 0; hy < HR; ++hy) {
            const int y = y0 - 1 + hy;
            const bool ok = (unsigned)y < (unsigned)a.H && d_x < a.W;
            const void* src = ok ? (const void*)group_ptr(a, n, y, d_x, c0 + 8 * d_g) : (const void*)&g_zero_group;
            __builtin_amdgcn_global_load_lds(src, ldsb + (hy * HW + 1 + 16 * wave) * PB, 16, 0, 0);
        }
        uint4 ev = make_uint4(0u, 0u, 0u, 0u);
        if (t < 8 * HR) ev = halo_group(a, n, y0 - 1 + e_hy, x0 - 1 + e_hx, c0 + 8 * e_g);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // the direct-to-LDS loads have landed
        if (t < 8 * HR) *reinterpret_cast<uint4*>(ldsb + e_off) = ev;
        __syncthreads();
        bf16x8 B[9][NT];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                B[tap][nt] = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4*>(ldsb + L::W_OFF + (tap * NT + nt) * 1024 + lane * 16));
#pragma unroll
        for (int h = 0; h < HR; ++h)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const bf16x8 A = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(ldsb + h * HW * PB + a_off[dx]));
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const int o = h - dy;
                    if (o >= 0 && o < R) {
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            acc[o][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B[3 * dy + dx][nt], acc[o][nt],
                                                                                  0, 0, 0);
                    }
                }
            }
    }
    // epilogue through LDS, as in k_conv_lds: per wave R rows of 16 pixels x 16 NT channels
    constexpr int TC = 16 * NT;
    constexpr int TS = TC + 8;                  // tile row stride (padding spreads the 4 row groups over the banks)
    __syncthreads();
    uint16_t* tile = lds + (size_t)wave * R * 16 * TS;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int co = 16 * nt + r;
        const float b = (a.bias && co < a.Cout) ? a.bias[co] : 0.0f;
#pragma unroll
        for (int o = 0; o < R; ++o)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = acc[o][nt][i] + b;
                if (a.relu) v = fmaxf(v, 0.0f);
                tile[(o * 16 + 4 * g + i) * TS + co] = f2bf(v);
            }
    }
    __syncthreads();
    const int c8n = a.Cout / 8;
    if (a.head_out) {
        // the network's head on each pixel of the tile, from the BF16 values the layer would have stored
        for (int px = lane; px < R * 16; px += 64) {
            const int o = px / 16, x = x0 + 16 * wave + (px % 16), y = y0 + o;
            if (x >= a.W || y >= a.H) continue;
            float f[32];
#pragma unroll
            for (int q = 0; q < 4; ++q) unpack8(*reinterpret_cast<const uint4*>(tile + px * TS + 8 * q), f + 8 * q);
            a.head_out[(size_t)(n * a.H + y) * a.W + x] = head_value(f, a.head_w, a.head_b);
        }
    } else {
        for (int q = lane; q < R * 16 * c8n; q += 64) {
            const int px = q / c8n, c8 = q - px * c8n;
            const int o = px / 16, x = x0 + 16 * wave + (px % 16), y = y0 + o;
            if (x >= a.W || y >= a.H) continue;
            uint4 v = *reinterpret_cast<const uint4*>(tile + px * TS + 8 * c8);
            const size_t off = ((size_t)(n * a.H + y) * a.W + x) * a.Cout + 8 * c8;
            if (a.mask) {
                float f[8], mk[8];
                unpack8(v, f);
                unpack8(*reinterpret_cast<const uint4*>(a.mask + off), mk);
#pragma unroll
                for (int e = 0; e < 8; ++e) f[e] = mk[e] > 0.0f ? f[e] : 0.0f;
                v = pack8(f);
            }
            *reinterpret_cast<uint4*>(a.out + off) = v;
        }
    }
    if (a.pool_out) {
        // 2x2 average pool of the wave's R rows x 16 pixels (tile origin and H, W even)
        const int Hp = a.H / 2, Wp = a.W / 2;
        for (int q = lane; q < (R / 2) * 8 * c8n; q += 64) {
            const int pp = q / c8n, c8 = q - pp * c8n;
            const int po = pp / 8, px2 = pp % 8;
            const int y = y0 + 2 * po, x = x0 + 16 * wave + 2 * px2;
            if (x >= a.W || y >= a.H) continue;
            const uint16_t* t0 = tile + (2 * po * 16 + 2 * px2) * TS + 8 * c8;
            const uint4 v = pool4(*reinterpret_cast<const uint4*>(t0), *reinterpret_cast<const uint4*>(t0 + TS),
                                  *reinterpret_cast<const uint4*>(t0 + 16 * TS),
                                  *reinterpret_cast<const uint4*>(t0 + 17 * TS));
            *reinterpret_cast<uint4*>(a.pool_out + ((size_t)(n * Hp + y / 2) * Wp + x / 2) * a.Cout + 8 * c8) = v;
        }
    }
}

// ---------------------------------------------------------------- FP32 copy of the network
// 3x3 convolution in FP32 on v_mfma_f32_16x16x4_f32: FP32 activations and weights (the master copy,
// transposed to [tap][ci][co]), FP32 accumulation.  Same tiling as k_conv_lds with one 16-pixel M-tile
// per wave; the halo of a CC-channel chunk is staged in LDS; the first layer reads the BF16 features, and
// the decoder's upsample + concat is fused into the halo load as in the BF16 kernel.
template <int NT, int CC>
__global__ __launch_bounds__(256) void k_conv_f32(ConvArgsF32 a)
{
    extern __shared__ float cf_lds[];
    constexpr int TW = 16, HW = TW + 2, HR = 6, PST = CC + 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles_x = (a.W + TW - 1) / TW, tiles_y = (a.H + 3) / 4;
    int tt = blockIdx.x;
    const int tx = tt % tiles_x;
    tt /= tiles_x;
    const int ty = tt % tiles_y, n = tt / tiles_y;
    const int x0 = tx * TW, y0 = ty * 4;
    const int r = lane & 15, kq = lane >> 4;
    const int Cs = a.Cin - a.Ca;
    f32x4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < a.Cin; c0 += CC) {
        __syncthreads();
        for (int i = threadIdx.x; i < HR * HW * (CC / 4); i += 256) {
            const int g4 = i % (CC / 4), pix = i / (CC / 4);
            const int hx = pix % HW, hy = pix / HW;
            const int y = y0 - 1 + hy, x = x0 - 1 + hx, ci = c0 + 4 * g4;
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (y >= 0 && y < a.H && x >= 0 && x < a.W) {
                if (a.in_bf16) {
                    const uint2 q = *reinterpret_cast<const uint2*>(
                        static_cast<const uint16_t*>(a.in) + ((size_t)(n * a.H + y) * a.W + x) * a.Cin + ci);
                    v[0] = __uint_as_float(q.x << 16); v[1] = __uint_as_float(q.x & 0xFFFF0000u);
                    v[2] = __uint_as_float(q.y << 16); v[3] = __uint_as_float(q.y & 0xFFFF0000u);
                } else {
                    const float* src;
                    if (a.in2 == nullptr)
                        src = static_cast<const float*>(a.in) + ((size_t)(n * a.H + y) * a.W + x) * a.Cin + ci;
                    else if (ci < a.Ca)
                        src = static_cast<const float*>(a.in) +
                              ((size_t)(n * (a.H / 2) + y / 2) * (a.W / 2) + x / 2) * a.Ca + ci;
                    else
                        src = a.in2 + ((size_t)(n * a.H + y) * a.W + x) * Cs + (ci - a.Ca);
                    const float4 q = *reinterpret_cast<const float4*>(src);
                    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) cf_lds[pix * PST + 4 * g4 + e] = v[e];
        }
        __syncthreads();
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;
            const float* arow = cf_lds + ((wave + dy) * HW + r + dx) * PST;
            const float* wrow = a.wt + ((size_t)tap * a.Cin + c0) * a.Cout + r;
            for (int kc = 0; kc < CC; kc += 4) {
                const float A = arow[kc + kq];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const float B = wrow[(size_t)(kc + kq) * a.Cout + 16 * nt];
                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A, B, acc[nt], 0, 0, 0);
                }
            }
        }
    }
    // D layout: lane holds column (channel) 16 nt + (lane & 15), rows (pixels) 4 (lane >> 4) + e
    const int y = y0 + wave;
    if (y >= a.H) return;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int co = 16 * nt + r;
        const float b = a.bias[co];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int x = x0 + 4 * kq + e;
            if (x >= a.W) continue;
            a.out[((size_t)(n * a.H + y) * a.W + x) * a.Cout + co] = fmaxf(acc[nt][e] + b, 0.0f);
        }
    }
}

__global__ __launch_bounds__(256) void k_pool2_f32(const float* in, int N, int H, int W, int C, float* out)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    int h = H / 2, w = W / 2, C4 = C / 4;
    size_t total = (size_t)N * h * w * C4;
    if (i >= total) return;
    int c = (int)(i % C4) * 4;
    size_t q = i / C4;
    int x = (int)(q % w), t = (int)(q / w), y = t % h, n = t / h;
    const float* b = in + (((size_t)n * H + 2 * y) * W + 2 * x) * C + c;
    float4 p0 = *reinterpret_cast<const float4*>(b), p1 = *reinterpret_cast<const float4*>(b + C);
    float4 p2 = *reinterpret_cast<const float4*>(b + (size_t)W * C), p3 = *reinterpret_cast<const float4*>(b + (size_t)W * C + C);
    float4 o;
    o.x = ((p0.x + p1.x) + (p2.x + p3.x)) * 0.25f;
    o.y = ((p0.y + p1.y) + (p2.y + p3.y)) * 0.25f;
    o.z = ((p0.z + p1.z) + (p2.z + p3.z)) * 0.25f;
    o.w = ((p0.w + p1.w) + (p2.w + p3.w)) * 0.25f;
    *reinterpret_cast<float4*>(out + q * C + c) = o;
}

// y = sigmoid(sum_c d1[p][c] wh[c] + bh) with the FP32 head weights
__global__ __launch_bounds__(256) void k_head_f32(const float* d1, const float* wh, const float* bh, int P, float* y)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float s = 0.0f;
    const float* row = d1 + (size_t)p * 32;
    for (int c = 0; c < 32; ++c) s += row[c] * wh[c];
    s += bh[0];
    y[p] = 1.0f / (1.0f + expf(-s));
}

// FP32 master [Cout][9][Cin] -> [9][Cin][Cout]
__global__ __launch_bounds__(256) void k_weights_f32t(const float* w, int Cout, int Cin, float* wt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n = Cout * 9 * Cin;
    if (i >= n) return;
    int ci = i % Cin, tap = (i / Cin) % 9, co = i / (9 * Cin);
    wt[((size_t)tap * Cin + ci) * Cout + co] = w[i];
}

// ---------------------------------------------------------------- weight gradient
// One wave per (pixel chunk, tap, 16-channel output tile, 16-channel input tile).
__global__ __launch_bounds__(64) void k_wgrad(WgradArgs a)
{
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
    const int P = a.N * a.H * a.W;
    const int chunk = blockIdx.x, tap = blockIdx.y;
    const int ci_tiles = (a.Cin + 15) / 16;
    const int co_t = blockIdx.z / ci_tiles, ci_t = blockIdx.z % ci_tiles;
    const int co = co_t * 16 + r, ci = ci_t * 16 + r;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int pb0 = chunk * a.chunk, pe = min(P, pb0 + a.chunk);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int pb = pb0; pb < pe; pb += 32) {
        uint16_t av[8], bv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int p = pb + 8 * g + e;
            av[e] = 0;
            bv[e] = 0;
            if (p < pe) {
                av[e] = a.g[(size_t)p * a.Cout + co];
                int x = p % a.W, t = p / a.W, y = t % a.H, n = t / a.H;
                int ys = y + dy, xs = x + dx;
                if (ci < a.Cin && ys >= 0 && ys < a.H && xs >= 0 && xs < a.W)
                    bv[e] = a.x[((size_t)(n * a.H + ys) * a.W + xs) * a.Cin + ci];
            }
        }
        uint4 ua, ub;
        ua.x = av[0] | ((uint32_t)av[1] << 16); ua.y = av[2] | ((uint32_t)av[3] << 16);
        ua.z = av[4] | ((uint32_t)av[5] << 16); ua.w = av[6] | ((uint32_t)av[7] << 16);
        ub.x = bv[0] | ((uint32_t)bv[1] << 16); ub.y = bv[2] | ((uint32_t)bv[3] << 16);
        ub.z = bv[4] | ((uint32_t)bv[5] << 16); ub.w = bv[6] | ((uint32_t)bv[7] << 16);
        bf16x8 A = __builtin_bit_cast(bf16x8, ua);
        bf16x8 B = __builtin_bit_cast(bf16x8, ub);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc, 0, 0, 0);
    }
    // D[i = output channel][j = input channel]: lane holds j = lane & 15, rows 4 (lane >> 4) + i
    int cio = ci_t * 16 + r;
    if (cio >= a.Cin) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int coo = co_t * 16 + 4 * g + i;
        a.partial[(((size_t)chunk * a.Cout + coo) * 9 + tap) * a.Cin + cio] = acc[i];
    }
}

// ---------------------------------------------------------------- weight gradient, LDS-tiled
// dW[co][tap][ci] = sum_p g[p][co] x[p + off(tap)][ci] as MFMA GEMMs with K = pixels.  Workgroup of 3
// waves; wave w owns the taps of kernel row dy = w.  Pixel tiles are 2 rows x 64 columns; for each tile
// the gradient (all Cout channels) is staged in LDS transposed to [channel][pixel], and the input halo
// (4 rows x 66 columns, 16 CI_T channels) in three copies shifted by dx = 0, 1, 2, also [channel][pixel],
// so that every MFMA operand (8 consecutive pixels of one channel) is one aligned 16-byte LDS read.  A
// workgroup accumulates a chunk of consecutive tiles for one group of input channels and writes its
// partial sums; the chunks are then added in chunk order, so the result is deterministic.
constexpr int WG_TW = 64, WG_R = 2;
template <int CO_T, int CI_T>
__global__ __launch_bounds__(192) void k_wgrad_lds(WgradArgs a, int tiles_per_chunk)
{
    extern __shared__ uint4 wg_lds[];
    constexpr int TW = WG_TW, R = WG_R, HRW = R + 2, HC = TW + 2;
    constexpr int CIN_T = 16 * CI_T, COUT = 16 * CO_T;
    constexpr int GS_CO = R * TW + 8;      // bf16 elements per gradient channel row (padded)
    constexpr int XS_CI = HRW * TW + 8;    // bf16 elements per input channel (4 halo rows, padded)
    constexpr int XS_DX = CIN_T * XS_CI;
    uint16_t* gs = reinterpret_cast<uint16_t*>(wg_lds);
    uint16_t* xs = gs + COUT * GS_CO;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int ci0 = blockIdx.y * CIN_T;
    const int tiles_x = (a.W + TW - 1) / TW, tiles_y = (a.H + R - 1) / R;
    const int n_tiles = a.N * tiles_x * tiles_y;
    const int t_begin = blockIdx.x * tiles_per_chunk, t_end = min(n_tiles, t_begin + tiles_per_chunk);
    const int c8_out = a.Cout / 8;
    f32x4 acc[3][CO_T][CI_T];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int i = 0; i < CO_T; ++i)
#pragma unroll
            for (int j = 0; j < CI_T; ++j) acc[dx][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int t = t_begin; t < t_end; ++t) {
        const int tx = t % tiles_x, rest = t / tiles_x, ty = rest % tiles_y, n = rest / tiles_y;
        const int x0 = tx * TW, y0 = ty * R;
        // Staging, transposed to [channel][pixel] in registers: a thread holds the 8-channel groups of 8 (10)
        // consecutive pixels and writes, for each of the 8 channels, the 8 pixels as one 16-byte LDS store
        // (two pixels per 32-bit word); the input's dx-shifted copies come from the same 10 registers.  All
        // loads of an item are in flight together (clamped addresses, zeros substituted afterwards).
        constexpr int X_ITEMS = HRW * (TW / 8) * (CIN_T / 8), G_ITEMS = R * (TW / 8) * (COUT / 8);
        static_assert(X_ITEMS <= 192, "one input item per thread");
        auto pack_ch = [](const uint4& lo, const uint4& hi, int e) -> uint32_t {
            const uint32_t wl = e < 2 ? lo.x : e < 4 ? lo.y : e < 6 ? lo.z : lo.w;
            const uint32_t wh = e < 2 ? hi.x : e < 4 ? hi.y : e < 6 ? hi.z : hi.w;
            return (e & 1) ? ((wl >> 16) | (wh & 0xFFFF0000u)) : ((wl & 0xFFFFu) | (wh << 16));
        };
        uint4 xv[10];
        int x_c8 = 0, x_q = 0, x_row = 0;
        const bool x_item = (int)threadIdx.x < X_ITEMS;
        // consecutive threads take consecutive 8-pixel groups q, so that the 16-byte stores of 8 neighbouring
        // lanes (one channel row, q = 0..7) cover all LDS banks
        if (x_item) {
            x_q = threadIdx.x % (TW / 8);
            const int rest = threadIdx.x / (TW / 8);
            x_c8 = rest % (CIN_T / 8);
            x_row = rest / (CIN_T / 8);
            const int y = y0 - 1 + x_row, ci = ci0 + 8 * x_c8;
            const bool rowok = y >= 0 && y < a.H && ci < a.Cin;
            const int yc = min(max(y, 0), a.H - 1), cic = ci < a.Cin ? ci : 0;
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                const int x = x0 - 1 + 8 * x_q + k;
                const int xc = min(max(x, 0), a.W - 1);
                const uint4 v = *reinterpret_cast<const uint4*>(a.x + ((size_t)(n * a.H + yc) * a.W + xc) * a.Cin + cic);
                xv[k] = (rowok && x >= 0 && x < a.W) ? v : make_uint4(0u, 0u, 0u, 0u);
            }
        }
        auto g_load = [&](int it, uint4* gv) {
            const int q = it % (TW / 8), rest = it / (TW / 8), c8 = rest % c8_out, row = rest / c8_out;
            const int y = y0 + row, yc = min(y, a.H - 1);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int x = x0 + 8 * q + k, xc = min(x, a.W - 1);
                const uint4 v = *reinterpret_cast<const uint4*>(a.g + ((size_t)(n * a.H + yc) * a.W + xc) * a.Cout + 8 * c8);
                gv[k] = (y < a.H && x < a.W) ? v : make_uint4(0u, 0u, 0u, 0u);
            }
        };
        auto g_store = [&](int it, const uint4* gv) {
            const int q = it % (TW / 8), rest = it / (TW / 8), c8 = rest % c8_out, row = rest / c8_out;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                *reinterpret_cast<uint4*>(gs + (8 * c8 + e) * GS_CO + row * TW + 8 * q) =
                    make_uint4(pack_ch(gv[0], gv[1], e), pack_ch(gv[2], gv[3], e), pack_ch(gv[4], gv[5], e),
                               pack_ch(gv[6], gv[7], e));
        };
        uint4 gv[8];
        const bool g_first = (int)threadIdx.x < G_ITEMS;
        if (g_first) g_load(threadIdx.x, gv);
        __syncthreads();   // every wave is done with the previous tile's operands
        if (x_item) {
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    *reinterpret_cast<uint4*>(xs + dx * XS_DX + (8 * x_c8 + e) * XS_CI + x_row * TW + 8 * x_q) =
                        make_uint4(pack_ch(xv[dx], xv[dx + 1], e), pack_ch(xv[dx + 2], xv[dx + 3], e),
                                   pack_ch(xv[dx + 4], xv[dx + 5], e), pack_ch(xv[dx + 6], xv[dx + 7], e));
        }
        if (g_first) g_store(threadIdx.x, gv);
        for (int it = threadIdx.x + 192; it < G_ITEMS; it += 192) {
            g_load(it, gv);
            g_store(it, gv);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < R * TW / 32; ++s) {
            const int row = s / (TW / 32), c0 = 32 * (s % (TW / 32));
            bf16x8 A[CO_T], B[3][CI_T];
#pragma unroll
            for (int i = 0; i < CO_T; ++i)
                A[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                                                       gs + (16 * i + r) * GS_CO + row * TW + c0 + 8 * g));
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int j = 0; j < CI_T; ++j)
                    B[dx][j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                                   xs + dx * XS_DX + (16 * j + r) * XS_CI + (row + wave) * TW + c0 + 8 * g));
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int i = 0; i < CO_T; ++i)
#pragma unroll
                    for (int j = 0; j < CI_T; ++j)
                        acc[dx][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i], B[dx][j], acc[dx][i][j], 0, 0, 0);
        }
    }
    // D[i = output channel][j = input channel]: lane holds j = lane & 15, rows 4 (lane >> 4) + e
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int i = 0; i < CO_T; ++i)
#pragma unroll
            for (int j = 0; j < CI_T; ++j) {
                const int ci = ci0 + 16 * j + r;
                if (ci >= a.Cin) continue;
                const int tap = 3 * wave + dx;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int co = 16 * i + 4 * g + e;
                    a.partial[(((size_t)blockIdx.x * a.Cout + co) * 9 + tap) * a.Cin + ci] = acc[dx][i][j][e];
                }
            }
}

// out[i] (+)= sum over chunks c of partial[c][i]: 16 outputs per workgroup, 16 lanes per output summing
// chunks q, q + 16, q + 32, ... in order, then a fixed-order tree over the 16 lanes
__global__ __launch_bounds__(256) void k_reduce_chunks(const float* partial, int n_chunks, int n, float* out, int add)
{
    __shared__ float sm[16][17];
    const int o = threadIdx.x & 15, q = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + o;
    float s = 0.0f;
    if (i < n)
        for (int c = q; c < n_chunks; c += 16) s += partial[(size_t)c * n + i];
    sm[q][o] = s;
    __syncthreads();
    for (int h = 8; h > 0; h >>= 1) {
        if (q < h) sm[q][o] += sm[q + h][o];
        __syncthreads();
    }
    if (q == 0 && i < n) out[i] = add ? out[i] + sm[0][o] : sm[0][o];
}

// Column sums of a bf16 [P][C] tensor (C a multiple of 8, at most 256), per block of COLSUM_ROWS pixels:
// a thread sums 8 channels over every G-th pixel of the block (G = 2048 / C pixel groups), then the
// groups are added in a fixed tree order, so the result does not depend on scheduling.
constexpr int COLSUM_ROWS = 1024;
__global__ __launch_bounds__(256) void k_colsum(const uint16_t* g, int P, int C, float* partial)
{
    __shared__ float sm[8][256];
    const int cg_n = C / 8, G = 256 / cg_n;
    const int t = threadIdx.x, cg = t % cg_n, grp = t / cg_n;
    const int p0 = blockIdx.x * COLSUM_ROWS, pe = min(P, p0 + COLSUM_ROWS);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (grp < G) {
        for (int p = p0 + grp; p < pe; p += G) {
            uint4 v = *reinterpret_cast<const uint4*>(g + (size_t)p * C + 8 * cg);
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                acc[2 * e] += __uint_as_float(w[e] << 16);
                acc[2 * e + 1] += __uint_as_float(w[e] & 0xFFFF0000u);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) sm[e][t] = acc[e];
    __syncthreads();
    for (int h = G / 2; h > 0; h >>= 1) {
        if (grp < h) {
#pragma unroll
            for (int e = 0; e < 8; ++e) sm[e][t] += sm[e][t + h * cg_n];
        }
        __syncthreads();
    }
    if (grp == 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) partial[(size_t)blockIdx.x * C + 8 * cg + e] = sm[e][t];
    }
}

// out[o] (+)= sum over blocks b of partial[b][o], o < n: one workgroup per output, fixed-order tree
__global__ __launch_bounds__(256) void k_reduce_blocks(const float* partial, int nb, int n, float* out, int add)
{
    __shared__ float sm[256];
    const int o = blockIdx.x, t = threadIdx.x;
    float s = 0.0f;
    for (int b = t; b < nb; b += 256) s += partial[(size_t)b * n + o];
    sm[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) sm[t] += sm[t + h];
        __syncthreads();
    }
    if (t == 0) out[o] = add ? out[o] + sm[0] : sm[0];
}

// ---------------------------------------------------------------- pooling / upsampling / concat
// All channel counts and offsets are multiples of 8: one thread handles 8 channels (16 bytes).
__device__ inline uint4 ld8(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ inline void st8(uint16_t* p, uint4 v) { *reinterpret_cast<uint4*>(p) = v; }

__global__ __launch_bounds__(256) void k_pool2(const uint16_t* in, int N, int H, int W, int C, uint16_t* out)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    int h = H / 2, w = W / 2, C8 = C / 8;
    size_t total = (size_t)N * h * w * C8;
    if (i >= total) return;
    int c = (int)(i % C8) * 8;
    size_t q = i / C8;
    int x = (int)(q % w), t = (int)(q / w), y = t % h, n = t / h;
    const uint16_t* b = in + (((size_t)n * H + 2 * y) * W + 2 * x) * C + c;
    st8(out + q * C + c, pool4(ld8(b), ld8(b + C), ld8(b + (size_t)W * C), ld8(b + (size_t)W * C + C)));
}

// out[N,2h,2w,Ca+Cs] = [nearest-upsampled a (Ca channels), skip (Cs channels)]
__global__ __launch_bounds__(256) void k_up2_concat(const uint16_t* a, const uint16_t* skip, int N, int H, int W,
                                                    int Ca, int Cs, uint16_t* out)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    int C = Ca + Cs, C8 = C / 8;
    size_t total = (size_t)N * H * W * C8;
    if (i >= total) return;
    int c = (int)(i % C8) * 8;
    size_t q = i / C8;
    int x = (int)(q % W), t = (int)(q / W), y = t % H, n = t / H;
    uint4 v = c < Ca ? ld8(a + (((size_t)n * (H / 2) + y / 2) * (W / 2) + x / 2) * Ca + c)
                     : ld8(skip + q * Cs + (c - Ca));
    st8(out + q * C + c, v);
}

// gradient of the upsampled part of a concat: out[n,y,x,c] = mask * sum_{2x2} g[n,2y+a,2x+b, c0 + c]
__global__ __launch_bounds__(256) void k_up_back_mask(const uint16_t* g, int N, int H2, int W2, int Ctot, int c0,
                                                      int C, const uint16_t* mask, uint16_t* out)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    int h = H2 / 2, w = W2 / 2, C8 = C / 8;
    size_t total = (size_t)N * h * w * C8;
    if (i >= total) return;
    int c = (int)(i % C8) * 8;
    size_t q = i / C8;
    int x = (int)(q % w), t = (int)(q / w), y = t % h, n = t / h;
    const uint16_t* b = g + (((size_t)n * H2 + 2 * y) * W2 + 2 * x) * Ctot + c0 + c;
    float a[8], bb[8], cc[8], d[8], mk[8], r[8];
    unpack8(ld8(b), a); unpack8(ld8(b + Ctot), bb);
    unpack8(ld8(b + (size_t)W2 * Ctot), cc); unpack8(ld8(b + (size_t)W2 * Ctot + Ctot), d);
    unpack8(ld8(mask + q * C + c), mk);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        float s = (a[e] + bb[e]) + (cc[e] + d[e]);
        r[e] = mk[e] > 0.0f ? s : 0.0f;
    }
    st8(out + q * C + c, pack8(r));
}

// out[n,y,x,c] = mask * (gpool[n,y/2,x/2,c] / 4 + gcat[n,y,x,c0 + c])
__global__ __launch_bounds__(256) void k_pool_back_add_mask(const uint16_t* gpool, const uint16_t* gcat, int N, int H,
                                                            int W, int C, int Ctot, int c0, const uint16_t* mask,
                                                            uint16_t* out)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    int C8 = C / 8;
    size_t total = (size_t)N * H * W * C8;
    if (i >= total) return;
    int c = (int)(i % C8) * 8;
    size_t q = i / C8;
    int x = (int)(q % W), t = (int)(q / W), y = t % H, n = t / H;
    float gp[8], gc[8], mk[8], r[8];
    unpack8(ld8(gpool + (((size_t)n * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c), gp);
    unpack8(ld8(gcat + q * Ctot + c0 + c), gc);
    unpack8(ld8(mask + q * C + c), mk);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        float v = gp[e] * 0.25f;
        v = v + gc[e];
        r[e] = mk[e] > 0.0f ? v : 0.0f;
    }
    st8(out + q * C + c, pack8(r));
}

// ---------------------------------------------------------------- head, loss
// y = sigmoid(sum_c d1[p][c] wh[c] + bh), wh rounded to BF16 like every weight, bh in FP32 like every bias
__global__ __launch_bounds__(256) void k_head(const uint16_t* d1, const float* wh, const float* bh, int P, float* y)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const uint16_t* row = d1 + (size_t)p * 32;
    float f[32];
#pragma unroll
    for (int q = 0; q < 4; ++q) unpack8(ld8(row + 8 * q), f + 8 * q);
    y[p] = head_value(f, wh, bh);
}

// per-chunk sums of mask and mask * (y - t)^2
__global__ __launch_bounds__(256) void k_loss_partials(const float* y, const float* t, const float* m, int P, int chunk,
                                                       float* partial)
{
    __shared__ float sm[256], sl[256];
    int p0 = blockIdx.x * chunk, pe = min(P, p0 + chunk);
    float a = 0.0f, b = 0.0f;
    for (int p = p0 + threadIdx.x; p < pe; p += blockDim.x) {
        float d = y[p] - t[p];
        a += m[p];
        b += m[p] * d * d;
    }
    sm[threadIdx.x] = a;
    sl[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) { sm[threadIdx.x] += sm[threadIdx.x + s]; sl[threadIdx.x] += sl[threadIdx.x + s]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { partial[2 * blockIdx.x] = sm[0]; partial[2 * blockIdx.x + 1] = sl[0]; }
}

// sums[0] = sum mask, sums[1] = loss = sum m (y-t)^2 / max(sum m, 1)
__global__ void k_loss_final(const float* partial, int n, float* sums)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float a = 0.0f, b = 0.0f;
    for (int i = 0; i < n; ++i) { a += partial[2 * i]; b += partial[2 * i + 1]; }
    sums[0] = a;
    sums[1] = b / fmaxf(a, 1.0f);
}

// dlogit = 2 m (y - t) / max(sum m, 1) * y (1 - y); gpre_d1 = mask(d1 > 0) * dlogit * wh; one pixel per
// thread, and per block of 256 pixels the partial head gradients (32 weights, then the bias) summed in a
// fixed tree order
__global__ __launch_bounds__(256) void k_head_back(const uint16_t* d1, const float* y, const float* t, const float* m,
                                                   const float* sums, const float* wh, int P, uint16_t* gpre,
                                                   float* partial)
{
    __shared__ float sm[33][256];
    const int tid = threadIdx.x;
    const int p = blockIdx.x * 256 + tid;
    float v[33];
#pragma unroll
    for (int c = 0; c < 33; ++c) v[c] = 0.0f;
    if (p < P) {
        const float inv = 2.0f / fmaxf(sums[0], 1.0f);
        const float yy = y[p];
        const float dl = m[p] * (yy - t[p]) * inv * yy * (1.0f - yy);
        const uint4* row = reinterpret_cast<const uint4*>(d1 + (size_t)p * 32);
        uint4* out = reinterpret_cast<uint4*>(gpre + (size_t)p * 32);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint4 r = row[q];
            uint32_t w[4] = {r.x, r.y, r.z, r.w}, o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float a0 = __uint_as_float(w[e] << 16), a1 = __uint_as_float(w[e] & 0xFFFF0000u);
                int c = 8 * q + 2 * e;
                v[c] = dl * a0;
                v[c + 1] = dl * a1;
                uint32_t g0 = a0 > 0.0f ? f2bf(dl * bf2f(f2bf(wh[c]))) : 0u;
                uint32_t g1 = a1 > 0.0f ? f2bf(dl * bf2f(f2bf(wh[c + 1]))) : 0u;
                o[e] = g0 | (g1 << 16);
            }
            out[q] = make_uint4(o[0], o[1], o[2], o[3]);
        }
        v[32] = dl;
    }
#pragma unroll
    for (int c = 0; c < 33; ++c) sm[c][tid] = v[c];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
#pragma unroll
            for (int c = 0; c < 33; ++c) sm[c][tid] += sm[c][tid + h];
        }
        __syncthreads();
    }
    if (tid < 33) partial[(size_t)blockIdx.x * 33 + tid] = sm[tid][0];
}

// ---------------------------------------------------------------- weights, Adam, features
// FP32 master [Cout][9][Cin] -> BF16 copies: forward layout and flipped/transposed Wf[ci][8 - tap][co]
__global__ __launch_bounds__(256) void k_weights_bf16(const float* w, int Cout, int Cin, uint16_t* wf, uint16_t* wb)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n = Cout * 9 * Cin;
    if (i >= n) return;
    int ci = i % Cin, tap = (i / Cin) % 9, co = i / (9 * Cin);
    uint16_t v = f2bf(w[i]);
    wf[i] = v;
    if (wb) wb[((size_t)ci * 9 + (8 - tap)) * Cout + co] = v;
}

__global__ __launch_bounds__(256) void k_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1,
                                              float b2, float eps, float c1, float c2)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float mh = mi / c1, vh = vi / c2;
    w[i] = w[i] - lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_fill_f32(float* p, float v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned nb(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

template <int MT, int NT, int CC, bool SW, int OCC>
void launch_conv_lds(const ConvArgs& a, hipStream_t st)
{
    constexpr int TW = 16 * MT;
    const size_t tiles = (size_t)a.N * ((a.H + 3) / 4) * ((a.W + TW - 1) / TW);
    const size_t lds = ConvLds<MT, NT, CC, SW>::bytes();
    hipLaunchKernelGGL((k_conv_lds<MT, NT, CC, SW, OCC>), dim3((unsigned)tiles), dim3(256), lds, st, a);
}

template <int R, int NT, int OCC>
void launch_conv_rows(const ConvArgs& a, hipStream_t st)
{
    const size_t tiles = (size_t)a.N * ((a.H + R - 1) / R) * ((a.W + 63) / 64);
    const size_t lds = ConvRows<R, NT>::bytes();
    hipLaunchKernelGGL((k_conv_rows<R, NT, OCC>), dim3((unsigned)tiles), dim3(256), lds, st, a);
}

void unet_conv3x3(const ConvArgs& a, hipStream_t st)
{
    const int nt = (a.Cout + 15) / 16;
    // up to 2 N-tiles: row-blocked waves over 32-channel chunks with the weights in registers (8-channel
    // inputs: the one-row kernel with 8-channel chunks, weights streamed through L1); from 4 N-tiles on: weights
    // staged in LDS, with chunks small enough that halo and weights fit in 64 KB (16 channels up to 8
    // N-tiles, padding a chunk's 144 K values to 160; 8 channels beyond)
    int cfg = 0;
    if (nt <= 2)
        cfg = a.Cin % 64 == 0 ? 264 : (a.Cin % 32 == 0 ? 232 : 208);
    else if (a.Cin % 16 == 0)
        cfg = nt * 100 + (nt <= 8 ? 16 : 8);
    static_assert(ConvRows<RC_CONV_ROWS, 2>::bytes() <= 65536 && ConvLds<4, 4, 16, true>::bytes() <= 65536 &&
                      ConvLds<2, 6, 16, true>::bytes() <= 65536 && ConvLds<2, 8, 16, true>::bytes() <= 65536 &&
                      ConvLds<2, 12, 8, true>::bytes() <= 65536,
                  "convolution LDS beyond 64 KB");
    switch (cfg) {
    case 208: launch_conv_lds<4, 2, 8, false, RC_OCC_E1A>(a, st); return;
    case 232:
    case 264:
        if (nt == 1) launch_conv_rows<RC_CONV_ROWS, 1, RC_OCC_ROWS + 1>(a, st);
        else launch_conv_rows<RC_CONV_ROWS, 2, RC_OCC_ROWS>(a, st);
        return;
    case 416: launch_conv_lds<4, 4, 16, true, RC_OCC_416>(a, st); return;
    case 616: launch_conv_lds<2, 6, 16, true, RC_OCC_816>(a, st); return;
    case 816: launch_conv_lds<2, 8, 16, true, RC_OCC_816>(a, st); return;
    case 1208: launch_conv_lds<2, 12, 8, true, 1>(a, st); return;
    default: break;
    }
    unet_conv3x3_direct(a, st);
}

void unet_conv3x3_direct(const ConvArgs& a, hipStream_t st)
{
    size_t P = (size_t)a.N * a.H * a.W;
    dim3 grid(nb(P, 128)), block(256);
    int nt = (a.Cout + 15) / 16;
    switch (nt) {
    case 1: hipLaunchKernelGGL(k_conv3x3<1>, grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_conv3x3<2>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_conv3x3<4>, grid, block, 0, st, a); break;
    case 6: hipLaunchKernelGGL(k_conv3x3<6>, grid, block, 0, st, a); break;
    case 8: hipLaunchKernelGGL(k_conv3x3<8>, grid, block, 0, st, a); break;
    case 12: hipLaunchKernelGGL(k_conv3x3<12>, grid, block, 0, st, a); break;
    default: break;   // channel counts of this network only
    }
}

int unet_wgrad_chunks(size_t P, int chunk) { return (int)((P + chunk - 1) / chunk); }

void unet_wgrad(const WgradArgs& a, hipStream_t st)
{
    size_t P = (size_t)a.N * a.H * a.W;
    int chunks = unet_wgrad_chunks(P, a.chunk);
    dim3 grid(chunks, 9, (a.Cout / 16) * ((a.Cin + 15) / 16));
    hipLaunchKernelGGL(k_wgrad, grid, dim3(64), 0, st, a);
}

namespace {
struct WgradShape {
    int co_t, ci_t, ci_groups, tiles_per_chunk, chunks;
};
WgradShape wgrad_shape(const WgradArgs& a)
{
    WgradShape w;
    w.co_t = a.Cout / 16;
    w.ci_t = w.co_t >= 8 ? 1 : (a.Cin <= 16 ? 1 : 2);
    w.ci_groups = (a.Cin + 16 * w.ci_t - 1) / (16 * w.ci_t);
    const int tiles = a.N * ((a.H + WG_R - 1) / WG_R) * ((a.W + WG_TW - 1) / WG_TW);
    const int target = std::max(1, 1024 / w.ci_groups);
    w.tiles_per_chunk = std::max(1, (tiles + target - 1) / target);
    w.chunks = (tiles + w.tiles_per_chunk - 1) / w.tiles_per_chunk;
    return w;
}
}  // namespace

int unet_wgrad_lds_chunks(const WgradArgs& a) { return wgrad_shape(a).chunks; }

bool unet_wgrad_lds(const WgradArgs& a, hipStream_t st)
{
    const WgradShape w = wgrad_shape(a);
    const size_t lds = ((size_t)16 * w.co_t * (WG_R * WG_TW + 8) + (size_t)3 * 16 * w.ci_t * ((WG_R + 2) * WG_TW + 8)) * 2;
    const dim3 grid(w.chunks, w.ci_groups);
    switch (w.co_t * 10 + w.ci_t) {
    case 21: hipLaunchKernelGGL((k_wgrad_lds<2, 1>), grid, dim3(192), lds, st, a, w.tiles_per_chunk); return true;
    case 22: hipLaunchKernelGGL((k_wgrad_lds<2, 2>), grid, dim3(192), lds, st, a, w.tiles_per_chunk); return true;
    case 42: hipLaunchKernelGGL((k_wgrad_lds<4, 2>), grid, dim3(192), lds, st, a, w.tiles_per_chunk); return true;
    case 81: hipLaunchKernelGGL((k_wgrad_lds<8, 1>), grid, dim3(192), lds, st, a, w.tiles_per_chunk); return true;
    default: return false;
    }
}

void unet_reduce_chunks(const float* partial, int n_chunks, int n, float* out, int add, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_chunks, dim3(nb(n, 16)), dim3(256), 0, st, partial, n_chunks, n, out, add);
}

int unet_colsum_blocks(int P) { return (P + COLSUM_ROWS - 1) / COLSUM_ROWS; }

void unet_colsum(const uint16_t* g, int P, int C, float* partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_colsum, dim3(unet_colsum_blocks(P)), dim3(256), 0, st, g, P, C, partial);
}

void unet_reduce_blocks(const float* partial, int n_blocks, int n, float* out, int add, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_blocks, dim3(n), dim3(256), 0, st, partial, n_blocks, n, out, add);
}

void unet_pool2(const uint16_t* in, int N, int H, int W, int C, uint16_t* out, hipStream_t st)
{
    size_t n = (size_t)N * (H / 2) * (W / 2) * (C / 8);
    hipLaunchKernelGGL(k_pool2, dim3(nb(n, 256)), dim3(256), 0, st, in, N, H, W, C, out);
}

void unet_up2_concat(const uint16_t* a, const uint16_t* skip, int N, int H, int W, int Ca, int Cs, uint16_t* out,
                     hipStream_t st)
{
    size_t n = (size_t)N * H * W * ((Ca + Cs) / 8);
    hipLaunchKernelGGL(k_up2_concat, dim3(nb(n, 256)), dim3(256), 0, st, a, skip, N, H, W, Ca, Cs, out);
}

void unet_up_back_mask(const uint16_t* g, int N, int H2, int W2, int Ctot, int c0, int C, const uint16_t* mask,
                       uint16_t* out, hipStream_t st)
{
    size_t n = (size_t)N * (H2 / 2) * (W2 / 2) * (C / 8);
    hipLaunchKernelGGL(k_up_back_mask, dim3(nb(n, 256)), dim3(256), 0, st, g, N, H2, W2, Ctot, c0, C, mask, out);
}

void unet_pool_back_add_mask(const uint16_t* gpool, const uint16_t* gcat, int N, int H, int W, int C, int Ctot, int c0,
                             const uint16_t* mask, uint16_t* out, hipStream_t st)
{
    size_t n = (size_t)N * H * W * (C / 8);
    hipLaunchKernelGGL(k_pool_back_add_mask, dim3(nb(n, 256)), dim3(256), 0, st, gpool, gcat, N, H, W, C, Ctot, c0,
                       mask, out);
}

void unet_head(const uint16_t* d1, const float* wh, const float* bh, int P, float* y, hipStream_t st)
{
    hipLaunchKernelGGL(k_head, dim3(nb(P, 256)), dim3(256), 0, st, d1, wh, bh, P, y);
}

void unet_loss(const float* y, const float* t, const float* m, int P, int chunk, float* partial, float* sums,
               hipStream_t st)
{
    int chunks = (P + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_loss_partials, dim3(chunks), dim3(256), 0, st, y, t, m, P, chunk, partial);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, partial, chunks, sums);
}

int unet_head_blocks(int P) { return (P + 255) / 256; }

void unet_head_back(const uint16_t* d1, const float* y, const float* t, const float* m, const float* sums,
                    const float* wh, int P, uint16_t* gpre, float* partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_head_back, dim3(unet_head_blocks(P)), dim3(256), 0, st, d1, y, t, m, sums, wh, P, gpre,
                       partial);
}

void unet_weights_bf16(const float* w, int Cout, int Cin, uint16_t* wf, uint16_t* wb, hipStream_t st)
{
    int n = Cout * 9 * Cin;
    hipLaunchKernelGGL(k_weights_bf16, dim3(nb(n, 256)), dim3(256), 0, st, w, Cout, Cin, wf, wb);
}

void unet_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps, float c1,
               float c2, hipStream_t st)
{
    hipLaunchKernelGGL(k_adam, dim3(nb(n, 256)), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

void unet_conv3x3_f32(const ConvArgsF32& a, hipStream_t st)
{
    const int nt = a.Cout / 16, cc = a.Cin % 32 == 0 ? 32 : 8;
    const size_t tiles = (size_t)a.N * ((a.H + 3) / 4) * ((a.W + 15) / 16);
    const size_t lds = (size_t)6 * 18 * (cc + 1) * 4;
    switch (nt * 100 + cc) {
    case 208: hipLaunchKernelGGL((k_conv_f32<2, 8>), dim3((unsigned)tiles), dim3(256), lds, st, a); break;
    case 232: hipLaunchKernelGGL((k_conv_f32<2, 32>), dim3((unsigned)tiles), dim3(256), lds, st, a); break;
    case 432: hipLaunchKernelGGL((k_conv_f32<4, 32>), dim3((unsigned)tiles), dim3(256), lds, st, a); break;
    case 832: hipLaunchKernelGGL((k_conv_f32<8, 32>), dim3((unsigned)tiles), dim3(256), lds, st, a); break;
    default: break;   // channel counts of this network only
    }
}

void unet_pool2_f32(const float* in, int N, int H, int W, int C, float* out, hipStream_t st)
{
    size_t n = (size_t)N * (H / 2) * (W / 2) * (C / 4);
    hipLaunchKernelGGL(k_pool2_f32, dim3(nb(n, 256)), dim3(256), 0, st, in, N, H, W, C, out);
}

void unet_head_f32(const float* d1, const float* wh, const float* bh, int P, float* y, hipStream_t st)
{
    hipLaunchKernelGGL(k_head_f32, dim3(nb(P, 256)), dim3(256), 0, st, d1, wh, bh, P, y);
}

void unet_weights_f32t(const float* w, int Cout, int Cin, float* wt, hipStream_t st)
{
    int n = Cout * 9 * Cin;
    hipLaunchKernelGGL(k_weights_f32t, dim3(nb(n, 256)), dim3(256), 0, st, w, Cout, Cin, wt);
}

void unet_fill_f32(float* p, float v, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_f32, dim3(nb(n, 256)), dim3(256), 0, st, p, v, n);
}
