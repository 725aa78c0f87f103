// Host driver of the U-Net shadow denoiser: parameters (FP32 master + BF16 copies), Adam state,
// activation/gradient workspace, forward, one training step, checkpoints.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <random>
#include <vector>

#include "../../include/raycast.h"
#include "rc_objects.h"
#include "rc_unet.h"

namespace {

struct LayerDef {
    int cin, cout;
};
// e1a e1b e2a e2b bna bnb d2a d2b d1a d1b
const LayerDef LAYERS[10] = {{8, 32}, {32, 32}, {32, 64}, {64, 64}, {64, 128},
                             {128, 128}, {192, 64}, {64, 64}, {96, 32}, {32, 32}};
enum { E1A, E1B, E2A, E2B, BNA, BNB, D2A, D2B, D1A, D1B, N_LAYERS };

size_t layer_w(int l) { return (size_t)LAYERS[l].cout * 9 * LAYERS[l].cin; }

const uint32_t CKPT_MAGIC = 0x4E444352u;   // "RCDN"
const uint32_t CKPT_VERSION = 1;

uint32_t crc32_update(uint32_t crc, const void* data, size_t n)
{
    const uint8_t* p = static_cast<const uint8_t*>(data);
    crc = ~crc;
    for (size_t i = 0; i < n; ++i) {
        crc ^= p[i];
        for (int k = 0; k < 8; ++k) crc = (crc >> 1) ^ (0xEDB88320u & (0u - (crc & 1u)));
    }
    return ~crc;
}

int hip_err(hipError_t e) { return e == hipErrorOutOfMemory ? RC_ERR_OUT_OF_MEMORY : RC_ERR_HIP; }

#define DN_HIP(call)                              \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) return hip_err(e_); \
    } while (0)

}  // namespace

struct rc_denoiser {
    int device = 0;
    size_t n_params = 0;
    size_t off_w[N_LAYERS + 1], off_b[N_LAYERS + 1];   // [N_LAYERS] = head
    uint64_t step = 0;
    float* d_w = nullptr;
    float* d_g = nullptr;
    float* d_m = nullptr;
    float* d_v = nullptr;
    uint16_t* d_wbf = nullptr;   // forward copies of all conv layers, concatenated
    uint16_t* d_wfl = nullptr;   // flipped / transposed copies
    size_t off_bf[N_LAYERS];
    // workspace
    int wn = 0, wh = 0, ww = 0;
    uint16_t* act = nullptr;
    uint16_t* grad = nullptr;
    float* d_y = nullptr;
    float* d_partial = nullptr;
    size_t partial_cap = 0;
    float* d_sums = nullptr;
    // activation offsets (elements) within act / grad
    size_t a_e1a, a_e1b, a_p1, a_e2a, a_e2b, a_p2, a_bna, a_bnb, a_u2, a_d2a, a_d2b, a_u1, a_d1a, a_d1b, a_total;
    size_t g_d1b, g_d1a, g_u1, g_d2b, g_d2a, g_u2, g_bnb, g_bna, g_p2, g_e2b, g_e2a, g_p1, g_e1b, g_e1a, g_total;
    // FP32 copy of the forward pass: transposed FP32 weights and an FP32 activation workspace
    float* d_wt32 = nullptr;
    float* act32 = nullptr;
    int fn = 0, fh = 0, fw = 0;
    size_t f_e1a, f_e1b, f_p1, f_e2a, f_e2b, f_p2, f_bna, f_bnb, f_d2a, f_d2b, f_d1a, f_d1b, f_y, f_total;
};

namespace {

hipStream_t ctx_stream(rc_ctx* c) { return c->stream; }
int ctx_device(rc_ctx* c) { return c->device; }

int refresh_bf16(rc_denoiser* d, hipStream_t st)
{
    for (int l = 0; l < N_LAYERS; ++l)
        unet_weights_bf16(d->d_w + d->off_w[l], LAYERS[l].cout, LAYERS[l].cin, d->d_wbf + d->off_bf[l],
                          d->d_wfl + d->off_bf[l], st);
    DN_HIP(hipGetLastError());
    return RC_OK;
}

int ensure_workspace(rc_denoiser* d, int n, int h, int w)
{
    if (d->wn == n && d->wh == h && d->ww == w && d->act) return RC_OK;
    hipFree(d->act);
    hipFree(d->grad);
    hipFree(d->d_y);
    d->act = d->grad = nullptr;
    d->d_y = nullptr;
    size_t P = (size_t)n * h * w, P2 = P / 4, P4 = P / 16;
    size_t o = 0;
    auto take = [&](size_t elems) { size_t r = o; o += (elems + 63) & ~size_t(63); return r; };
    d->a_e1a = take(P * 32); d->a_e1b = take(P * 32); d->a_p1 = take(P2 * 32);
    d->a_e2a = take(P2 * 64); d->a_e2b = take(P2 * 64); d->a_p2 = take(P4 * 64);
    d->a_bna = take(P4 * 128); d->a_bnb = take(P4 * 128); d->a_u2 = take(P2 * 192);
    d->a_d2a = take(P2 * 64); d->a_d2b = take(P2 * 64); d->a_u1 = take(P * 96);
    d->a_d1a = take(P * 32); d->a_d1b = take(P * 32);
    d->a_total = o;
    o = 0;
    d->g_d1b = take(P * 32); d->g_d1a = take(P * 32); d->g_u1 = take(P * 96);
    d->g_d2b = take(P2 * 64); d->g_d2a = take(P2 * 64); d->g_u2 = take(P2 * 192);
    d->g_bnb = take(P4 * 128); d->g_bna = take(P4 * 128); d->g_p2 = take(P4 * 64);
    d->g_e2b = take(P2 * 64); d->g_e2a = take(P2 * 64); d->g_p1 = take(P2 * 32);
    d->g_e1b = take(P * 32); d->g_e1a = take(P * 32);
    d->g_total = o;
    DN_HIP(hipMalloc(reinterpret_cast<void**>(&d->act), d->a_total * 2));
    DN_HIP(hipMalloc(reinterpret_cast<void**>(&d->grad), d->g_total * 2));
    DN_HIP(hipMalloc(reinterpret_cast<void**>(&d->d_y), P * 4));
    d->wn = n; d->wh = h; d->ww = w;
    return RC_OK;
}

int ensure_workspace_f32(rc_denoiser* d, int n, int h, int w)
{
    if (!d->d_wt32) DN_HIP(hipMalloc(reinterpret_cast<void**>(&d->d_wt32), d->off_bf[N_LAYERS - 1] * 4 +
                                                                               layer_w(N_LAYERS - 1) * 4));
    if (d->fn == n && d->fh == h && d->fw == w && d->act32) return RC_OK;
    hipFree(d->act32);
    d->act32 = nullptr;
    size_t P = (size_t)n * h * w, P2 = P / 4, P4 = P / 16;
    size_t o = 0;
    auto take = [&](size_t elems) { size_t r = o; o += (elems + 63) & ~size_t(63); return r; };
    d->f_e1a = take(P * 32); d->f_e1b = take(P * 32); d->f_p1 = take(P2 * 32);
    d->f_e2a = take(P2 * 64); d->f_e2b = take(P2 * 64); d->f_p2 = take(P4 * 64);
    d->f_bna = take(P4 * 128); d->f_bnb = take(P4 * 128);
    d->f_d2a = take(P2 * 64); d->f_d2b = take(P2 * 64); d->f_d1a = take(P * 32); d->f_d1b = take(P * 32);
    d->f_y = take(P);
    d->f_total = o;
    DN_HIP(hipMalloc(reinterpret_cast<void**>(&d->act32), d->f_total * 4));
    d->fn = n; d->fh = h; d->fw = w;
    return RC_OK;
}

int ensure_partial(rc_denoiser* d, size_t floats)
{
    if (floats <= d->partial_cap) return RC_OK;
    hipFree(d->d_partial);
    d->d_partial = nullptr;
    d->partial_cap = 0;
    DN_HIP(hipMalloc(reinterpret_cast<void**>(&d->d_partial), floats * 4));
    d->partial_cap = floats;
    return RC_OK;
}

int chunk_for(size_t P)
{
    size_t c = (P + 63) / 64;             // at most 64 split-K chunks
    c = std::max<size_t>(c, 1024);
    return (int)((c + 31) & ~size_t(31));
}

// layer l; with `skip`, the input is [2x nearest-upsampled `in` (Ca channels), skip] read directly
// pool_out: also write the 2x2 average pool of the output; head_out: write the network's head of the output
// (layer D1B) instead of the output
void conv(rc_denoiser* d, const uint16_t* in, int n, int h, int w, int l, uint16_t* out, hipStream_t st,
          const uint16_t* skip = nullptr, int Ca = 0, uint16_t* pool_out = nullptr, float* head_out = nullptr)
{
    ConvArgs a = {};
    a.in = in; a.in2 = skip; a.Ca = Ca;
    a.N = n; a.H = h; a.W = w; a.Cin = LAYERS[l].cin;
    a.wt = d->d_wbf + d->off_bf[l];
    a.bias = d->d_w + d->off_b[l];
    a.mask = nullptr;
    a.out = out;
    a.Cout = LAYERS[l].cout;
    a.relu = 1;
    a.pool_out = pool_out;
    if (head_out) {
        a.head_w = d->d_w + d->off_w[N_LAYERS];
        a.head_b = d->d_w + d->off_b[N_LAYERS];
        a.head_out = head_out;
        a.out = nullptr;
    }
    unet_conv3x3(a, st);
}

// gradient w.r.t. the input of layer l from the pre-activation gradient g (masked by `mask` if given)
void conv_back_data(rc_denoiser* d, const uint16_t* g, int n, int h, int w, int l, const uint16_t* mask,
                    uint16_t* out, hipStream_t st)
{
    ConvArgs a = {};
    a.in = g; a.N = n; a.H = h; a.W = w; a.Cin = LAYERS[l].cout;
    a.wt = d->d_wfl + d->off_bf[l];
    a.bias = nullptr;
    a.mask = mask;
    a.out = out;
    a.Cout = LAYERS[l].cin;
    a.relu = 0;
    unet_conv3x3(a, st);
}

// dW and db of layer l from its input x and pre-activation gradient g, written into d_g
void conv_back_weights(rc_denoiser* d, const uint16_t* x, const uint16_t* g, int n, int h, int w, int l, hipStream_t st)
{
    size_t P = (size_t)n * h * w;
    int chunk = chunk_for(P);
    int chunks = unet_wgrad_chunks(P, chunk);
    WgradArgs a;
    a.x = x; a.g = g; a.N = n; a.H = h; a.W = w; a.Cin = LAYERS[l].cin; a.Cout = LAYERS[l].cout;
    a.chunk = chunk;
    a.partial = d->d_partial;
    if (unet_wgrad_lds(a, st)) {
        unet_reduce_chunks(d->d_partial, unet_wgrad_lds_chunks(a), (int)layer_w(l), d->d_g + d->off_w[l], 0, st);
    } else {
        unet_wgrad(a, st);
        unet_reduce_chunks(d->d_partial, chunks, (int)layer_w(l), d->d_g + d->off_w[l], 0, st);
    }
    unet_colsum(g, (int)P, LAYERS[l].cout, d->d_partial, st);
    unet_reduce_blocks(d->d_partial, unet_colsum_blocks((int)P), LAYERS[l].cout, d->d_g + d->off_b[l], 0, st);
}

// keep_concat: also materialise the decoder's concatenated inputs (the weight gradients read them).
// y_out (inference): the head is computed in the last convolution's epilogue and written there, and the
// last layer's activations are not stored; otherwise they are, and the head writes d_y.
int forward(rc_denoiser* d, const uint16_t* x, int n, int h, int w, hipStream_t st, bool keep_concat,
            float* y_out = nullptr)
{
    int st_ = ensure_workspace(d, n, h, w);
    if (st_ != RC_OK) return st_;
    uint16_t* A = d->act;
    int h2 = h / 2, w2 = w / 2, h4 = h / 4, w4 = w / 4;
    conv(d, x, n, h, w, E1A, A + d->a_e1a, st);
    conv(d, A + d->a_e1a, n, h, w, E1B, A + d->a_e1b, st, nullptr, 0, A + d->a_p1);
    conv(d, A + d->a_p1, n, h2, w2, E2A, A + d->a_e2a, st);
    conv(d, A + d->a_e2a, n, h2, w2, E2B, A + d->a_e2b, st, nullptr, 0, A + d->a_p2);
    conv(d, A + d->a_p2, n, h4, w4, BNA, A + d->a_bna, st);
    conv(d, A + d->a_bna, n, h4, w4, BNB, A + d->a_bnb, st);
    if (keep_concat) unet_up2_concat(A + d->a_bnb, A + d->a_e2b, n, h2, w2, 128, 64, A + d->a_u2, st);
    conv(d, A + d->a_bnb, n, h2, w2, D2A, A + d->a_d2a, st, A + d->a_e2b, 128);
    conv(d, A + d->a_d2a, n, h2, w2, D2B, A + d->a_d2b, st);
    if (keep_concat) unet_up2_concat(A + d->a_d2b, A + d->a_e1b, n, h, w, 64, 32, A + d->a_u1, st);
    conv(d, A + d->a_d2b, n, h, w, D1A, A + d->a_d1a, st, A + d->a_e1b, 64);
    if (y_out) {
        conv(d, A + d->a_d1a, n, h, w, D1B, nullptr, st, nullptr, 0, nullptr, y_out);
    } else {
        conv(d, A + d->a_d1a, n, h, w, D1B, A + d->a_d1b, st);
        unet_head(A + d->a_d1b, d->d_w + d->off_w[N_LAYERS], d->d_w + d->off_b[N_LAYERS], n * h * w, d->d_y, st);
    }
    DN_HIP(hipGetLastError());
    return RC_OK;
}

// layer l in FP32 (input `in` float, or the BF16 features for the first layer)
void conv_f32(rc_denoiser* d, const void* in, bool in_bf16, int n, int h, int w, int l, float* out, hipStream_t st,
              const float* skip = nullptr, int Ca = 0)
{
    ConvArgsF32 a = {};
    a.in = in; a.in_bf16 = in_bf16 ? 1 : 0; a.in2 = skip; a.Ca = Ca;
    a.N = n; a.H = h; a.W = w; a.Cin = LAYERS[l].cin;
    a.wt = d->d_wt32 + d->off_bf[l];
    a.bias = d->d_w + d->off_b[l];
    a.out = out;
    a.Cout = LAYERS[l].cout;
    unet_conv3x3_f32(a, st);
}

int forward_f32(rc_denoiser* d, const uint16_t* x, int n, int h, int w, hipStream_t st)
{
    int st_ = ensure_workspace_f32(d, n, h, w);
    if (st_ != RC_OK) return st_;
    for (int l = 0; l < N_LAYERS; ++l)
        unet_weights_f32t(d->d_w + d->off_w[l], LAYERS[l].cout, LAYERS[l].cin, d->d_wt32 + d->off_bf[l], st);
    float* F = d->act32;
    int h2 = h / 2, w2 = w / 2, h4 = h / 4, w4 = w / 4;
    conv_f32(d, x, true, n, h, w, E1A, F + d->f_e1a, st);
    conv_f32(d, F + d->f_e1a, false, n, h, w, E1B, F + d->f_e1b, st);
    unet_pool2_f32(F + d->f_e1b, n, h, w, 32, F + d->f_p1, st);
    conv_f32(d, F + d->f_p1, false, n, h2, w2, E2A, F + d->f_e2a, st);
    conv_f32(d, F + d->f_e2a, false, n, h2, w2, E2B, F + d->f_e2b, st);
    unet_pool2_f32(F + d->f_e2b, n, h2, w2, 64, F + d->f_p2, st);
    conv_f32(d, F + d->f_p2, false, n, h4, w4, BNA, F + d->f_bna, st);
    conv_f32(d, F + d->f_bna, false, n, h4, w4, BNB, F + d->f_bnb, st);
    conv_f32(d, F + d->f_bnb, false, n, h2, w2, D2A, F + d->f_d2a, st, F + d->f_e2b, 128);
    conv_f32(d, F + d->f_d2a, false, n, h2, w2, D2B, F + d->f_d2b, st);
    conv_f32(d, F + d->f_d2b, false, n, h, w, D1A, F + d->f_d1a, st, F + d->f_e1b, 64);
    conv_f32(d, F + d->f_d1a, false, n, h, w, D1B, F + d->f_d1b, st);
    unet_head_f32(F + d->f_d1b, d->d_w + d->off_w[N_LAYERS], d->d_w + d->off_b[N_LAYERS], n * h * w,
                  F + d->f_y, st);
    DN_HIP(hipGetLastError());
    return RC_OK;
}

int backward(rc_denoiser* d, const uint16_t* x, const float* t, const float* m, int n, int h, int w, hipStream_t st)
{
    uint16_t* A = d->act;
    uint16_t* G = d->grad;
    size_t P = (size_t)n * h * w;
    int h2 = h / 2, w2 = w / 2, h4 = h / 4, w4 = w / 4;
    int chunk = chunk_for(P);
    int chunks = unet_wgrad_chunks(P, chunk);
    size_t need = 0;
    for (int l = 0; l < N_LAYERS; ++l) {
        need = std::max(need, (size_t)chunks * layer_w(l));
        const int s = (l == E1A || l == E1B || l == D1A || l == D1B) ? 1 : (l == BNA || l == BNB ? 4 : 2);
        WgradArgs q = {};
        q.N = n; q.H = h / s; q.W = w / s; q.Cin = LAYERS[l].cin; q.Cout = LAYERS[l].cout;
        need = std::max(need, (size_t)unet_wgrad_lds_chunks(q) * layer_w(l));
    }
    need = std::max(need, (size_t)chunks * 64);
    need = std::max(need, (size_t)unet_colsum_blocks((int)P) * 128);
    need = std::max(need, (size_t)unet_head_blocks((int)P) * 33);
    int st_ = ensure_partial(d, need);
    if (st_ != RC_OK) return st_;
    if (!d->d_sums) DN_HIP(hipMalloc(reinterpret_cast<void**>(&d->d_sums), 64));
    // loss and head
    unet_loss(d->d_y, t, m, (int)P, chunk, d->d_partial, d->d_sums, st);
    unet_head_back(A + d->a_d1b, d->d_y, t, m, d->d_sums, d->d_w + d->off_w[N_LAYERS], (int)P, G + d->g_d1b,
                   d->d_partial, st);
    unet_reduce_blocks(d->d_partial, unet_head_blocks((int)P), 33, d->d_g + d->off_w[N_LAYERS], 0, st);   // head.w, head.b
    // decoder level 1
    conv_back_weights(d, A + d->a_d1a, G + d->g_d1b, n, h, w, D1B, st);
    conv_back_data(d, G + d->g_d1b, n, h, w, D1B, A + d->a_d1a, G + d->g_d1a, st);
    conv_back_weights(d, A + d->a_u1, G + d->g_d1a, n, h, w, D1A, st);
    conv_back_data(d, G + d->g_d1a, n, h, w, D1A, nullptr, G + d->g_u1, st);
    unet_up_back_mask(G + d->g_u1, n, h, w, 96, 0, 64, A + d->a_d2b, G + d->g_d2b, st);
    // decoder level 2
    conv_back_weights(d, A + d->a_d2a, G + d->g_d2b, n, h2, w2, D2B, st);
    conv_back_data(d, G + d->g_d2b, n, h2, w2, D2B, A + d->a_d2a, G + d->g_d2a, st);
    conv_back_weights(d, A + d->a_u2, G + d->g_d2a, n, h2, w2, D2A, st);
    conv_back_data(d, G + d->g_d2a, n, h2, w2, D2A, nullptr, G + d->g_u2, st);
    unet_up_back_mask(G + d->g_u2, n, h2, w2, 192, 0, 128, A + d->a_bnb, G + d->g_bnb, st);
    // bottleneck
    conv_back_weights(d, A + d->a_bna, G + d->g_bnb, n, h4, w4, BNB, st);
    conv_back_data(d, G + d->g_bnb, n, h4, w4, BNB, A + d->a_bna, G + d->g_bna, st);
    conv_back_weights(d, A + d->a_p2, G + d->g_bna, n, h4, w4, BNA, st);
    conv_back_data(d, G + d->g_bna, n, h4, w4, BNA, nullptr, G + d->g_p2, st);
    unet_pool_back_add_mask(G + d->g_p2, G + d->g_u2, n, h2, w2, 64, 192, 128, A + d->a_e2b, G + d->g_e2b, st);
    // encoder level 2
    conv_back_weights(d, A + d->a_e2a, G + d->g_e2b, n, h2, w2, E2B, st);
    conv_back_data(d, G + d->g_e2b, n, h2, w2, E2B, A + d->a_e2a, G + d->g_e2a, st);
    conv_back_weights(d, A + d->a_p1, G + d->g_e2a, n, h2, w2, E2A, st);
    conv_back_data(d, G + d->g_e2a, n, h2, w2, E2A, nullptr, G + d->g_p1, st);
    unet_pool_back_add_mask(G + d->g_p1, G + d->g_u1, n, h, w, 32, 96, 64, A + d->a_e1b, G + d->g_e1b, st);
    // encoder level 1
    conv_back_weights(d, A + d->a_e1a, G + d->g_e1b, n, h, w, E1B, st);
    conv_back_data(d, G + d->g_e1b, n, h, w, E1B, A + d->a_e1a, G + d->g_e1a, st);
    conv_back_weights(d, x, G + d->g_e1a, n, h, w, E1A, st);
    DN_HIP(hipGetLastError());
    return RC_OK;
}

void normal_fill(std::vector<float>& v, size_t off, size_t n, double sd, std::mt19937_64& rng)
{
    // Box-Muller on 53-bit uniforms
    for (size_t i = 0; i < n; i += 2) {
        double u1 = ((rng() >> 11) + 1.0) * 0x1p-53, u2 = (rng() >> 11) * 0x1p-53;
        double r = sqrt(-2.0 * log(u1));
        v[off + i] = (float)(sd * r * cos(6.283185307179586 * u2));
        if (i + 1 < n) v[off + i + 1] = (float)(sd * r * sin(6.283185307179586 * u2));
    }
}

bool dims_ok(uint32_t n, uint32_t h, uint32_t w)
{
    return n > 0 && h >= 4 && w >= 4 && h % 4 == 0 && w % 4 == 0 && (uint64_t)n * h * w <= (1ull << 28);
}

}  // namespace

extern "C" {

int rc_denoiser_n_params(void)
{
    size_t n = 0;
    for (int l = 0; l < N_LAYERS; ++l) n += layer_w(l) + LAYERS[l].cout;
    return (int)(n + 33);
}

int rc_denoiser_create(rc_ctx* c, uint32_t seed, rc_denoiser** out)
{
    if (!c || !out) return RC_ERR_INVALID_ARG;
    *out = nullptr;
    DN_HIP(hipSetDevice(ctx_device(c)));
    rc_denoiser* d = new (std::nothrow) rc_denoiser();
    if (!d) return RC_ERR_OUT_OF_MEMORY;
    d->device = ctx_device(c);
    size_t o = 0, ob = 0;
    for (int l = 0; l < N_LAYERS; ++l) {
        d->off_w[l] = o; o += layer_w(l);
        d->off_b[l] = o; o += LAYERS[l].cout;
        d->off_bf[l] = ob; ob += layer_w(l);
    }
    d->off_w[N_LAYERS] = o; o += 32;
    d->off_b[N_LAYERS] = o; o += 1;
    d->n_params = o;
    // He-normal conv weights (fan-in 9 Cin), zero biases, head N(0, 1/32)
    std::vector<float> w(o, 0.0f);
    std::mt19937_64 rng(0x9E3779B97F4A7C15ull ^ seed);
    for (int l = 0; l < N_LAYERS; ++l) normal_fill(w, d->off_w[l], layer_w(l), sqrt(2.0 / (9.0 * LAYERS[l].cin)), rng);
    normal_fill(w, d->off_w[N_LAYERS], 32, sqrt(1.0 / 32.0), rng);
    int st = RC_OK;
    auto alloc = [&](void** p, size_t bytes) { if (st == RC_OK && hipMalloc(p, bytes) != hipSuccess) st = RC_ERR_OUT_OF_MEMORY; };
    alloc(reinterpret_cast<void**>(&d->d_w), o * 4);
    alloc(reinterpret_cast<void**>(&d->d_g), o * 4);
    alloc(reinterpret_cast<void**>(&d->d_m), o * 4);
    alloc(reinterpret_cast<void**>(&d->d_v), o * 4);
    alloc(reinterpret_cast<void**>(&d->d_wbf), ob * 2);
    alloc(reinterpret_cast<void**>(&d->d_wfl), ob * 2);
    if (st == RC_OK && hipMemcpy(d->d_w, w.data(), o * 4, hipMemcpyHostToDevice) != hipSuccess) st = RC_ERR_HIP;
    if (st == RC_OK) {
        hipStream_t s = ctx_stream(c);
        unet_fill_f32(d->d_g, 0.0f, o, s);
        unet_fill_f32(d->d_m, 0.0f, o, s);
        unet_fill_f32(d->d_v, 0.0f, o, s);
        st = refresh_bf16(d, s);
        if (st == RC_OK && hipStreamSynchronize(s) != hipSuccess) st = RC_ERR_HIP;
    }
    if (st != RC_OK) { rc_denoiser_destroy(c, d); return st; }
    *out = d;
    return RC_OK;
}

int rc_denoiser_destroy(rc_ctx* c, rc_denoiser* d)
{
    if (!c || !d) return RC_ERR_INVALID_ARG;
    hipSetDevice(d->device);
    hipStreamSynchronize(ctx_stream(c));
    hipFree(d->d_w); hipFree(d->d_g); hipFree(d->d_m); hipFree(d->d_v);
    hipFree(d->d_wbf); hipFree(d->d_wfl);
    hipFree(d->act); hipFree(d->grad); hipFree(d->d_y); hipFree(d->d_partial); hipFree(d->d_sums);
    hipFree(d->d_wt32); hipFree(d->act32);
    delete d;
    return RC_OK;
}

int rc_denoiser_get_params(rc_ctx* c, const rc_denoiser* d, float* out)
{
    if (!c || !d || !out) return RC_ERR_INVALID_ARG;
    DN_HIP(hipSetDevice(d->device));
    DN_HIP(hipStreamSynchronize(ctx_stream(c)));
    DN_HIP(hipMemcpy(out, d->d_w, d->n_params * 4, hipMemcpyDeviceToHost));
    return RC_OK;
}

int rc_denoiser_get_grads(rc_ctx* c, const rc_denoiser* d, float* out)
{
    if (!c || !d || !out) return RC_ERR_INVALID_ARG;
    DN_HIP(hipSetDevice(d->device));
    DN_HIP(hipStreamSynchronize(ctx_stream(c)));
    DN_HIP(hipMemcpy(out, d->d_g, d->n_params * 4, hipMemcpyDeviceToHost));
    return RC_OK;
}

int rc_denoiser_set_params(rc_ctx* c, rc_denoiser* d, const float* in)
{
    if (!c || !d || !in) return RC_ERR_INVALID_ARG;
    for (size_t i = 0; i < d->n_params; ++i)
        if (!isfinite(in[i])) return RC_ERR_INVALID_VALUE;
    DN_HIP(hipSetDevice(d->device));
    hipStream_t s = ctx_stream(c);
    DN_HIP(hipStreamSynchronize(s));
    DN_HIP(hipMemcpy(d->d_w, in, d->n_params * 4, hipMemcpyHostToDevice));
    unet_fill_f32(d->d_m, 0.0f, d->n_params, s);
    unet_fill_f32(d->d_v, 0.0f, d->n_params, s);
    d->step = 0;
    return refresh_bf16(d, s);
}

int rc_denoiser_infer(rc_ctx* c, rc_denoiser* d, const uint16_t* d_feat, uint32_t n, uint32_t h, uint32_t w, float* d_out)
{
    if (!c || !d || !d_feat || !d_out) return RC_ERR_INVALID_ARG;
    if (!dims_ok(n, h, w)) return RC_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(d_feat) & 15u) return RC_ERR_INVALID_ARG;
    DN_HIP(hipSetDevice(d->device));
    hipStream_t s = ctx_stream(c);
    if (reinterpret_cast<uintptr_t>(d_out) & 3u) return RC_ERR_INVALID_ARG;
    return forward(d, d_feat, (int)n, (int)h, (int)w, s, false, d_out);
}

int rc_denoiser_infer_fp32(rc_ctx* c, rc_denoiser* d, const uint16_t* d_feat, uint32_t n, uint32_t h, uint32_t w,
                           float* d_out)
{
    if (!c || !d || !d_feat || !d_out) return RC_ERR_INVALID_ARG;
    if (!dims_ok(n, h, w)) return RC_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(d_feat) & 15u) return RC_ERR_INVALID_ARG;
    DN_HIP(hipSetDevice(d->device));
    hipStream_t s = ctx_stream(c);
    int st = forward_f32(d, d_feat, (int)n, (int)h, (int)w, s);
    if (st != RC_OK) return st;
    DN_HIP(hipMemcpyAsync(d_out, d->act32 + d->f_y, (size_t)n * h * w * 4, hipMemcpyDeviceToDevice, s));
    return RC_OK;
}

int rc_denoiser_train_step(rc_ctx* c, rc_denoiser* d, const uint16_t* d_feat, const float* d_target,
                           const float* d_mask, uint32_t n, uint32_t h, uint32_t w, float lr, float* loss_out)
{
    if (!c || !d || !d_feat || !d_target || !d_mask) return RC_ERR_INVALID_ARG;
    if (!dims_ok(n, h, w) || !(lr >= 0.0f) || !isfinite(lr)) return RC_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(d_feat) & 15u) return RC_ERR_INVALID_ARG;
    DN_HIP(hipSetDevice(d->device));
    hipStream_t s = ctx_stream(c);
    int st = forward(d, d_feat, (int)n, (int)h, (int)w, s, true);
    if (st == RC_OK) st = backward(d, d_feat, d_target, d_mask, (int)n, (int)h, (int)w, s);
    if (st != RC_OK) return st;
    d->step++;
    const double b1 = 0.9, b2 = 0.999;
    float c1 = (float)(1.0 - pow(b1, (double)d->step)), c2 = (float)(1.0 - pow(b2, (double)d->step));
    unet_adam(d->d_w, d->d_g, d->d_m, d->d_v, (int)d->n_params, lr, (float)b1, (float)b2, 1e-8f, c1, c2, s);
    st = refresh_bf16(d, s);
    if (st != RC_OK) return st;
    if (loss_out) {
        float sums[2];
        DN_HIP(hipMemcpyAsync(sums, d->d_sums, 8, hipMemcpyDeviceToHost, s));
        DN_HIP(hipStreamSynchronize(s));
        *loss_out = sums[1];
    }
    return RC_OK;
}

int rc_denoiser_save(rc_ctx* c, const rc_denoiser* d, const char* path)
{
    if (!c || !d || !path) return RC_ERR_INVALID_ARG;
    size_t n = d->n_params;
    std::vector<float> buf(3 * n);
    DN_HIP(hipSetDevice(d->device));
    DN_HIP(hipStreamSynchronize(ctx_stream(c)));
    DN_HIP(hipMemcpy(buf.data(), d->d_w, n * 4, hipMemcpyDeviceToHost));
    DN_HIP(hipMemcpy(buf.data() + n, d->d_m, n * 4, hipMemcpyDeviceToHost));
    DN_HIP(hipMemcpy(buf.data() + 2 * n, d->d_v, n * 4, hipMemcpyDeviceToHost));
    uint32_t hdr[6] = {CKPT_MAGIC, CKPT_VERSION, (uint32_t)n, (uint32_t)(d->step & 0xFFFFFFFFu),
                       (uint32_t)(d->step >> 32), 0u};
    uint32_t crc = crc32_update(0, hdr, sizeof(hdr));
    crc = crc32_update(crc, buf.data(), buf.size() * 4);
    FILE* f = fopen(path, "wb");
    if (!f) return RC_ERR_INVALID_ARG;
    bool ok = fwrite(hdr, sizeof(hdr), 1, f) == 1 && fwrite(buf.data(), 4, buf.size(), f) == buf.size() &&
              fwrite(&crc, 4, 1, f) == 1;
    ok = (fclose(f) == 0) && ok;
    return ok ? RC_OK : RC_ERR_INVALID_ARG;
}

int rc_denoiser_load(rc_ctx* c, rc_denoiser* d, const char* path)
{
    if (!c || !d || !path) return RC_ERR_INVALID_ARG;
    FILE* f = fopen(path, "rb");
    if (!f) return RC_ERR_BAD_CHECKPOINT;
    uint32_t hdr[6];
    size_t n = d->n_params;
    std::vector<float> buf(3 * n);
    uint32_t crc_file = 0;
    bool ok = fread(hdr, sizeof(hdr), 1, f) == 1;
    ok = ok && hdr[0] == CKPT_MAGIC && hdr[1] == CKPT_VERSION && hdr[2] == (uint32_t)n;
    ok = ok && fread(buf.data(), 4, buf.size(), f) == buf.size() && fread(&crc_file, 4, 1, f) == 1;
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;   // no trailing bytes
    fclose(f);
    if (!ok) return RC_ERR_BAD_CHECKPOINT;
    uint32_t crc = crc32_update(0, hdr, sizeof(hdr));
    crc = crc32_update(crc, buf.data(), buf.size() * 4);
    if (crc != crc_file) return RC_ERR_BAD_CHECKPOINT;
    for (float x : buf)
        if (!isfinite(x)) return RC_ERR_BAD_CHECKPOINT;
    DN_HIP(hipSetDevice(d->device));
    hipStream_t s = ctx_stream(c);
    DN_HIP(hipStreamSynchronize(s));
    DN_HIP(hipMemcpy(d->d_w, buf.data(), n * 4, hipMemcpyHostToDevice));
    DN_HIP(hipMemcpy(d->d_m, buf.data() + n, n * 4, hipMemcpyHostToDevice));
    DN_HIP(hipMemcpy(d->d_v, buf.data() + 2 * n, n * 4, hipMemcpyHostToDevice));
    d->step = (uint64_t)hdr[3] | ((uint64_t)hdr[4] << 32);
    return refresh_bf16(d, s);
}

}  // extern "C"
