// Kernel launchers of the U-Net denoiser (k_unet.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct ConvArgs {
    const uint16_t* in;     // NHWC bf16, Cin channels (Cin a multiple of 8); with in2: N x H/2 x W/2 x Ca
    const uint16_t* in2;    // optional second source: the input is the concatenation of the 2x nearest-
                            // upsampled `in` (channels [0, Ca)) and in2 (N x H x W x (Cin - Ca))
    int Ca;
    int N, H, W, Cin;
    const uint16_t* wt;     // [Cout][9][Cin] bf16
    const float* bias;      // Cout floats or NULL
    const uint16_t* mask;   // optional NHWC [Cout]: the output is zeroed where mask <= 0
    uint16_t* out;          // NHWC bf16, Cout channels
    int Cout;
    int relu;
    uint16_t* pool_out;     // optional: also the 2x2 average pool of the output, N x H/2 x W/2 x Cout (H, W even;
                            // the LDS-tiled kernels)
    const float* head_w;    // optional 1x1 head for Cout = 32 (the row-blocked kernel): with head_out the
    const float* head_b;    // epilogue writes sigmoid(head_b + sum_c out[c] head_w[c]) per pixel (FP32) and
    float* head_out;        // not `out`
};

struct ConvArgsF32 {
    const void* in;         // NHWC float (bf16 when in_bf16), Cin channels; with in2: N x H/2 x W/2 x Ca float
    int in_bf16;
    const float* in2;       // optional skip tensor N x H x W x (Cin - Ca) (concatenated after upsampled `in`)
    int Ca;
    int N, H, W, Cin;
    const float* wt;        // [9][Cin][Cout] float
    const float* bias;      // Cout floats
    float* out;             // NHWC float, Cout channels (ReLU applied)
    int Cout;
};

struct WgradArgs {
    const uint16_t* x;      // layer input NHWC [Cin]
    const uint16_t* g;      // gradient of the pre-activation NHWC [Cout]
    int N, H, W, Cin, Cout;
    int chunk;              // pixels per split-K chunk (multiple of 32)
    float* partial;         // [chunks][Cout][9][Cin]
};

// LDS-tiled kernel for the channel counts of this network (any in2); unet_conv3x3_direct: the direct
// kernel without LDS staging (no second source)
void unet_conv3x3(const ConvArgs& a, hipStream_t st);
void unet_conv3x3_direct(const ConvArgs& a, hipStream_t st);
int unet_wgrad_chunks(size_t P, int chunk);
// LDS-tiled weight gradient: partial sums per chunk of pixel tiles ([chunks][Cout][9][Cin], `chunk`
// unused); returns false for channel counts it has no instance for
int unet_wgrad_lds_chunks(const WgradArgs& a);
bool unet_wgrad_lds(const WgradArgs& a, hipStream_t st);
void unet_wgrad(const WgradArgs& a, hipStream_t st);
void unet_reduce_chunks(const float* partial, int n_chunks, int n, float* out, int add, hipStream_t st);
// bias gradients: per-block column sums, then a fixed-order reduction over the blocks
int unet_colsum_blocks(int P);
void unet_colsum(const uint16_t* g, int P, int C, float* partial, hipStream_t st);
void unet_reduce_blocks(const float* partial, int n_blocks, int n, float* out, int add, hipStream_t st);
void unet_pool2(const uint16_t* in, int N, int H, int W, int C, uint16_t* out, hipStream_t st);
void unet_up2_concat(const uint16_t* a, const uint16_t* skip, int N, int H, int W, int Ca, int Cs, uint16_t* out,
                     hipStream_t st);
void unet_up_back_mask(const uint16_t* g, int N, int H2, int W2, int Ctot, int c0, int C, const uint16_t* mask,
                       uint16_t* out, hipStream_t st);
void unet_pool_back_add_mask(const uint16_t* gpool, const uint16_t* gcat, int N, int H, int W, int C, int Ctot, int c0,
                             const uint16_t* mask, uint16_t* out, hipStream_t st);
void unet_head(const uint16_t* d1, const float* wh, const float* bh, int P, float* y, hipStream_t st);
void unet_loss(const float* y, const float* t, const float* m, int P, int chunk, float* partial, float* sums,
               hipStream_t st);
int unet_head_blocks(int P);
void unet_head_back(const uint16_t* d1, const float* y, const float* t, const float* m, const float* sums,
                    const float* wh, int P, uint16_t* gpre, float* partial, hipStream_t st);
void unet_weights_bf16(const float* w, int Cout, int Cin, uint16_t* wf, uint16_t* wb, hipStream_t st);
void unet_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps, float c1,
               float c2, hipStream_t st);
void unet_fill_f32(float* p, float v, size_t n, hipStream_t st);
// FP32 copy of the forward pass
void unet_conv3x3_f32(const ConvArgsF32& a, hipStream_t st);
void unet_pool2_f32(const float* in, int N, int H, int W, int C, float* out, hipStream_t st);
void unet_head_f32(const float* d1, const float* wh, const float* bh, int P, float* y, hipStream_t st);
void unet_weights_f32t(const float* w, int Cout, int Cin, float* wt, hipStream_t st);
