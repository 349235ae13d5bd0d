// Kernels of the warm-start surrogate network (circular 3x3 convolutions on
// bf16 matrix cores, fp32 accumulation) and their launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace casclb {
namespace nn {

typedef uint16_t bf16_t;  // bfloat16 bit pattern

// An NHWC tensor view: element (n, y, x, c) at base[((n*H + y)*W + x)*cs + co + c].
struct View {
    void* base;
    int32_t cs;  // channel stride (elements per pixel), multiple of 8
    int32_t co;  // channel offset, multiple of 8
};

// y = conv3x3(x) (+ bias, relu) over N x H x W pixels, circular padding.
//  x: bf16 (x_f32 = false) or fp32 view with ci_pad channels (multiple of 16;
//     channels past the layer's inputs must hold finite values, their weights are 0)
//  wt: bf16 [co_pad32][kpad], k = tap*ci_pad + c, tap = 3*a + c_x (a: row offset + 1),
//     kpad = 9*ci_pad rounded up to 32, zero past 9*ci_pad and past the real outputs
//  bias: fp32 [co] or null; y: bf16 or fp32 view; writes channels [0, co);
//  accumulate: y += result (fp32 output only).
struct ConvArgs {
    View x;
    View y;
    const bf16_t* wt;
    const float* bias;
    int32_t n, h, w;
    int32_t ci_pad, kpad, co, co_pad32;
    int32_t relu, accumulate;
    // tiled kernel only (launch_conv_tiled):
    View x2;            // base != null: input channels [c_split, ci_pad) come from this bf16 view at half
                        // resolution (nearest 2x upsampling fused into the load), [0, c_split) from x
    int32_t c_split;
    View pool;          // base != null: also write the 2x2 means of the bf16 output here (half resolution)
    const float* xin;   // != null: the input is this raw fp32 [pixels][cin_raw] array (zeros past cin_raw)
    int32_t cin_raw;
    FastDiv div_w, div_h;   // plain kernel only, set by launch_conv
};
hipError_t launch_conv(const ConvArgs& a, bool x_f32, bool y_f32, hipStream_t s);

// The same convolution (bf16 or raw fp32 input, bf16 or fp32 output) with the
// input tile and its circular halo staged in LDS: a workgroup computes an
// 8 x 32 (or 16 x 16) pixel tile of one image for all output channels.  Needs
// w a multiple of 16 and h of 16 (or w of 32 and h of 8) and ci_pad <= 128;
// returns hipErrorInvalidValue otherwise (use launch_conv).
bool conv_tiled_fits(int32_t h, int32_t w, int32_t ci_pad);
// Whether the tensors and strides of a tiled convolution fit its 32-bit offsets and 24-bit multiplies.
bool conv_tiled_offsets_fit(const ConvArgs& a);
hipError_t launch_conv_tiled(const ConvArgs& a, bool y_f32, hipStream_t s);

// Weight gradient dW[o][tap][c] = sum_p g[p][o] x[p shifted by tap][c] over
// N x H x W pixels: g fp32 view (co channels), x bf16 view (ci channels).
// Writes split partial sums to `partials` [splits][co_pad16][9][ci_pad16] and
// then their ordered sum into out [co][3][3][ci] (fp32, `accumulate`: +=).
struct WgradArgs {
    View g;
    View x;
    int32_t n, h, w;
    int32_t co, ci, co_pad16, ci_pad16;
    int32_t splits, chunks_per_wave;  // pixels per wave = 32 * chunks_per_wave
    float* partials;
    float* out;
    int32_t accumulate;
    FastDiv div_w, div_h;   // set by launch_wgrad
};
int32_t wgrad_splits(int64_t pixels, int32_t* chunks_per_wave);
hipError_t launch_wgrad(const WgradArgs& a, hipStream_t s);

// Bias gradient db[o] = sum_p g[p][o], o < co; two ordered passes via partials
// [blocks][co]; `accumulate`: db += sum.
hipError_t launch_bias_grad(View g, int64_t pixels, int32_t co, float* partials, int32_t max_blocks, float* db,
                            int32_t accumulate, hipStream_t s);
int32_t bias_grad_blocks(int64_t pixels);

// Elementwise / resampling (all over N x H x W output pixels, `c` channels):
// avgpool2: dst (H/2 x W/2) = mean of 2x2 of src (H x W), bf16 -> bf16.
hipError_t launch_avgpool(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, hipStream_t s);
// avgpool2 backward, accumulating: dst (H x W, fp32) += src (H/2 x W/2, fp32) / 4.
hipError_t launch_avgpool_bwd(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, hipStream_t s);
// upsample2 (nearest): dst (H x W, bf16) = src (H/2 x W/2, bf16).
hipError_t launch_upsample(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, hipStream_t s);
// upsample2 backward: dst (H/2 x W/2, fp32) = sum of 2x2 of src (H x W, fp32).
hipError_t launch_upsample_bwd(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, hipStream_t s);
// g (fp32) *= (act > 0) (act bf16), over N*H*W pixels, c channels.
hipError_t launch_relu_mask(View g, View act, int64_t pixels, int32_t c, hipStream_t s);
// Pack fp32 [pixels][cin] into a bf16 view with cpad channels (zeros past cin).
hipError_t launch_pack_input(const float* x, int32_t cin, View dst, int32_t cpad, int64_t pixels, hipStream_t s);
// Copy channels [0, c) of an fp32 view into a dense fp32 [pixels][c] array.
hipError_t launch_unpack_output(View src, int32_t c, float* y, int64_t pixels, hipStream_t s);
// Mean squared error: grad (fp32 view, c channels) = 2 weight (y - t) / (pixels*c);
// per-block float64 partial sums of (y - t)^2 into partials[blocks].
hipError_t launch_mse(View y, const float* t, int32_t c, int64_t pixels, View grad, double* partials, int32_t blocks,
                      float weight, hipStream_t s);
// 2x2 mean of an fp32 view: dst (H/2 x W/2) from src (H x W), c channels.
hipError_t launch_avgpool_f32(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, hipStream_t s);
// Adjoint of launch_avgpool_f32: dst (H x W) (+)= src (H/2 x W/2) / 4.
hipError_t launch_unpool_f32(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, int32_t accumulate,
                             hipStream_t s);
// Adam on a flat fp32 vector (bias correction factors given by the host).
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                       float eps, float c1, float c2, hipStream_t s);
// Weight packing from the fp32 parameter layout w[co][3][3][ci]:
// forward layout (see ConvArgs) and the input-gradient layout
// wt_t[c][k'] with k' = tap'*co_pad16 + o holding w[o][8 - tap'][c].
hipError_t launch_pack_weights(const float* w, int32_t co, int32_t ci, bf16_t* fwd, int32_t ci_pad, int32_t kpad,
                               int32_t co_pad32, bf16_t* bwd, int32_t co_pad16, int32_t kpad_t, int32_t ci_pad32,
                               hipStream_t s);
// Ordered sum of doubles (single block).
hipError_t launch_sum(const double* in, int32_t n, double* out, hipStream_t s);

}  // namespace nn
}  // namespace casclb
