// Index arithmetic of the LDS-tiled convolution (nn.hip), written with 32-bit
// offsets and 24-bit multiplies (full-rate instructions on gfx950) instead of
// 64-bit pixel x stride products.  Host and device: the host side checks the
// bounds that make them exact (conv_tiled_offsets_fit).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace casclb {
namespace nn {

__host__ __device__ inline uint32_t mul24(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul24(a, b);
#else
    return (a & 0xffffffu) * (b & 0xffffffu);
#endif
}

// q / D for 0 <= q < N by a multiply and a shift (exact over that range; checked at compile time).
template <int D, int N>
struct SmallDiv {
    static constexpr uint32_t kShift = 20;
    static constexpr uint32_t kMul = ((1u << kShift) + D - 1) / D;
    static constexpr bool exact() {
        for (uint32_t q = 0; q < (uint32_t)N; ++q)
            if (((q * kMul) >> kShift) != q / D) return false;
        return true;
    }
    static_assert((uint64_t)N * kMul < (1ull << 32), "product must fit 32 bits");
    static_assert(exact(), "multiply-shift division must be exact on [0, N)");
    __host__ __device__ static uint32_t div(uint32_t q) { return mul24(q, kMul) >> kShift; }
};

// Chunk e (0 <= e < tile pixels x cpp <= 340 x 16) of the staging loop -> pixel
// q = e / cpp of the tile and first channel c0 = 8 (e mod cpp); cpp = ci_pad / 8
// <= 16, inv = 1 / cpp.  (e + 1/2) / cpp lies at least 1/32 from an integer,
// while float rounding moves it by less than 1e-3 on that range.
__host__ __device__ inline void chunk_of(uint32_t e, uint32_t cpp, float inv, uint32_t& q, uint32_t& c0) {
    q = (uint32_t)(((float)e + 0.5f) * inv);
    c0 = (e - mul24(q, cpp)) << 3;
}

// x / d by a float reciprocal inv = 1 / d, exact for x < 16,384 and 1 <= d <= 2,048
// (the tile sizes it serves; tests/nn_index_check.cpp checks every pair).
__host__ __device__ inline uint32_t div_by_inv(uint32_t x, float inv) {
    return (uint32_t)(((float)x + 0.5f) * inv);
}

// Element offset of channel c of pixel (img, y, x) in a view of an N x H x W
// image stack with channel stride cs and channel offset co:
// ((img H + y) W + x) cs + co + c, as img_base + y (W cs) + x cs + co + c.
struct PixelOffsets {
    uint32_t img_base;   // img H W cs
    uint32_t row;        // W cs (< 2^24)
    uint32_t cs;         // (< 2^24)
    uint32_t co;
    __host__ __device__ uint32_t at(uint32_t y, uint32_t x, uint32_t c) const {
        return img_base + mul24(y, row) + mul24(x, cs) + co + c;
    }
};

__host__ __device__ inline PixelOffsets pixel_offsets(uint32_t img, uint32_t h, uint32_t w, uint32_t cs,
                                                      uint32_t co) {
    PixelOffsets p;
    p.row = w * cs;
    p.img_base = img * h * p.row;
    p.cs = cs;
    p.co = co;
    return p;
}

// Tap and channel of K index k = tap ci_pad + c, stepped by 32 (ci_pad >= 16, a
// multiple of 8, so a step crosses at most two taps).
struct TapCursor {
    uint32_t tap, c;
    __host__ __device__ void start(uint32_t k, uint32_t ci_pad) {
        tap = 0;
        c = k;
        while (c >= ci_pad) {
            c -= ci_pad;
            ++tap;
        }
    }
    __host__ __device__ void advance32(uint32_t ci_pad) {
        c += 32;
        if (c >= ci_pad) {
            c -= ci_pad;
            ++tap;
        }
        if (c >= ci_pad) {
            c -= ci_pad;
            ++tap;
        }
    }
};

// tap / 3 for tap < 10.
__host__ __device__ inline uint32_t tap_row(uint32_t tap) { return (tap * 11u) >> 5; }

}  // namespace nn
}  // namespace casclb
