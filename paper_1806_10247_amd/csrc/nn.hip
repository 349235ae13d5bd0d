// Kernels of the warm-start surrogate network: circular 3x3 convolutions as
// implicit GEMMs on the bf16 matrix cores of gfx950 (fp32 accumulation), the
// weight gradient as a split-K GEMM over pixels on the same instructions, and
// the bandwidth-bound elementwise and resampling kernels around them.
//
// Matrix-core tile: v_mfma_f32_16x16x32_bf16 (one wavefront): A is 16 x 32,
// B is 32 x 16, D is 16 x 16.  Lane l holds A row l%16 / B column l%16 at
// k = 8*(l/16) + i (i < 8), and D rows 4*(l/16) + j (j < 4) of column l%16.
#include <hip/hip_runtime.h>
#include <math.h>

#include "nn.hpp"
#include "nn_index.hpp"

namespace casclb {
namespace nn {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ bf16_t f2bf(float f) {
    const __bf16 b = (__bf16)f;  // round to nearest even
    return __builtin_bit_cast(bf16_t, b);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <class T>
__device__ __forceinline__ T* at(const View& v, int64_t pix, int c) {
    return reinterpret_cast<T*>(v.base) + pix * v.cs + v.co + c;
}

// 8 consecutive channels of one pixel as a bf16 A/B fragment.
template <bool F32>
__device__ __forceinline__ bf16x8 load8(const View& v, int64_t pix, int c0) {
    if constexpr (F32) {
        const float4* p = reinterpret_cast<const float4*>(at<const float>(v, pix, c0));
        const float4 lo = p[0], hi = p[1];
        bf16x8 r;
        r[0] = (__bf16)lo.x; r[1] = (__bf16)lo.y; r[2] = (__bf16)lo.z; r[3] = (__bf16)lo.w;
        r[4] = (__bf16)hi.x; r[5] = (__bf16)hi.y; r[6] = (__bf16)hi.z; r[7] = (__bf16)hi.w;
        return r;
    } else {
        return *reinterpret_cast<const bf16x8*>(at<const bf16_t>(v, pix, c0));
    }
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---------------------------------------------------------------------------
// forward convolution (also the input gradient with transposed weights)
// ---------------------------------------------------------------------------
// Workgroup: 4 wavefronts, each computing 16 consecutive pixels x 32 output
// channels (two D tiles sharing each A fragment); grid.x covers the pixels
// in 64-pixel blocks, grid.y the 32-channel groups.  No barriers: a wave
// past the last pixel returns.
template <bool XF32, bool YF32>
__global__ void __launch_bounds__(256) conv3x3_mfma(ConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t npix = (int64_t)a.n * a.h * a.w;
    const int64_t p0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    if (p0 >= npix) return;  // npix is a multiple of 16: a started tile is whole
    const int grp = lane >> 4, col = lane & 15;
    // pixel coordinates by multiply-high division (npix < 2^31), taps by a cursor
    const uint32_t p = (uint32_t)(p0 + col);
    const uint32_t t = a.div_w.div(p), px = p - t * (uint32_t)a.w;
    const uint32_t pn = a.div_h.div(t), py = t - pn * (uint32_t)a.h;
    const int ktot = 9 * a.ci_pad;
    TapCursor kc;
    kc.start(8 * grp, a.ci_pad);
    const bf16_t* w0 = a.wt + (int64_t)(blockIdx.y * 32 + col) * a.kpad;
    const bf16_t* w1 = w0 + (int64_t)16 * a.kpad;
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < a.kpad; k += 32) {
        const int k0 = k + 8 * grp;
        bf16x8 av;
        if (k0 < ktot) {
            const int dy = (int)tap_row(kc.tap), dx = (int)kc.tap - 3 * dy;
            const int yy = wrap((int)py + dy - 1, a.h);
            const int xx = wrap((int)px + dx - 1, a.w);
            av = load8<XF32>(a.x, (int64_t)((pn * (uint32_t)a.h + (uint32_t)yy) * (uint32_t)a.w + (uint32_t)xx),
                             (int)kc.c);
        } else {
            for (int i = 0; i < 8; ++i) av[i] = (__bf16)0.0f;
        }
        kc.advance32(a.ci_pad);
        const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(w0 + k0);
        const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(w1 + k0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b1, acc1, 0, 0, 0);
    }
    for (int tt = 0; tt < 2; ++tt) {
        const int o = blockIdx.y * 32 + 16 * tt + col;
        if (o >= a.co) continue;
        const float bias = a.bias ? a.bias[o] : 0.0f;
        for (int j = 0; j < 4; ++j) {
            float v = (tt == 0 ? acc0[j] : acc1[j]) + bias;
            if (a.relu) v = fmaxf(v, 0.0f);
            const int64_t q = p0 + 4 * grp + j;
            if constexpr (YF32) {
                float* dst = at<float>(a.y, q, o);
                *dst = a.accumulate ? *dst + v : v;
            } else {
                *at<bf16_t>(a.y, q, o) = f2bf(v);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// forward convolution with the input tile in LDS
// ---------------------------------------------------------------------------
// Workgroup = 4 wavefronts = one TH x TW pixel tile of one image (TW = 32,
// TH = 8, or TW = 16, TH = 16).  The tile plus a one-pixel circular halo is
// staged once in LDS as bf16 (pixel stride ci_pad + 8 elements: the 16 lanes
// reading 16 consecutive pixels hit distinct banks).  Wave w owns R = 64/TW
// rows, i.e. four 16-pixel matrix-core tiles; per 32-wide K slice a lane reads
// its four A fragments from LDS and one B fragment (8 weights of one output
// channel) per 16-channel output tile from global memory, each B feeding four
// products.  The output tiles are taken NU at a time (NU = min(tiles, 4)): the
// accumulators of a pass are 16 NU registers, so a 16-channel layer keeps
// enough waves per SIMD to overlap one workgroup's staging with another's
// products.  Epilogue: bias, ReLU, store; with `pool`, the 2 x 2 means of the
// bf16-rounded outputs (the two pixels of a row pair are in one lane, the two
// rows in tiles t and t + TW/16 of the same lane), in the order of avgpool_k.
template <int TW, int XMODE, bool YF32, int NU, int PF>
__global__ void __launch_bounds__(256) conv3x3_tiled(ConvArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    bf16_t* tile = reinterpret_cast<bf16_t*>(lds_raw);
    constexpr int R = 64 / TW, TH = 4 * R, HW = TW + 2, HH = TH + 2, NP = HW * HH, TPR = TW / 16;
    using DivHW = SmallDiv<HW, NP>;
    // addresses are 32-bit element offsets with 24-bit multiplies (conv_tiled_offsets_fit
    // checks on the host that every tensor and row stride fits)
    const uint32_t ps = a.ci_pad + 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, grp = lane >> 4, col = lane & 15;
    const int tiles_x = a.w / TW, tiles_y = a.h / TH;
    int b = blockIdx.x;
    const int tx = b % tiles_x;
    b /= tiles_x;
    const int ty = b % tiles_y;
    const uint32_t img = b / tiles_y;
    const int x0 = tx * TW, y0 = ty * TH;
    const uint32_t cpp = a.ci_pad / 8;   // 8-channel chunks per pixel
    const float inv_cpp = 1.0f / (float)cpp;
    const PixelOffsets src = pixel_offsets(img, a.h, a.w, XMODE == 0 ? a.x.cs : a.cin_raw, XMODE == 0 ? a.x.co : 0);
    const PixelOffsets src2 = pixel_offsets(img, a.h >> 1, a.w >> 1, a.x2.cs, a.x2.co);
    // staged in rounds of SB chunks per thread, all loads of a round issued
    // before its LDS stores (one memory latency per round, not per chunk)
    constexpr int SB = 8;
    if constexpr (XMODE == 2) {
        // raw fp32 input, cin_raw floats per pixel: the lanes read consecutive floats of
        // each tile row (one halo row = HW pixels, contiguous in memory unless it wraps),
        // and the channels from cin_raw to ci_pad are zeroed apart
        const uint32_t cr = a.cin_raw, seg = HW * cr, total = HH * seg;
        const float inv_cr = 1.0f / (float)cr, inv_seg = 1.0f / (float)seg;
        for (uint32_t f0 = 0; f0 < total; f0 += SB * 256) {
            float v[SB];
            uint32_t at_lds[SB];
#pragma unroll
            for (int r = 0; r < SB; ++r) {
                const uint32_t f = f0 + r * 256 + threadIdx.x;
                if (f < total) {
                    const uint32_t row = div_by_inv(f, inv_seg), fr = f - mul24(row, seg);
                    const uint32_t qx = div_by_inv(fr, inv_cr), c = fr - mul24(qx, cr);
                    const int yy = wrap(y0 - 1 + (int)row, a.h), xx = wrap(x0 - 1 + (int)qx, a.w);
                    v[r] = a.xin[src.at(yy, xx, c)];
                    at_lds[r] = mul24(row * HW + qx, ps) + c;
                }
            }
#pragma unroll
            for (int r = 0; r < SB; ++r)
                if (f0 + r * 256 + threadIdx.x < total) tile[at_lds[r]] = __builtin_bit_cast(bf16_t, (__bf16)v[r]);
        }
        const uint32_t padc = a.ci_pad - cr;
        if (padc > 0) {
            const float inv_pad = 1.0f / (float)padc;
            for (uint32_t z = threadIdx.x; z < NP * padc; z += 256) {
                const uint32_t q = div_by_inv(z, inv_pad), c = cr + z - mul24(q, padc);
                tile[mul24(q, ps) + c] = 0;
            }
        }
    }
    for (int e0 = 0; XMODE == 0 && e0 < NP * (int)cpp; e0 += SB * 256) {   // bf16 input (XMODE 0)
        bf16x8 v[SB];
#pragma unroll
        for (int r = 0; r < SB; ++r) {
            const uint32_t e = e0 + r * 256 + threadIdx.x;
            if (e < NP * cpp) {
                uint32_t q, c0;
                chunk_of(e, cpp, inv_cpp, q, c0);
                const uint32_t qy = DivHW::div(q), qx = q - qy * HW;
                const int yy = wrap(y0 - 1 + (int)qy, a.h), xx = wrap(x0 - 1 + (int)qx, a.w);
                const bf16_t* xb = reinterpret_cast<const bf16_t*>(a.x.base);
                const bf16_t* x2b = reinterpret_cast<const bf16_t*>(a.x2.base);
                if ((int)c0 < a.c_split)
                    v[r] = *reinterpret_cast<const bf16x8*>(xb + src.at(yy, xx, c0));
                else
                    v[r] = *reinterpret_cast<const bf16x8*>(x2b + src2.at(yy >> 1, xx >> 1, c0 - a.c_split));
            }
        }
#pragma unroll
        for (int r = 0; r < SB; ++r) {
            const uint32_t e = e0 + r * 256 + threadIdx.x;
            if (e < NP * cpp) {
                uint32_t q, c0;
                chunk_of(e, cpp, inv_cpp, q, c0);
                *reinterpret_cast<bf16x8*>(tile + mul24(q, ps) + c0) = v[r];
            }
        }
    }
    __syncthreads();
    const int ktot = 9 * a.ci_pad;
    const int co16 = (a.co + 15) >> 4;
    // LDS element offset of this lane's A row (halo coordinates) in pixel tile t
    uint32_t lp[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) lp[t] = mul24((wave * R + t / TPR) * HW + 16 * (t % TPR) + col, ps);
    const PixelOffsets dst = pixel_offsets(img, a.h, a.w, a.y.cs, a.y.co);
    const PixelOffsets dpool = pixel_offsets(img, a.h >> 1, a.w >> 1, a.pool.cs, a.pool.co);
    for (int cg = 0; cg < co16; cg += NU) {
        f32x4 acc[4][NU];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < NU; ++u) acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};
        const bf16_t* wrow = a.wt + (int64_t)(cg * 16 + col) * a.kpad + 8 * grp;
        // B fragments of the next PF K slices are in flight while the current one is used
        // (slice s in bq[s % PF]; the loop is unrolled by PF so the ring is indexed statically)
        bf16x8 bq[PF][NU];
#pragma unroll
        for (int q = 0; q < PF; ++q)
#pragma unroll
            for (int u = 0; u < NU; ++u)
                if (cg + u < co16 && 32 * q < a.kpad)
                    bq[q][u] = *reinterpret_cast<const bf16x8*>(wrow + (int64_t)u * 16 * a.kpad + 32 * q);
        // tap and channel of this lane's K index 8 grp + 32 s in slice s
        TapCursor kc;
        kc.start(8 * grp, a.ci_pad);
        for (int k = 0; k < a.kpad; k += 32 * PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int kq = k + 32 * q;
                if (kq >= a.kpad) break;
                const int k0 = kq + 8 * grp;
                bf16x8 bc[NU];
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    bc[u] = bq[q][u];
                    if (cg + u < co16 && kq + 32 * PF < a.kpad)
                        bq[q][u] = *reinterpret_cast<const bf16x8*>(wrow + (int64_t)u * 16 * a.kpad + kq + 32 * PF);
                }
                bf16x8 av[4];
                if (k0 < ktot) {
                    const uint32_t dy = tap_row(kc.tap), dx = kc.tap - 3 * dy;
                    const uint32_t off = mul24(dy * HW + dx, ps) + kc.c;
#pragma unroll
                    for (int t = 0; t < 4; ++t) av[t] = *reinterpret_cast<const bf16x8*>(tile + lp[t] + off);
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
#pragma unroll
                        for (int i = 0; i < 8; ++i) av[t][i] = (__bf16)0.0f;
                }
                kc.advance32(a.ci_pad);
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    if (cg + u < co16) {
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[t], bc[u], acc[t][u], 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int o = (cg + u) * 16 + col;
            if (cg + u >= co16 || o >= a.co) continue;
            const float bias = a.bias ? a.bias[o] : 0.0f;
            float v[4][4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int row = y0 + wave * R + t / TPR;
                const uint32_t base = dst.at(row, x0 + 16 * (t % TPR) + 4 * grp, o);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float x = acc[t][u][j] + bias;
                    if (a.relu) x = fmaxf(x, 0.0f);
                    const uint32_t off = base + j * dst.cs;
                    if constexpr (YF32) {
                        float* d = reinterpret_cast<float*>(a.y.base) + off;
                        *d = a.accumulate ? *d + x : x;
                    } else {
                        const bf16_t hb = f2bf(x);
                        reinterpret_cast<bf16_t*>(a.y.base)[off] = hb;
                        x = bf2f(hb);
                    }
                    v[t][j] = x;
                }
            }
            if constexpr (!YF32) {
                if (a.pool.base) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        if ((t / TPR) % 2) continue;   // the upper row of each row pair
                        const int t2 = t + TPR;
                        const int prow = (y0 + wave * R + t / TPR) >> 1;
#pragma unroll
                        for (int j = 0; j < 4; j += 2) {
                            const float sum = (v[t][j] + v[t][j + 1]) + (v[t2][j] + v[t2][j + 1]);
                            const int px = (x0 + 16 * (t % TPR) + 4 * grp + j) >> 1;
                            reinterpret_cast<bf16_t*>(a.pool.base)[dpool.at(prow, px, o)] = f2bf(0.25f * sum);
                        }
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient
// ---------------------------------------------------------------------------
// Workgroup = one (16 outputs o, 16 inputs c) tile, all 9 taps, and one split
// of the pixels; its 4 wavefronts take consecutive pixel ranges of
// 32*chunks_per_wave pixels, all running the same number of chunks (pixels past
// the end add 0), then sum their tiles in LDS in a fixed order.  Per chunk a
// lane loads its 8 output-gradient values once and the 8 inputs of each tap's
// shifted pixels: one A fragment feeds 9 matrix-core products.  When the width
// is a multiple of 8, the 8 pixels of a lane lie in one row (chunks start at
// multiples of 8), so their coordinates are computed once per chunk.
template <bool ROW8>
__global__ void __launch_bounds__(256) wgrad_mfma(WgradArgs a) {
    __shared__ float red[4][9 * 256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane >> 4, col = lane & 15;
    const int ot_n = a.co_pad16 / 16;
    const int ot = blockIdx.x % ot_n;
    const int ct = blockIdx.x / ot_n;
    const int64_t npix = (int64_t)a.n * a.h * a.w;
    const int64_t per_wave = (int64_t)32 * a.chunks_per_wave;
    const int64_t start = ((int64_t)blockIdx.y * 4 + wave) * per_wave;
    const int o = ot * 16 + col;   // A row of this lane
    const int c = ct * 16 + col;   // B column of this lane
    const bool row8 = (a.w & 7) == 0;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (ROW8) {
        // width a multiple of 8 (so is the pixel count) and npix < 2^31: a lane's 8
        // pixels lie in one row, wholly inside or wholly past the end; coordinates by
        // multiply-high division, loads unconditional from in-range addresses with
        // the values selected afterwards (no per-element branches), so a chunk's
        // loads issue together; the products are those of the general path, in order
        const uint32_t np32 = (uint32_t)npix, w = a.w, h = a.h;
        const bool c_ok = c < a.ci, o_ok = o < a.co;
        const uint32_t csx = a.x.cs, csg = a.g.cs;
        const bf16_t* xb = reinterpret_cast<const bf16_t*>(a.x.base) + a.x.co + (c_ok ? c : 0);
        const float* gb = reinterpret_cast<const float*>(a.g.base) + a.g.co + (o_ok ? o : 0);
        for (int ch = 0; ch < a.chunks_per_wave; ++ch) {
            const int64_t pb64 = start + (int64_t)ch * 32 + 8 * grp;
            const bool ok = pb64 < (int64_t)np32;
            const uint32_t pc = ok ? (uint32_t)pb64 : 0u;
            const float* gp = gb + (uint64_t)pc * csg;
            bf16x8 av;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float gv = gp[(uint32_t)i * csg];
                av[i] = (__bf16)(ok && o_ok ? gv : 0.0f);
            }
            const uint32_t t = a.div_w.div(pc), px = pc - t * w;
            const uint32_t pn = a.div_h.div(t), py = t - pn * h;
            const bool x_ok = ok && c_ok;
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3 - 1, dx = tap % 3 - 1;
                const uint32_t rowpix = (pn * h + (uint32_t)wrap((int)py + dy, (int)h)) * w;
                const bf16_t* rp = xb + (uint64_t)rowpix * csx;
                bf16x8 bv;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const bf16_t xv = rp[(uint32_t)wrap((int)px + i + dx, (int)w) * csx];
                    bv[i] = __builtin_bit_cast(__bf16, x_ok ? xv : (bf16_t)0);
                }
                acc[tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[tap], 0, 0, 0);
            }
        }
    }
    for (int ch = 0; !ROW8 && ch < a.chunks_per_wave; ++ch) {
        const int64_t pb = start + (int64_t)ch * 32 + 8 * grp;
        bf16x8 av;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t p = pb + i;
            const float gv = (p < npix && o < a.co) ? *at<const float>(a.g, p, o) : 0.0f;
            av[i] = (__bf16)gv;
        }
        int px = 0, py = 0;
        int64_t pn = 0;
        if (row8 && pb < npix) {
            px = (int)(pb % a.w);
            const int64_t t = pb / a.w;
            py = (int)(t % a.h);
            pn = t / a.h;
        }
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3 - 1, dx = tap % 3 - 1;
            bf16x8 bv;
            if (row8) {
                const int64_t rowq = (pn * a.h + wrap(py + dy, a.h)) * a.w;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    bf16_t xv = 0;
                    if (pb + i < npix && c < a.ci) xv = *at<const bf16_t>(a.x, rowq + wrap(px + i + dx, a.w), c);
                    bv[i] = __builtin_bit_cast(__bf16, xv);
                }
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int64_t p = pb + i;
                    bf16_t xv = 0;
                    if (p < npix && c < a.ci) {
                        const int qx = (int)(p % a.w);
                        const int64_t t = p / a.w;
                        const int qy = (int)(t % a.h);
                        const int64_t qn = t / a.h;
                        const int64_t q = (qn * a.h + wrap(qy + dy, a.h)) * a.w + wrap(qx + dx, a.w);
                        xv = *at<const bf16_t>(a.x, q, c);
                    }
                    bv[i] = __builtin_bit_cast(__bf16, xv);
                }
            }
            acc[tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[tap], 0, 0, 0);
        }
    }
    // D element (row 4*grp + j = output o, column col = input c), per tap
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
        for (int j = 0; j < 4; ++j) red[wave][tap * 256 + (4 * grp + j) * 16 + col] = acc[tap][j];
    __syncthreads();
    if (wave == 0) {
        for (int tap = 0; tap < 9; ++tap)
            for (int j = 0; j < 4; ++j) {
                const int e = tap * 256 + (4 * grp + j) * 16 + col;
                const float s = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
                const int oo = ot * 16 + 4 * grp + j;
                a.partials[(((int64_t)blockIdx.y * a.co_pad16 + oo) * 9 + tap) * a.ci_pad16 + c] = s;
            }
    }
}

// Fixed-order sum over the block (every thread's value, then a tree in LDS).
__device__ float block_sum_f32(float v, float* lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    return lds[0];
}

// Sum over the splits: 64 consecutive (padded) weight entries per workgroup,
// one per lane; the 4 wavefronts take interleaved splits, each lane with four
// independent partial sums, then the wavefronts' sums are added in LDS in a
// fixed order.
__global__ void __launch_bounds__(256) wgrad_reduce(WgradArgs a) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t per_split = (int64_t)a.co_pad16 * 9 * a.ci_pad16;
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    if (e < per_split) {
        int sp = wave;
        for (; sp + 12 < a.splits; sp += 16) {
            s0 += a.partials[(int64_t)sp * per_split + e];
            s1 += a.partials[(int64_t)(sp + 4) * per_split + e];
            s2 += a.partials[(int64_t)(sp + 8) * per_split + e];
            s3 += a.partials[(int64_t)(sp + 12) * per_split + e];
        }
        for (; sp < a.splits; sp += 4) s0 += a.partials[(int64_t)sp * per_split + e];
    }
    red[wave][lane] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (wave == 0 && e < per_split) {
        const int c = (int)(e % a.ci_pad16);
        const int tap = (int)((e / a.ci_pad16) % 9);
        const int o = (int)(e / ((int64_t)9 * a.ci_pad16));
        if (o < a.co && c < a.ci) {
            const float s = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
            const int64_t i = ((int64_t)o * 9 + tap) * a.ci + c;
            a.out[i] = a.accumulate ? a.out[i] + s : s;
        }
    }
}

// ---------------------------------------------------------------------------
// bias gradient: threads of a block are (channel, lane-in-channel) pairs
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) bias_partial(View g, int64_t pixels, int co, int co16, float* partials) {
    __shared__ float red[256];
    const int per = 256 / co16;                 // threads per channel (>= 1)
    const int ch = threadIdx.x % co16, sub = threadIdx.x / co16;
    const int64_t span = (pixels + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = (int64_t)blockIdx.x * span;
    const int64_t b1 = b0 + span < pixels ? b0 + span : pixels;
    // four independent partial sums keep four loads in flight per thread
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    if (sub < per && ch < co) {
        int64_t p = b0 + sub;
        for (; p + 3 * per < b1; p += 4 * per) {
            s0 += *at<const float>(g, p, ch);
            s1 += *at<const float>(g, p + per, ch);
            s2 += *at<const float>(g, p + 2 * per, ch);
            s3 += *at<const float>(g, p + 3 * per, ch);
        }
        for (; p < b1; p += per) s0 += *at<const float>(g, p, ch);
    }
    red[threadIdx.x] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (threadIdx.x < co) {
        float t = 0.0f;
        for (int k = 0; k < per; ++k) t += red[k * co16 + threadIdx.x];
        partials[(int64_t)blockIdx.x * co + threadIdx.x] = t;
    }
}

__global__ void __launch_bounds__(256) bias_reduce(const float* partials, int blocks, int co, float* db,
                                                   int accumulate) {
    // one workgroup per channel: threads take interleaved blocks, fixed-order tree
    __shared__ float lds[256];
    const int o = blockIdx.x;
    float s = 0.0f;
    for (int b = threadIdx.x; b < blocks; b += 256) s += partials[(int64_t)b * co + o];
    const float t = block_sum_f32(s, lds);
    if (threadIdx.x == 0) db[o] = accumulate ? db[o] + t : t;
}

// ---------------------------------------------------------------------------
// resampling and elementwise kernels (grid-stride over output elements)
// ---------------------------------------------------------------------------
#define GRID_STRIDE(i, total) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (total); i += (int64_t)gridDim.x * blockDim.x)

// output pixel (n, y, x) of an H x W grid from a flat index over pixels
__device__ __forceinline__ void decode(int64_t p, int h, int w, int64_t& n, int& y, int& x) {
    x = (int)(p % w);
    const int64_t t = p / w;
    y = (int)(t % h);
    n = t / h;
}

__global__ void avgpool_k(View src, View dst, int n, int h, int w, int c) {
    const int ho = h / 2, wo = w / 2;
    const int64_t total = (int64_t)n * ho * wo * c;
    GRID_STRIDE(i, total) {
        const int ch = (int)(i % c);
        int64_t nn;
        int y, x;
        decode(i / c, ho, wo, nn, y, x);
        const int64_t q = (nn * h + 2 * y) * w + 2 * x;
        const float s = (bf2f(*at<const bf16_t>(src, q, ch)) + bf2f(*at<const bf16_t>(src, q + 1, ch))) +
                        (bf2f(*at<const bf16_t>(src, q + w, ch)) + bf2f(*at<const bf16_t>(src, q + w + 1, ch)));
        *at<bf16_t>(dst, i / c, ch) = f2bf(0.25f * s);
    }
}

__global__ void avgpool_bwd_k(View src, View dst, int n, int h, int w, int c) {
    const int64_t total = (int64_t)n * h * w * c;  // over the fine grid
    GRID_STRIDE(i, total) {
        const int ch = (int)(i % c);
        int64_t nn;
        int y, x;
        decode(i / c, h, w, nn, y, x);
        const int64_t q = (nn * (h / 2) + y / 2) * (w / 2) + x / 2;
        float* d = at<float>(dst, i / c, ch);
        *d += 0.25f * *at<const float>(src, q, ch);
    }
}

__global__ void upsample_k(View src, View dst, int n, int h, int w, int c) {
    const int64_t total = (int64_t)n * h * w * c;  // over the fine grid
    GRID_STRIDE(i, total) {
        const int ch = (int)(i % c);
        int64_t nn;
        int y, x;
        decode(i / c, h, w, nn, y, x);
        const int64_t q = (nn * (h / 2) + y / 2) * (w / 2) + x / 2;
        *at<bf16_t>(dst, i / c, ch) = *at<const bf16_t>(src, q, ch);
    }
}

__global__ void upsample_bwd_k(View src, View dst, int n, int h, int w, int c) {
    const int ho = h / 2, wo = w / 2;
    const int64_t total = (int64_t)n * ho * wo * c;  // over the coarse grid
    GRID_STRIDE(i, total) {
        const int ch = (int)(i % c);
        int64_t nn;
        int y, x;
        decode(i / c, ho, wo, nn, y, x);
        const int64_t q = (nn * h + 2 * y) * w + 2 * x;
        const float s = (*at<const float>(src, q, ch) + *at<const float>(src, q + 1, ch)) +
                        (*at<const float>(src, q + w, ch) + *at<const float>(src, q + w + 1, ch));
        *at<float>(dst, i / c, ch) = s;
    }
}

__global__ void avgpool_f32_k(View src, View dst, int n, int h, int w, int c) {
    const int ho = h / 2, wo = w / 2;
    const int64_t total = (int64_t)n * ho * wo * c;
    GRID_STRIDE(i, total) {
        const int ch = (int)(i % c);
        int64_t nn;
        int y, x;
        decode(i / c, ho, wo, nn, y, x);
        const int64_t q = (nn * h + 2 * y) * w + 2 * x;
        const float s = (*at<const float>(src, q, ch) + *at<const float>(src, q + 1, ch)) +
                        (*at<const float>(src, q + w, ch) + *at<const float>(src, q + w + 1, ch));
        *at<float>(dst, i / c, ch) = 0.25f * s;
    }
}

__global__ void unpool_f32_k(View src, View dst, int n, int h, int w, int c, int accumulate) {
    const int64_t total = (int64_t)n * h * w * c;  // over the fine grid
    GRID_STRIDE(i, total) {
        const int ch = (int)(i % c);
        int64_t nn;
        int y, x;
        decode(i / c, h, w, nn, y, x);
        const int64_t q = (nn * (h / 2) + y / 2) * (w / 2) + x / 2;
        float* d = at<float>(dst, i / c, ch);
        const float v = 0.25f * *at<const float>(src, q, ch);
        *d = accumulate ? *d + v : v;
    }
}

__global__ void relu_mask_k(View g, View act, int64_t pixels, int c) {
    GRID_STRIDE(i, pixels * c) {
        const int ch = (int)(i % c);
        const int64_t p = i / c;
        if (!(bf2f(*at<const bf16_t>(act, p, ch)) > 0.0f)) *at<float>(g, p, ch) = 0.0f;
    }
}

__global__ void pack_input_k(const float* x, int cin, View dst, int cpad, int64_t pixels) {
    GRID_STRIDE(i, pixels * cpad) {
        const int ch = (int)(i % cpad);
        const int64_t p = i / cpad;
        *at<bf16_t>(dst, p, ch) = f2bf(ch < cin ? x[p * cin + ch] : 0.0f);
    }
}

__global__ void unpack_output_k(View src, int c, float* y, int64_t pixels) {
    GRID_STRIDE(i, pixels * c) y[i] = *at<const float>(src, i / c, (int)(i % c));
}

__global__ void __launch_bounds__(256) mse_k(View y, const float* t, int c, int64_t pixels, View grad,
                                             double* partials, float weight) {
    __shared__ double red[256];
    const int64_t total = pixels * c;
    const float scale = (float)(2.0 * (double)weight / (double)total);
    double s = 0.0;
    GRID_STRIDE(i, total) {
        const int ch = (int)(i % c);
        const int64_t p = i / c;
        const float d = *at<const float>(y, p, ch) - t[i];
        *at<float>(grad, p, ch) = scale * d;
        s += (double)d * (double)d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void sum_k(const double* in, int n, double* out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += in[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void adam_k(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    GRID_STRIDE(i, n) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

__global__ void pack_weights_k(const float* w, int co, int ci, bf16_t* fwd, int ci_pad, int kpad, int co_pad32,
                               bf16_t* bwd, int co_pad16, int kpad_t, int ci_pad32) {
    const int64_t nf = (int64_t)co_pad32 * kpad, nb = (int64_t)ci_pad32 * kpad_t;
    GRID_STRIDE(i, nf + nb) {
        if (i < nf) {
            const int o = (int)(i / kpad), k = (int)(i % kpad);
            const int tap = k / ci_pad, c = k % ci_pad;
            const float val = (o < co && tap < 9 && c < ci) ? w[((int64_t)o * 9 + tap) * ci + c] : 0.0f;
            fwd[i] = f2bf(val);
        } else {
            const int64_t j = i - nf;
            const int c = (int)(j / kpad_t), k = (int)(j % kpad_t);
            const int tap = k / co_pad16, o = k % co_pad16;
            const float val = (c < ci && tap < 9 && o < co) ? w[((int64_t)o * 9 + (8 - tap)) * ci + c] : 0.0f;
            bwd[j] = f2bf(val);
        }
    }
}

inline unsigned grid_for(int64_t total, int block = 256, int64_t cap = 16384) {
    int64_t b = (total + block - 1) / block;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_conv(const ConvArgs& a_in, bool x_f32, bool y_f32, hipStream_t s) {
    const int64_t npix = (int64_t)a_in.n * a_in.h * a_in.w;
    // the kernel's coordinate division and tap cursor need npix < 2^31 and ci_pad >= 16
    if (npix >= ((int64_t)1 << 31) || a_in.ci_pad < 16 || a_in.ci_pad % 8) return hipErrorInvalidValue;
    ConvArgs a = a_in;
    a.div_w = FastDiv((uint32_t)a.w);
    a.div_h = FastDiv((uint32_t)a.h);
    const dim3 grid((unsigned)((npix + 63) / 64), (unsigned)(a.co_pad32 / 32));
    if (x_f32 && y_f32) hipLaunchKernelGGL((conv3x3_mfma<true, true>), grid, dim3(256), 0, s, a);
    else if (x_f32) hipLaunchKernelGGL((conv3x3_mfma<true, false>), grid, dim3(256), 0, s, a);
    else if (y_f32) hipLaunchKernelGGL((conv3x3_mfma<false, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((conv3x3_mfma<false, false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// Dynamic LDS above the default limit needs the kernel attribute (once per instance).
template <int TW, int XMODE, bool YF32, int NU, int PF>
hipError_t conv_tiled_lds_limit(size_t lds) {
    static bool done = false;
    if (lds <= 65536 || done) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute((const void*)conv3x3_tiled<TW, XMODE, YF32, NU, PF>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    done = e == hipSuccess;
    return e;
}

template <int TW, int NU, int PF>
hipError_t launch_conv_tiled_nu(const ConvArgs& a, bool raw, bool y_f32, dim3 grid, size_t lds, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (raw && y_f32) e = conv_tiled_lds_limit<TW, 2, true, NU, PF>(lds);
    else if (raw) e = conv_tiled_lds_limit<TW, 2, false, NU, PF>(lds);
    else if (y_f32) e = conv_tiled_lds_limit<TW, 0, true, NU, PF>(lds);
    else e = conv_tiled_lds_limit<TW, 0, false, NU, PF>(lds);
    if (e != hipSuccess) return e;
    const dim3 blk(256);
    if (raw && y_f32) hipLaunchKernelGGL((conv3x3_tiled<TW, 2, true, NU, PF>), grid, blk, lds, s, a);
    else if (raw) hipLaunchKernelGGL((conv3x3_tiled<TW, 2, false, NU, PF>), grid, blk, lds, s, a);
    else if (y_f32) hipLaunchKernelGGL((conv3x3_tiled<TW, 0, true, NU, PF>), grid, blk, lds, s, a);
    else hipLaunchKernelGGL((conv3x3_tiled<TW, 0, false, NU, PF>), grid, blk, lds, s, a);
    return hipGetLastError();
}

// Weight fragments in flight: one K slice ahead where the grid fills the chip (the
// other workgroups hide the latency), kDeepPrefetch slices where a few workgroups
// each run a long K loop alone.
constexpr int kDeepPrefetch = 4;
constexpr int64_t kDeepPrefetchBlocks = 512;

template <int TW, int NU>
hipError_t launch_conv_tiled_pf(const ConvArgs& a, bool raw, bool y_f32, dim3 grid, size_t lds, hipStream_t s) {
    if (grid.x <= kDeepPrefetchBlocks) return launch_conv_tiled_nu<TW, NU, kDeepPrefetch>(a, raw, y_f32, grid, lds, s);
    return launch_conv_tiled_nu<TW, NU, 1>(a, raw, y_f32, grid, lds, s);
}

template <int TW>
hipError_t launch_conv_tiled_tw(const ConvArgs& a, bool raw, bool y_f32, dim3 grid, size_t lds, hipStream_t s) {
    switch ((a.co + 15) >> 4) {
        case 1: return launch_conv_tiled_pf<TW, 1>(a, raw, y_f32, grid, lds, s);
        case 2: return launch_conv_tiled_pf<TW, 2>(a, raw, y_f32, grid, lds, s);
        case 3: return launch_conv_tiled_pf<TW, 3>(a, raw, y_f32, grid, lds, s);
        default: return launch_conv_tiled_pf<TW, 4>(a, raw, y_f32, grid, lds, s);
    }
}

bool conv_tiled_fits(int32_t h, int32_t w, int32_t ci_pad) {
    if (ci_pad < 16 || ci_pad > 128 || ci_pad % 8) return false;
    return (w % 32 == 0 && h % 8 == 0) || (w % 16 == 0 && h % 16 == 0);
}

bool conv_tiled_offsets_fit(const ConvArgs& a) {
    // every tensor the kernel addresses in 32-bit element offsets, and every row
    // stride and coordinate within the 24-bit multiplies
    const int64_t px = (int64_t)a.n * a.h * a.w;
    const int64_t lim = (int64_t)1 << 31, lim24 = (int64_t)1 << 24;
    const int64_t cs[5] = {a.x.base ? a.x.cs : 0, a.y.cs, a.x2.base ? a.x2.cs : 0, a.pool.base ? a.pool.cs : 0,
                           a.xin ? a.cin_raw : 0};
    if (a.h >= lim24 || a.w >= lim24 || a.n >= lim24) return false;
    for (int64_t c : cs)
        if (px * (c + 8) >= lim || (int64_t)a.w * (c + 8) >= lim24) return false;
    return true;
}

hipError_t launch_conv_tiled(const ConvArgs& a, bool y_f32, hipStream_t s) {
    if (!conv_tiled_fits(a.h, a.w, a.ci_pad) || !conv_tiled_offsets_fit(a)) return hipErrorInvalidValue;
    const bool wide = a.w % 32 == 0 && a.h % 8 == 0;
    const int tw = wide ? 32 : 16, th = wide ? 8 : 16;
    const int64_t blocks = (int64_t)a.n * (a.h / th) * (a.w / tw);
    const size_t lds = (size_t)(tw + 2) * (th + 2) * (a.ci_pad + 8) * sizeof(bf16_t);
    const dim3 grid((unsigned)blocks);
    const bool raw = a.xin != nullptr;
    return wide ? launch_conv_tiled_tw<32>(a, raw, y_f32, grid, lds, s)
                : launch_conv_tiled_tw<16>(a, raw, y_f32, grid, lds, s);
}

int32_t wgrad_splits(int64_t pixels, int32_t* chunks_per_wave) {
    // about 512 pixels per wavefront (each feeds 9 products per chunk), at least one split
    int32_t cpw = 16;
    int64_t per_block = (int64_t)4 * 32 * cpw;
    if (pixels < per_block) {
        cpw = (int32_t)((pixels + 127) / 128);
        if (cpw < 1) cpw = 1;
        per_block = (int64_t)4 * 32 * cpw;
    }
    *chunks_per_wave = cpw;
    return (int32_t)((pixels + per_block - 1) / per_block);
}

hipError_t launch_wgrad(const WgradArgs& a, hipStream_t s) {
    const unsigned tiles = (unsigned)((a.co_pad16 / 16) * (a.ci_pad16 / 16));
    // the row-aligned path needs w % 8 == 0, npix < 2^31 and w x (channel stride) < 2^31
    const int64_t npix = (int64_t)a.n * a.h * a.w;
    const bool row8 = a.w % 8 == 0 && npix < ((int64_t)1 << 31) && (int64_t)a.w * a.x.cs < ((int64_t)1 << 31) &&
                      (int64_t)8 * a.g.cs < ((int64_t)1 << 31);
    if (row8) {
        WgradArgs b = a;
        b.div_w = FastDiv((uint32_t)a.w);
        b.div_h = FastDiv((uint32_t)a.h);
        hipLaunchKernelGGL(wgrad_mfma<true>, dim3(tiles, (unsigned)a.splits), dim3(256), 0, s, b);
    } else {
        hipLaunchKernelGGL(wgrad_mfma<false>, dim3(tiles, (unsigned)a.splits), dim3(256), 0, s, a);
    }
    const int64_t entries = (int64_t)a.co_pad16 * 9 * a.ci_pad16;
    hipLaunchKernelGGL(wgrad_reduce, dim3((unsigned)((entries + 63) / 64)), dim3(256), 0, s, a);
    return hipGetLastError();
}

int32_t bias_grad_blocks(int64_t pixels) {
    int64_t b = (pixels + 511) / 512;
    if (b > 4096) b = 4096;
    return (int32_t)(b < 1 ? 1 : b);
}

hipError_t launch_bias_grad(View g, int64_t pixels, int32_t co, float* partials, int32_t max_blocks, float* db,
                            int32_t accumulate, hipStream_t s) {
    const int co16 = (co + 15) / 16 * 16;
    int32_t blocks = bias_grad_blocks(pixels);
    if (blocks > max_blocks) blocks = max_blocks;
    hipLaunchKernelGGL(bias_partial, dim3((unsigned)blocks), dim3(256), 0, s, g, pixels, co, co16, partials);
    hipLaunchKernelGGL(bias_reduce, dim3((unsigned)co), dim3(256), 0, s, partials, blocks, co, db, accumulate);
    return hipGetLastError();
}

hipError_t launch_avgpool(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, hipStream_t s) {
    hipLaunchKernelGGL(avgpool_k, dim3(grid_for((int64_t)n * (h / 2) * (w / 2) * c)), dim3(256), 0, s, src, dst, n, h,
                       w, c);
    return hipGetLastError();
}

hipError_t launch_avgpool_bwd(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, hipStream_t s) {
    hipLaunchKernelGGL(avgpool_bwd_k, dim3(grid_for((int64_t)n * h * w * c)), dim3(256), 0, s, src, dst, n, h, w, c);
    return hipGetLastError();
}

hipError_t launch_upsample(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, hipStream_t s) {
    hipLaunchKernelGGL(upsample_k, dim3(grid_for((int64_t)n * h * w * c)), dim3(256), 0, s, src, dst, n, h, w, c);
    return hipGetLastError();
}

hipError_t launch_upsample_bwd(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, hipStream_t s) {
    hipLaunchKernelGGL(upsample_bwd_k, dim3(grid_for((int64_t)n * (h / 2) * (w / 2) * c)), dim3(256), 0, s, src, dst,
                       n, h, w, c);
    return hipGetLastError();
}

hipError_t launch_relu_mask(View g, View act, int64_t pixels, int32_t c, hipStream_t s) {
    hipLaunchKernelGGL(relu_mask_k, dim3(grid_for(pixels * c)), dim3(256), 0, s, g, act, pixels, c);
    return hipGetLastError();
}

hipError_t launch_pack_input(const float* x, int32_t cin, View dst, int32_t cpad, int64_t pixels, hipStream_t s) {
    hipLaunchKernelGGL(pack_input_k, dim3(grid_for(pixels * cpad)), dim3(256), 0, s, x, cin, dst, cpad, pixels);
    return hipGetLastError();
}

hipError_t launch_unpack_output(View src, int32_t c, float* y, int64_t pixels, hipStream_t s) {
    hipLaunchKernelGGL(unpack_output_k, dim3(grid_for(pixels * c)), dim3(256), 0, s, src, c, y, pixels);
    return hipGetLastError();
}

hipError_t launch_mse(View y, const float* t, int32_t c, int64_t pixels, View grad, double* partials, int32_t blocks,
                      float weight, hipStream_t s) {
    hipLaunchKernelGGL(mse_k, dim3((unsigned)blocks), dim3(256), 0, s, y, t, c, pixels, grad, partials, weight);
    return hipGetLastError();
}

hipError_t launch_avgpool_f32(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, hipStream_t s) {
    hipLaunchKernelGGL(avgpool_f32_k, dim3(grid_for((int64_t)n * (h / 2) * (w / 2) * c)), dim3(256), 0, s, src, dst, n,
                       h, w, c);
    return hipGetLastError();
}

hipError_t launch_unpool_f32(View src, View dst, int32_t n, int32_t h, int32_t w, int32_t c, int32_t accumulate,
                             hipStream_t s) {
    hipLaunchKernelGGL(unpool_f32_k, dim3(grid_for((int64_t)n * h * w * c)), dim3(256), 0, s, src, dst, n, h, w, c,
                       accumulate);
    return hipGetLastError();
}

hipError_t launch_sum(const double* in, int32_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_k, dim3(1), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                       float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_k, dim3(grid_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_pack_weights(const float* w, int32_t co, int32_t ci, bf16_t* fwd, int32_t ci_pad, int32_t kpad,
                               int32_t co_pad32, bf16_t* bwd, int32_t co_pad16, int32_t kpad_t, int32_t ci_pad32,
                               hipStream_t s) {
    const int64_t total = (int64_t)co_pad32 * kpad + (int64_t)ci_pad32 * kpad_t;
    hipLaunchKernelGGL(pack_weights_k, dim3(grid_for(total)), dim3(256), 0, s, w, co, ci, fwd, ci_pad, kpad, co_pad32,
                       bwd, co_pad16, kpad_t, ci_pad32);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace casclb
