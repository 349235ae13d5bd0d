// Field operations of the warm start (include/casclb_warm.h): restriction and
// prolongation between lattices, the two-level Richardson combination, the
// projection that removes the mean and the Nyquist lines, packing of the
// network's NHWC input and unpacking of its output, and the initial moments.
// All are bandwidth-bound passes over float64 planes, run once per problem;
// the plane-wide sums are done by one workgroup per plane in a fixed order so
// results do not depend on timing.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "casclb_warm.h"

namespace casclb_warm {

constexpr int kBlock = 256;

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// fixed-order sum over the block: each thread's partial, then a tree in LDS
__device__ double block_sum(double v, double* lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kBlock) restrict_k(const double* __restrict__ src, int64_t planes, int L,
                                                     double scale, double* __restrict__ dst) {
    const int Lc = L / 2;
    const int64_t total = planes * (int64_t)Lc * Lc;
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < total; k += (int64_t)gridDim.x * kBlock) {
        const int64_t p = k / ((int64_t)Lc * Lc);
        const int r = (int)(k - p * (int64_t)Lc * Lc);
        const int Y = r / Lc, X = r - Y * Lc;
        const double* a = src + p * (int64_t)L * L + (int64_t)(2 * Y) * L + 2 * X;
        dst[k] = scale * (0.25 * ((a[0] + a[1]) + (a[L] + a[L + 1])));
    }
}

// Catmull-Rom weights of the four taps at t = 1/4 (odd fine nodes, taps X-1..X+2)
// and t = 3/4 (even fine nodes, taps X-2..X+1): exact binary fractions.
__constant__ double kW[2][4] = {{-0.0234375, 0.2265625, 0.8671875, -0.0703125},
                                {-0.0703125, 0.8671875, 0.2265625, -0.0234375}};

__global__ void __launch_bounds__(kBlock) prolong_k(const double* __restrict__ src, int64_t planes, int Lc,
                                                    double scale, double* __restrict__ dst) {
    const int L = 2 * Lc;
    const int64_t total = planes * (int64_t)L * L;
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < total; k += (int64_t)gridDim.x * kBlock) {
        const int64_t p = k / ((int64_t)L * L);
        const int r = (int)(k - p * (int64_t)L * L);
        const int y = r / L, x = r - y * L;
        // first tap and weight row per axis
        const int ox = x & 1, oy = y & 1;
        const int x0 = (x >> 1) - 2 + ox, y0 = (y >> 1) - 2 + oy;
        const double* a = src + p * (int64_t)Lc * Lc;
        double acc = 0.0;
        for (int j = 0; j < 4; ++j) {
            const double* row = a + (int64_t)wrap(y0 + j, Lc) * Lc;
            double s = 0.0;
            for (int i = 0; i < 4; ++i) s += kW[ox][i] * row[wrap(x0 + i, Lc)];
            acc += kW[oy][j] * s;
        }
        dst[k] = scale * acc;
    }
}

__global__ void __launch_bounds__(kBlock) axpby_k(int64_t n, double a, const double* x, double b, const double* y,
                                                  double* out) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        out[i] = a * x[i] + b * y[i];
}

// One workgroup per plane.  rows[y] = mean over x of (-1)^x A(x, y); after
// removing (-1)^x rows[y], cols[x] = mean over y of (-1)^y of the rest; the mean
// of the plane is unchanged by both (L even).  The low modes (0 < kx^2 + ky^2 <=
// k2max, one of each +-k pair) are orthogonal to all of these, so their
// coefficients come from the original plane and everything is subtracted in
// one pass.  LDS: 2 L doubles + the sum tree.
constexpr int kMaxLowModes = 12;   // half-plane modes with kx^2 + ky^2 <= 8

__device__ __forceinline__ void mode_angle(int kx, int ky, int x, int y, int L, double* c, double* s) {
    // phase reduced exactly on integers, then sin / cos of pi * 2m / L
    int m = (kx * x + ky * y) % L;
    if (m < 0) m += L;
    sincospi(2.0 * (double)m / (double)L, s, c);
}

__global__ void __launch_bounds__(kBlock) project_k(double* data, int L, int nmodes, int4 modes_a, int4 modes_b,
                                                    int4 modes_c, int4 modes_d, int4 modes_e, int4 modes_f) {
    extern __shared__ double lds[];
    double* rows = lds;
    double* cols = lds + L;
    double* tree = lds + 2 * L;
    double* A = data + (int64_t)blockIdx.x * L * L;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double inv = 1.0 / (double)L;
    // (kx, ky) of the low modes, two per int4
    const int4 packed[6] = {modes_a, modes_b, modes_c, modes_d, modes_e, modes_f};
    int kx[kMaxLowModes], ky[kMaxLowModes];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        kx[2 * i] = packed[i].x;
        ky[2 * i] = packed[i].y;
        kx[2 * i + 1] = packed[i].z;
        ky[2 * i + 1] = packed[i].w;
    }
    // row sums: each wave takes rows, lanes stride along x (coalesced)
    for (int y = wave; y < L; y += kBlock / 64) {
        double s = 0.0;
#pragma unroll 8
        for (int x = lane; x < L; x += 64) s += (x & 1) ? -A[(int64_t)y * L + x] : A[(int64_t)y * L + x];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) rows[y] = s * inv;
    }
    __syncthreads();
    // column sums of the row-projected plane, the plane sum and the low-mode sums
    double total = 0.0;
    double mc[kMaxLowModes], ms[kMaxLowModes];
#pragma unroll
    for (int i = 0; i < kMaxLowModes; ++i) mc[i] = ms[i] = 0.0;
    for (int x = threadIdx.x; x < L; x += kBlock) {
        const double sx = (x & 1) ? -1.0 : 1.0;
        double s = 0.0;
        // unrolled so that several rows' loads are in flight (one workgroup per
        // plane); the sums keep their order
#pragma unroll 8
        for (int y = 0; y < L; ++y) {
            const double v = A[(int64_t)y * L + x];
            total += v;
            const double w = v - sx * rows[y];
            s += (y & 1) ? -w : w;
#pragma unroll
            for (int i = 0; i < kMaxLowModes; ++i) {
                if (i < nmodes) {
                    double c, sn;
                    mode_angle(kx[i], ky[i], x, y, L, &c, &sn);
                    mc[i] += v * c;
                    ms[i] += v * sn;
                }
            }
        }
        cols[x] = s * inv;
    }
    const double mean = block_sum(total, tree) * inv * inv;
    const double two_over_n = 2.0 * inv * inv;
#pragma unroll
    for (int i = 0; i < kMaxLowModes; ++i) {
        if (i < nmodes) {   // nmodes is uniform: every thread takes the same barriers
            mc[i] = block_sum(mc[i], tree) * two_over_n;
            ms[i] = block_sum(ms[i], tree) * two_over_n;
        }
    }
    // block_sum ends with a barrier, so cols[] is complete here
    for (int64_t k = threadIdx.x; k < (int64_t)L * L; k += kBlock) {
        const int y = (int)(k / L), x = (int)(k - (int64_t)y * L);
        const double sx = (x & 1) ? -1.0 : 1.0, sy = (y & 1) ? -1.0 : 1.0;
        double low = 0.0;
#pragma unroll
        for (int i = 0; i < kMaxLowModes; ++i) {
            if (i < nmodes) {
                double c, sn;
                mode_angle(kx[i], ky[i], x, y, L, &c, &sn);
                low += mc[i] * c + ms[i] * sn;
            }
        }
        A[k] = A[k] - sx * rows[y] - sy * cols[x] - mean - low;
    }
}

struct Channels {
    lb_warm_channel c[LB_WARM_MAX_CHANNELS];
};

// The channel loops run over the compile-time maximum with a guard, so every
// access to the argument struct has a constant index (no private-memory copy).
__global__ void __launch_bounds__(kBlock) pack_k(Channels ch, int nc, int64_t total, float* out) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < LB_WARM_MAX_CHANNELS; ++c) {
            if (c < nc) {
                const double v = ch.c[c].src ? ch.c[c].scale * ch.c[c].src[i] + ch.c[c].offset : ch.c[c].offset;
                out[i * nc + c] = (float)v;
            }
        }
    }
}

__global__ void __launch_bounds__(kBlock) unpack_k(const float* y, Channels ch, int nc, int64_t total) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < LB_WARM_MAX_CHANNELS; ++c)
            if (c < nc) ch.c[c].dst[i] = ch.c[c].src[i] + ch.c[c].scale * (double)y[i * nc + c];
    }
}

// One workgroup per problem b.
__global__ void __launch_bounds__(kBlock) initial_state_k(const double* drho, const double* u, const double* phi,
                                                          const double* F, const double* S, int batch, int64_t n,
                                                          double rho0, int zero_momentum, double* rho_out,
                                                          double* u_out, double* phi_out) {
    __shared__ double tree[kBlock];
    const int64_t b = blockIdx.x;
    const int64_t o = b * n, comp = (int64_t)batch * n;
    double shift_x = 0.0, shift_y = 0.0;
    if (zero_momentum) {
        double sr = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll 8
        for (int64_t i = threadIdx.x; i < n; i += kBlock) {
            const double r = rho0 + drho[o + i];
            sr += r;
            sx += r * u[o + i];
            sy += r * u[comp + o + i];
        }
        const double tr = block_sum(sr, tree);
        shift_x = block_sum(sx, tree) / tr;
        shift_y = block_sum(sy, tree) / tr;
    }
#pragma unroll 8
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double r = rho0 + drho[o + i];
        rho_out[o + i] = r;
        u_out[o + i] = (u[o + i] - shift_x) - F[o + i] / (2.0 * r);
        u_out[comp + o + i] = (u[comp + o + i] - shift_y) - F[comp + o + i] / (2.0 * r);
        if (phi_out) phi_out[o + i] = phi[o + i] - (S ? 0.5 * S[o + i] : 0.0);
    }
}

int grid_for(int64_t total) {
    const int64_t blocks = (total + kBlock - 1) / kBlock;
    return (int)(blocks < 65536 ? (blocks > 0 ? blocks : 1) : 65536);
}

int done(hipError_t e) { return e == hipSuccess ? LB_OK : LB_EHIP; }

}  // namespace casclb_warm

using namespace casclb_warm;

extern "C" {

int lb_warm_restrict(const double* src, int32_t planes, int32_t L, double scale, double* dst, void* stream) {
    if (!src || !dst || planes < 1 || L < 2 || L > LB_WARM_MAX_L || (L & 1)) return LB_EINVAL;
    const int64_t total = (int64_t)planes * (L / 2) * (L / 2);
    hipLaunchKernelGGL(restrict_k, dim3(grid_for(total)), dim3(kBlock), 0, (hipStream_t)stream, src, (int64_t)planes,
                       (int)L, scale, dst);
    return done(hipGetLastError());
}

int lb_warm_prolong(const double* src, int32_t planes, int32_t Lc, double scale, double* dst, void* stream) {
    if (!src || !dst || planes < 1 || Lc < 2 || 2 * Lc > LB_WARM_MAX_L) return LB_EINVAL;
    const int64_t total = (int64_t)planes * (2 * Lc) * (2 * Lc);
    hipLaunchKernelGGL(prolong_k, dim3(grid_for(total)), dim3(kBlock), 0, (hipStream_t)stream, src, (int64_t)planes,
                       (int)Lc, scale, dst);
    return done(hipGetLastError());
}

int lb_warm_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out, void* stream) {
    if (n < 0 || (n > 0 && (!x || !y || !out))) return LB_EINVAL;
    if (n == 0) return LB_OK;
    hipLaunchKernelGGL(axpby_k, dim3(grid_for(n)), dim3(kBlock), 0, (hipStream_t)stream, n, a, x, b, y, out);
    return done(hipGetLastError());
}

int lb_warm_project(double* data, int32_t planes, int32_t L, int32_t k2max, void* stream) {
    if (!data || planes < 1 || L < 2 || L > LB_WARM_MAX_L || (L & 1)) return LB_EINVAL;
    if (k2max < 0 || k2max > LB_WARM_MAX_K2) return LB_EINVAL;
    // one mode of each +-k pair: kx > 0, or kx = 0 and ky > 0; |k| far below the Nyquist lines
    int m[2 * kMaxLowModes] = {0};
    int n = 0;
    for (int kx = 0; kx * kx <= k2max; ++kx)
        for (int ky = -3; ky <= 3; ++ky) {
            if (kx * kx + ky * ky == 0 || kx * kx + ky * ky > k2max) continue;
            if (kx == 0 && ky <= 0) continue;
            if (2 * kx >= L || 2 * (ky < 0 ? -ky : ky) >= L) return LB_EINVAL;
            m[2 * n] = kx;
            m[2 * n + 1] = ky;
            ++n;
        }
    const size_t lds = (size_t)(2 * L + kBlock) * sizeof(double);
    hipLaunchKernelGGL(project_k, dim3(planes), dim3(kBlock), lds, (hipStream_t)stream, data, (int)L, n,
                       make_int4(m[0], m[1], m[2], m[3]), make_int4(m[4], m[5], m[6], m[7]),
                       make_int4(m[8], m[9], m[10], m[11]), make_int4(m[12], m[13], m[14], m[15]),
                       make_int4(m[16], m[17], m[18], m[19]), make_int4(m[20], m[21], m[22], m[23]));
    return done(hipGetLastError());
}

static int channels_of(const lb_warm_channel* in, int32_t nc, bool unpack, Channels* out) {
    if (!in || nc < 1 || nc > LB_WARM_MAX_CHANNELS) return LB_EINVAL;
    for (int c = 0; c < nc; ++c) {
        if (unpack && (!in[c].src || !in[c].dst)) return LB_EINVAL;
        out->c[c] = in[c];
    }
    return LB_OK;
}

int lb_warm_pack(const lb_warm_channel* channels, int32_t nchannels, int32_t batch, int64_t n, float* out,
                 void* stream) {
    Channels ch{};
    if (channels_of(channels, nchannels, false, &ch) || !out || batch < 1 || n < 1) return LB_EINVAL;
    const int64_t total = (int64_t)batch * n;
    hipLaunchKernelGGL(pack_k, dim3(grid_for(total)), dim3(kBlock), 0, (hipStream_t)stream, ch, (int)nchannels, total,
                       out);
    return done(hipGetLastError());
}

int lb_warm_unpack(const float* y, const lb_warm_channel* channels, int32_t nchannels, int32_t batch, int64_t n,
                   void* stream) {
    Channels ch{};
    if (channels_of(channels, nchannels, true, &ch) || !y || batch < 1 || n < 1) return LB_EINVAL;
    const int64_t total = (int64_t)batch * n;
    hipLaunchKernelGGL(unpack_k, dim3(grid_for(total)), dim3(kBlock), 0, (hipStream_t)stream, y, ch, (int)nchannels,
                       total);
    return done(hipGetLastError());
}

int lb_warm_initial_state(const double* drho, const double* u, const double* phi, const double* F, const double* S,
                          int32_t batch, int64_t n, double rho0, int32_t zero_momentum, double* rho_out,
                          double* u_out, double* phi_out, void* stream) {
    if (!drho || !u || !F || !rho_out || !u_out || batch < 1 || n < 1) return LB_EINVAL;
    if ((phi == nullptr) != (phi_out == nullptr)) return LB_EINVAL;
    hipLaunchKernelGGL(initial_state_k, dim3(batch), dim3(kBlock), 0, (hipStream_t)stream, drho, u, phi, F, S,
                       (int)batch, n, rho0, (int)(zero_momentum != 0), rho_out, u_out, phi_out);
    return done(hipGetLastError());
}

}  // extern "C"
