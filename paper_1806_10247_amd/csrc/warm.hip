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

// One workgroup of kProjBlock threads per plane, two passes over it.
//
// With R[y] = mean over x of (-1)^x A(x, y) and C[x] = mean over y of
// (-1)^y A(x, y), the Nyquist lines of the plane are (-1)^x R[y] +
// (-1)^y (C[x] - (-1)^x c), c = mean over y of (-1)^y R[y] (the (pi, pi)
// coefficient, shared by both lines); the mean and the low modes (0 <
// kx^2 + ky^2 <= k2max, one of each +-k pair, kx in 0..2, |ky| <= 2) are
// orthogonal to both lines and to each other, so every coefficient comes from
// the original plane and one second pass subtracts them all.
//
// Pass 1: wave w takes rows w, w + 16, ...; lane l the columns l + 64 j.  Each
// row's sums over x (the (-1)^x sum, the plain sum and, with low modes, the
// sums against cos / sin (kx x 2 pi / L), kx = 1, 2) are reduced across the
// wave by a butterfly and kept in LDS; each lane keeps its columns' (-1)^y
// sums in registers.  Then the plane sums (total, (pi, pi) and the low-mode
// coefficients, whose y factor exp(i ky y 2 pi / L) multiplies the row sums:
// the modes are separable) are formed one per wave from the row sums, and the
// column sums are added in wave order through LDS.  Pass 2 subtracts, per row,
// R[y], the column terms and the low modes regrouped as a_kx(y) cos(kx x ..) +
// b_kx(y) sin(kx x ..).  Every sum has a fixed order: results do not depend on
// timing.
constexpr int kProjBlock = 1024;
constexpr int kProjWaves = kProjBlock / 64;
constexpr int kMaxLowModes = 12;   // half-plane modes with kx^2 + ky^2 <= 8
constexpr int kProjSums = 2 + 2 * kMaxLowModes;

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// index of the twiddle for wave number k at position i (|k| <= 2, 0 <= i < L)
__device__ __forceinline__ int twiddle_index(int k, int i, int L) {
    int m = (k * i) % L;
    return m < 0 ? m + L : m;
}

size_t project_lds_bytes(int L, int nmodes) {
    return (size_t)((nmodes > 0 ? 9 : 3) * L + kProjWaves * 64 + kProjSums) * sizeof(double);
}

template <int J>
__global__ void __launch_bounds__(kProjBlock) project_k(double* data, int L, int nmodes, int4 modes_a, int4 modes_b,
                                                        int4 modes_c, int4 modes_d, int4 modes_e, int4 modes_f) {
    extern __shared__ double lds[];
    double* red = lds;                          // [kProjWaves][64] wave partials
    double* fin = red + kProjWaves * 64;        // [kProjSums] plane sums
    double* rowR = fin + kProjSums;             // R[y]
    double* rowT = rowR + L;                    // row sums
    double* col = rowT + L;                     // C[x] - (-1)^x c
    double* ct = col + L;                       // with low modes: cos(2 pi m / L)
    double* st = ct + L;                        //   sin(2 pi m / L)
    double* rc1 = st + L;                       //   row sums against cos / sin(kx x 2 pi / L), kx = 1, 2
    double* rs1 = rc1 + L;
    double* rc2 = rs1 + L;
    double* rs2 = rc2 + L;
    double* A = data + (int64_t)blockIdx.x * L * L;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double inv = 1.0 / (double)L;
    __shared__ int mkx[kMaxLowModes], mky[kMaxLowModes];   // wave numbers of the low modes
    if (nmodes > 0) {
        if (threadIdx.x == 0) {
            const int4 packed[6] = {modes_a, modes_b, modes_c, modes_d, modes_e, modes_f};
#pragma unroll
            for (int i = 0; i < 6; ++i) {   // constant indexes: stays in registers
                mkx[2 * i] = packed[i].x;
                mky[2 * i] = packed[i].y;
                mkx[2 * i + 1] = packed[i].z;
                mky[2 * i + 1] = packed[i].w;
            }
        }
        for (int m = threadIdx.x; m < L; m += kProjBlock) sincospi(2.0 * (double)m / (double)L, &st[m], &ct[m]);
        __syncthreads();
    }
    // ---- pass 1: row sums to LDS, column sums in registers
    double colacc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) colacc[j] = 0.0;
    for (int y = wave; y < L; y += kProjWaves) {
        const double* row = A + (int64_t)y * L;
        const double sy = (y & 1) ? -1.0 : 1.0;
        double alt = 0.0, tot = 0.0, c1 = 0.0, s1 = 0.0, c2 = 0.0, s2 = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int x = lane + 64 * j;   // x is even exactly when lane is
            if (x < L) {
                const double v = row[x];
                alt += (lane & 1) ? -v : v;
                tot += v;
                colacc[j] += sy * v;
                if (nmodes > 0) {
                    const int x2 = twiddle_index(2, x, L);
                    c1 += v * ct[x];
                    s1 += v * st[x];
                    c2 += v * ct[x2];
                    s2 += v * st[x2];
                }
            }
        }
        alt = wave_sum(alt);
        tot = wave_sum(tot);
        if (nmodes > 0) {   // uniform: every lane of the block takes the same branch
            c1 = wave_sum(c1);
            s1 = wave_sum(s1);
            c2 = wave_sum(c2);
            s2 = wave_sum(s2);
        }
        if (lane == 0) {
            rowR[y] = alt * inv;
            rowT[y] = tot;
            if (nmodes > 0) {
                rc1[y] = c1;
                rs1[y] = s1;
                rc2[y] = c2;
                rs2[y] = s2;
            }
        }
    }
    __syncthreads();
    // ---- plane sums, one per wave: q = 0 total, 1 (-1)^y R[y], 2 + 2 i and 3 + 2 i the
    // cos and sin coefficients of low mode i
    for (int q = wave; q < 2 + 2 * nmodes; q += kProjWaves) {
        const int kx = q >= 2 ? mkx[(q - 2) >> 1] : 0, ky = q >= 2 ? mky[(q - 2) >> 1] : 0;
        double s = 0.0;
        for (int y = lane; y < L; y += 64) {
            if (q == 0) {
                s += rowT[y];
            } else if (q == 1) {
                s += (y & 1) ? -rowR[y] : rowR[y];
            } else {
                const double pc = kx == 0 ? rowT[y] : (kx == 1 ? rc1[y] : rc2[y]);
                const double ps = kx == 0 ? 0.0 : (kx == 1 ? rs1[y] : rs2[y]);
                const int t = twiddle_index(ky, y, L);
                s += (q & 1) ? ps * ct[t] + pc * st[t] : pc * ct[t] - ps * st[t];
            }
        }
        s = wave_sum(s);
        if (lane == 0) fin[q] = q == 0 ? s * inv * inv : (q == 1 ? s * inv : 2.0 * s * inv * inv);
    }
    __syncthreads();
    const double mean = fin[0], cnn = fin[1];
    // ---- column sums, 64 columns at a time, added in wave order
#pragma unroll
    for (int j = 0; j < J; ++j) {
        red[wave * 64 + lane] = colacc[j];
        __syncthreads();
        const int x = 64 * j + (int)threadIdx.x;
        if (threadIdx.x < 64 && x < L) {
            double s = 0.0;
            for (int w = 0; w < kProjWaves; ++w) s += red[w * 64 + threadIdx.x];
            col[x] = s * inv - ((x & 1) ? -cnn : cnn);
        }
        __syncthreads();
    }
    // ---- pass 2
    for (int y = wave; y < L; y += kProjWaves) {
        double* row = A + (int64_t)y * L;
        const double sy = (y & 1) ? -1.0 : 1.0;
        const double ry = rowR[y];
        double a0 = mean, a1 = 0.0, b1 = 0.0, a2 = 0.0, b2 = 0.0;
        for (int i = 0; i < nmodes; ++i) {
            const int kx = mkx[i], t = twiddle_index(mky[i], y, L);
            const double mc = fin[2 + 2 * i], ms = fin[3 + 2 * i];
            const double a = mc * ct[t] + ms * st[t], b = ms * ct[t] - mc * st[t];
            if (kx == 0) {
                a0 += a;
            } else if (kx == 1) {
                a1 += a;
                b1 += b;
            } else {
                a2 += a;
                b2 += b;
            }
        }
        const double sx0 = (lane & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int x = lane + 64 * j;
            if (x < L) {
                double low = a0;
                if (nmodes > 0) {
                    const int x2 = twiddle_index(2, x, L);
                    low += a1 * ct[x] + b1 * st[x] + a2 * ct[x2] + b2 * st[x2];
                }
                row[x] = row[x] - sx0 * ry - sy * col[x] - low;
            }
        }
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
            if (c < nc)
                ch.c[c].dst[i] = (ch.c[c].src ? ch.c[c].src[i] : 0.0) + ch.c[c].scale * (double)y[i * nc + c];
    }
}

// One workgroup of kProjBlock threads per problem b; the momentum sums are
// reduced per wave by a butterfly and then added in wave order (deterministic).
__global__ void __launch_bounds__(kProjBlock) initial_state_k(const double* drho, const double* u, const double* phi,
                                                              const double* F, const double* S, int batch, int64_t n,
                                                              double rho0, int zero_momentum, double* rho_out,
                                                              double* u_out, double* phi_out) {
    __shared__ double red[3][kProjWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t b = blockIdx.x;
    const int64_t o = b * n, comp = (int64_t)batch * n;
    double shift_x = 0.0, shift_y = 0.0;
    if (zero_momentum) {
        double sr = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll 4
        for (int64_t i = threadIdx.x; i < n; i += kProjBlock) {
            const double r = rho0 + drho[o + i];
            sr += r;
            sx += r * u[o + i];
            sy += r * u[comp + o + i];
        }
        sr = wave_sum(sr);
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        if (lane == 0) {
            red[0][wave] = sr;
            red[1][wave] = sx;
            red[2][wave] = sy;
        }
        __syncthreads();
        double tr = 0.0, tx = 0.0, ty = 0.0;
        for (int w = 0; w < kProjWaves; ++w) {
            tr += red[0][w];
            tx += red[1][w];
            ty += red[2][w];
        }
        shift_x = tx / tr;
        shift_y = ty / tr;
    }
#pragma unroll 4
    for (int64_t i = threadIdx.x; i < n; i += kProjBlock) {
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
    const size_t lds = project_lds_bytes(L, n);
    const int4 ma = make_int4(m[0], m[1], m[2], m[3]), mb = make_int4(m[4], m[5], m[6], m[7]),
               mc = make_int4(m[8], m[9], m[10], m[11]), md = make_int4(m[12], m[13], m[14], m[15]),
               me = make_int4(m[16], m[17], m[18], m[19]), mf = make_int4(m[20], m[21], m[22], m[23]);
    // columns per lane, rounded up to a power of two
    const int cols = (L + 63) / 64;
    auto kernel = cols <= 1 ? project_k<1> : cols <= 2 ? project_k<2> : cols <= 4 ? project_k<4>
                : cols <= 8 ? project_k<8> : cols <= 16 ? project_k<16> : project_k<32>;
    if (lds > 65536) {   // the largest lattices need more than the default dynamic LDS limit
        const hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return LB_EHIP;
    }
    hipLaunchKernelGGL(kernel, dim3(planes), dim3(kProjBlock), lds, (hipStream_t)stream, data, (int)L, n, ma, mb, mc,
                       md, me, mf);
    return done(hipGetLastError());
}

static int channels_of(const lb_warm_channel* in, int32_t nc, bool unpack, Channels* out) {
    if (!in || nc < 1 || nc > LB_WARM_MAX_CHANNELS) return LB_EINVAL;
    for (int c = 0; c < nc; ++c) {
        if (unpack && !in[c].dst) return LB_EINVAL;
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
    hipLaunchKernelGGL(initial_state_k, dim3(batch), dim3(kProjBlock), 0, (hipStream_t)stream, drho, u, phi, F, S,
                       (int)batch, n, rho0, (int)(zero_momentum != 0), rho_out, u_out, phi_out);
    return done(hipGetLastError());
}

}  // extern "C"
