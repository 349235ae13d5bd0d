// Batched solver: thousands of independent small D2Q9 channels (x periodic,
// halfway bounce-back walls on y) with a uniform driving force F_b and the
// velocity-dependent Lorentz force -s u_x (Hartmann flow, Sec. 6), advanced
// to a steady residual by one persistent launch.
//
// Each workgroup takes domains from a work queue (one global atomic counter)
// and runs a domain to completion by itself: domains are independent, so the
// only synchronisation between time steps is a workgroup barrier.  A domain
// whose two population buffers fit in the workgroup's LDS is copied in once,
// stepped entirely in LDS and copied back; a larger one is stepped in its two
// global-memory buffers.  Every K steps the workgroup reduces the residual
// r = ||u^n - u^{n-K}|| / (K ||u^n||) of the half-forced velocity and stops
// the domain when r < tol, when u did not change at all in K steps (storage
// precision reached), at max_steps, or on a non-finite value.  Finished
// domains retire; when the queue is empty every wave of the grid exits.
#include <hip/hip_runtime.h>
#include <math.h>

#include "batch.hpp"
#include "lattice.hpp"

namespace casclb {

namespace {

template <class T>
__device__ __forceinline__ T bld(const T* p) {
    return *p;
}

// One D2Q9 node of one domain: pull from `src` ([9][n] deviations, order of
// eq. 15), implicit Lorentz half step, collision, store into `dst`.
// Returns the half-forced velocity.
template <class Real, class Store>
__device__ __forceinline__ void batch_node(const Store* src, Store* dst, int n, int nx, int ny, int x, int y,
                                           const BatchParams& bp, const BatchDomain& dom, Real (&u)[3]) {
    constexpr int Q = 9;
    const int node = x + nx * y;
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    Real m[Q];
    static_for<Q>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        constexpr int EX = Flow<2>::velocity(A, 0), EY = Flow<2>::velocity(A, 1);
        const int sy = y - EY;
        const bool wall = sy < 0 || sy >= ny;  // walls on both y ends
        const int sx = EX == 0 ? x : (EX > 0 ? xm : xp);
        const int idx = wall ? Flow<2>::opposite(A) * n + node : A * n + sx + nx * sy;
        m[Flow<2>::grid_of(A)] = static_cast<Real>(bld(src + idx));
    });
    // implicit half step of the velocity-dependent force:
    // rho u_x = j_x + (F_b - s u_x)/2, the step's force is F_b - s u_x
    Real drho = Real(0), jx = Real(0);
    static_for<Q>([&](auto kk) {
        constexpr int K = decltype(kk)::value;
        drho += m[K];
        jx += Real(grid_velocity(K, 0)) * m[K];
    });
    const Real rho = Real(bp.rho0) + drho;
    const Real s = Real(dom.lorentz), fb = Real(dom.force_x);
    const Real ux = (jx + Real(0.5) * fb) / (rho + Real(0.5) * s);
    const Real fx = fb - s * ux;
    const Real f[3] = {fx, Real(0), Real(0)};
    const FlowRates<Real> w{Real(dom.w_shear), Real(bp.w_bulk), Real(bp.w_third), Real(bp.w_fourth)};
    Real rho_out;
    collide_flow<2, Real>(m, Real(bp.rho0), f, f, w, rho_out, u);
    static_for<Q>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        dst[A * n + node] = static_cast<Store>(m[Flow<2>::grid_of(A)]);
    });
}

// FP64 workgroup sum of two values; every thread gets the result.
__device__ __forceinline__ void wg_sum2(double& a, double& b, double* red) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    // every lane of a wave holds the wave's sums after the butterfly; all of
    // them store it (same value, same address): no lane-divergent branch in a
    // loop that contains barriers
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    red[2 * wave] = a;
    red[2 * wave + 1] = b;
    __syncthreads();
    a = 0.0;
    b = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) {
        a += red[2 * w];
        b += red[2 * w + 1];
    }
}

// Runs one domain to completion with buffers `b0` (holding the state) and
// `b1`; returns which of the two holds the final state.
template <class Real, class Store>
__device__ int run_domain(Store* b0, Store* b1, Real* uprev, const BatchParams& bp, const BatchDomain& dom,
                          double* red, int64_t& steps_out, double& res_out, int& status_out) {
    const int nx = dom.nx, ny = dom.ny, n = nx * ny;
    Store* cur = b0;
    Store* nxt = b1;
    int which = 0;
    bool have_prev = false;
    double res = INFINITY;
    int status = kBatchMaxSteps;
    int64_t s = 0;
    for (; s < bp.max_steps;) {
        const bool check = ((s + 1) % bp.check_interval) == 0;
        double du2 = 0.0, u2 = 0.0;
        bool finite = true;
        for (int node = threadIdx.x; node < n; node += blockDim.x) {
            const int y = node / nx, x = node - y * nx;
            Real u[3];
            batch_node<Real, Store>(cur, nxt, n, nx, ny, x, y, bp, dom, u);
            if (check) {
                const double ux = (double)u[0], uy = (double)u[1];
                const double ox = (double)uprev[node], oy = (double)uprev[n + node];
                uprev[node] = u[0];
                uprev[n + node] = u[1];
                du2 += (ux - ox) * (ux - ox) + (uy - oy) * (uy - oy);
                u2 += ux * ux + uy * uy;
                finite = finite && isfinite(ux) && isfinite(uy);
            }
        }
        __syncthreads();  // the step's writes are visible before the next step reads them
        Store* t = cur;
        cur = nxt;
        nxt = t;
        which ^= 1;
        ++s;
        if (check) {
            double bad = finite ? 0.0 : 1.0, unused = 0.0;
            wg_sum2(du2, u2, red);
            wg_sum2(bad, unused, red + 64);
            int stop = 0;
            if (bad > 0.0) {
                stop = kBatchNonFinite;
            } else if (have_prev) {
                res = sqrt(du2) / ((double)bp.check_interval * sqrt(u2));
                if (du2 == 0.0)
                    stop = kBatchStationary;
                else if (res < bp.tol)
                    stop = kBatchConverged;
            }
            // Every lane holds the same sums; broadcasting the decision from lane 0
            // makes the loop exit a scalar branch.  Left as a per-lane value the
            // compiler may build an exec-mask loop around the barriers that re-runs
            // without the work-queue atomic of the enclosing loop (a hang).
            stop = __builtin_amdgcn_readfirstlane(stop);
            if (stop) {
                status = stop;
                break;
            }
            have_prev = true;
        }
    }
    steps_out = s;
    res_out = res;
    status_out = status;
    return which;
}

}  // namespace

template <class Real, class Store>
__global__ void __launch_bounds__(1024) casclb_batch(BatchParams bp) {
    extern __shared__ unsigned char lds_raw[];
    __shared__ int s_next;
    __shared__ double red[160];
    Store* lds = reinterpret_cast<Store*>(lds_raw);
    // Control flow of this loop is kept scalar (wave-uniform in registers the
    // compiler can see): a lane-divergent branch in a loop that holds barriers
    // lets the compiler split it into nested exec-mask loops in which the other
    // lanes re-enter the barriers without the work-queue atomic (a hang).
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (;;) {
        if (wave == 0) {
            // every lane executes the atomic, only lane 0 adds 1; lane 0's
            // result is the index this workgroup took
            const int v = atomicAdd(bp.queue, threadIdx.x == 0 ? 1 : 0);
            s_next = __builtin_amdgcn_readfirstlane(v);
        }
        __syncthreads();
        const int d = __builtin_amdgcn_readfirstlane(s_next);
        __syncthreads();
        if (d >= bp.ndomains) break;
        const BatchDomain dom = bp.domains[bp.order[d]];
        const int n = dom.nx * dom.ny;
        Store* g0 = reinterpret_cast<Store*>(bp.pool) + dom.offset;
        Store* g1 = g0 + (int64_t)9 * n;
        Real* uprev = reinterpret_cast<Real*>(bp.uprev) + dom.uprev_offset;
        int64_t steps = 0;
        double res = INFINITY;
        int status = 0;
        if (n <= bp.lds_nodes) {
            Store* l0 = lds;
            Store* l1 = lds + (int64_t)9 * n;
            for (int i = threadIdx.x; i < 9 * n; i += blockDim.x) l0[i] = g0[i];
            __syncthreads();
            const int which = run_domain<Real, Store>(l0, l1, uprev, bp, dom, red, steps, res, status);
            const Store* fin = which ? l1 : l0;
            for (int i = threadIdx.x; i < 9 * n; i += blockDim.x) g0[i] = fin[i];
            __syncthreads();
        } else {
            const int which = run_domain<Real, Store>(g0, g1, uprev, bp, dom, red, steps, res, status);
            if (which) {
                for (int i = threadIdx.x; i < 9 * n; i += blockDim.x) g0[i] = g1[i];
                __syncthreads();
            }
        }
        if (wave == 0) {  // all lanes of wave 0 store the same values
            const int id = bp.order[d];
            bp.out_steps[id] = steps;
            bp.out_residual[id] = res;
            bp.out_status[id] = status;
        }
    }
}

__global__ void casclb_batch_reset(int* queue) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
}

// Half-forced velocity and density of every node of one domain.
template <class Real, class Store>
__global__ void casclb_batch_moments(BatchParams bp, int id, double* rho_out, double* u_out) {
    const BatchDomain dom = bp.domains[id];
    const int nx = dom.nx, ny = dom.ny, n = nx * ny;
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= n) return;
    const int y = node / nx, x = node - y * nx;
    const Store* src = reinterpret_cast<const Store*>(bp.pool) + dom.offset;
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    Real drho = Real(0), jx = Real(0), jy = Real(0);
    static_for<9>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        constexpr int EX = Flow<2>::velocity(A, 0), EY = Flow<2>::velocity(A, 1);
        const int sy = y - EY;
        const bool wall = sy < 0 || sy >= ny;
        const int sx = EX == 0 ? x : (EX > 0 ? xm : xp);
        const Real v = static_cast<Real>(src[wall ? Flow<2>::opposite(A) * n + node : A * n + sx + nx * sy]);
        drho += v;
        jx += Real(EX) * v;
        jy += Real(EY) * v;
    });
    const Real rho = Real(bp.rho0) + drho;
    rho_out[node] = (double)rho;
    u_out[node] = (double)((jx + Real(0.5) * Real(dom.force_x)) / (rho + Real(0.5) * Real(dom.lorentz)));
    u_out[n + node] = (double)(jy / rho);
}

// Rest state (deviations zero) of every domain's first buffer.
template <class Store>
__global__ void casclb_batch_zero(Store* pool, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        pool[i] = Store(0);
}

// ---- routed domains: one ordinary launch per step over all of them

template <class Real, class Store, bool CHECK>
__global__ void __launch_bounds__(kWideBlock) casclb_batch_wide(WideParams p, int parity) {
    // the routed domains are the batch's longest chains of steps: their waves take
    // precedence in issue over the persistent launch's, which runs beside them
    __builtin_amdgcn_s_setprio(3);
    __shared__ double red[3][kWideBlock / 64];
    const int4 t = p.tiles[blockIdx.x];
    if (p.state[t.x] >= 2) return;   // the slot stopped: uniform over the workgroup
    const BatchDomain dom = p.domains[p.ids[t.x]];
    const int nx = dom.nx, ny = dom.ny, n = nx * ny;
    Store* g0 = reinterpret_cast<Store*>(p.pool) + dom.offset;
    Store* g1 = g0 + (int64_t)9 * n;
    const Store* src = parity ? g1 : g0;
    Store* dst = parity ? g0 : g1;
    BatchParams bp{};
    bp.rho0 = p.rho0;
    bp.w_bulk = p.w_bulk;
    bp.w_third = p.w_third;
    bp.w_fourth = p.w_fourth;
    const int node = t.y + (int)threadIdx.x;
    double du2 = 0.0, u2 = 0.0, bad = 0.0;
    if (node < n) {
        const int y = node / nx, x = node - y * nx;
        Real u[3];
        batch_node<Real, Store>(src, dst, n, nx, ny, x, y, bp, dom, u);
        if (CHECK) {
            Real* uprev = reinterpret_cast<Real*>(p.uprev) + dom.uprev_offset;
            const double ux = (double)u[0], uy = (double)u[1];
            const double ox = (double)uprev[node], oy = (double)uprev[n + node];
            uprev[node] = u[0];
            uprev[n + node] = u[1];
            du2 = (ux - ox) * (ux - ox) + (uy - oy) * (uy - oy);
            u2 = ux * ux + uy * uy;
            bad = (isfinite(ux) && isfinite(uy)) ? 0.0 : 1.0;
        }
    }
    if (CHECK) {
        // wave butterflies, then the waves in order: a fixed summation order
        for (int off = 32; off > 0; off >>= 1) {
            du2 += __shfl_xor(du2, off, 64);
            u2 += __shfl_xor(u2, off, 64);
            bad += __shfl_xor(bad, off, 64);
        }
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[0][wave] = du2;
            red[1][wave] = u2;
            red[2][wave] = bad;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            double s = 0.0;
            for (int w = 0; w < kWideBlock / 64; ++w) s += red[threadIdx.x][w];
            p.partials[(int64_t)blockIdx.x * 3 + threadIdx.x] = s;
        }
    }
}

__global__ void casclb_wide_init(WideParams p) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) *p.step = 0;
    if (r >= p.nslots) return;
    const int id = p.ids[r];
    p.state[r] = 0;
    p.out_steps[id] = 0;
    p.out_residual[id] = INFINITY;
    p.out_status[id] = kBatchNotRun;
}

// One thread per slot: the slot's tile partials in tile order, then the
// stopping rule of the persistent kernel.  The step counter is advanced by a
// separate launch, after every slot has read it.
__global__ void casclb_wide_check(WideParams p) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= p.nslots) return;
    const int st = p.state[r];
    if (st >= 2) return;
    double du2 = 0.0, u2 = 0.0, bad = 0.0;
    const int t0 = p.tile_first[r], nt = p.tile_count[r];
    for (int t = t0; t < t0 + nt; ++t) {
        du2 += p.partials[(int64_t)t * 3];
        u2 += p.partials[(int64_t)t * 3 + 1];
        bad += p.partials[(int64_t)t * 3 + 2];
    }
    const int id = p.ids[r];
    int stop = 0;
    if (bad > 0.0) {
        stop = kBatchNonFinite;
    } else if (st == 1) {
        const double res = sqrt(du2) / ((double)p.check_interval * sqrt(u2));
        p.out_residual[id] = res;
        if (du2 == 0.0)
            stop = kBatchStationary;
        else if (res < p.tol)
            stop = kBatchConverged;
    }
    if (stop) {
        p.state[r] = 2;
        p.out_status[id] = stop;
        p.out_steps[id] = *p.step + p.check_interval;
    } else {
        p.state[r] = 1;
        atomicAdd(p.active, 1);   // an integer count: exact in any order
    }
}

__global__ void casclb_wide_advance(WideParams p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p.step += p.check_interval;
}

__global__ void casclb_wide_reset_active(WideParams p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p.active = 0;
}

__global__ void casclb_wide_close(WideParams p, int64_t steps) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= p.nslots || p.state[r] >= 2) return;
    const int id = p.ids[r];
    p.state[r] = 2;
    p.out_status[id] = kBatchMaxSteps;
    p.out_steps[id] = steps;
}

template <class Store>
__global__ void __launch_bounds__(kWideBlock) casclb_wide_gather(WideParams p) {
    const int4 t = p.tiles[blockIdx.x];
    const int id = p.ids[t.x];
    if ((p.out_steps[id] & 1) == 0) return;
    const BatchDomain dom = p.domains[id];
    const int n = dom.nx * dom.ny;
    const int node = t.y + (int)threadIdx.x;
    if (node >= n) return;
    Store* g0 = reinterpret_cast<Store*>(p.pool) + dom.offset;
    const Store* g1 = g0 + (int64_t)9 * n;
    for (int a = 0; a < 9; ++a) g0[(int64_t)a * n + node] = g1[(int64_t)a * n + node];
}

hipError_t launch_wide_step(bool f64, const WideParams& p, int ntiles, int parity, bool check, hipStream_t s) {
    if (ntiles < 1) return hipSuccess;
    if (f64) {
        if (check)
            hipLaunchKernelGGL((casclb_batch_wide<double, double, true>), dim3(ntiles), dim3(kWideBlock), 0, s, p, parity);
        else
            hipLaunchKernelGGL((casclb_batch_wide<double, double, false>), dim3(ntiles), dim3(kWideBlock), 0, s, p, parity);
    } else {
        if (check)
            hipLaunchKernelGGL((casclb_batch_wide<float, float, true>), dim3(ntiles), dim3(kWideBlock), 0, s, p, parity);
        else
            hipLaunchKernelGGL((casclb_batch_wide<float, float, false>), dim3(ntiles), dim3(kWideBlock), 0, s, p, parity);
    }
    return hipGetLastError();
}

static int slot_blocks(const WideParams& p) { return (p.nslots + 255) / 256; }

hipError_t launch_wide_init(const WideParams& p, hipStream_t s) {
    hipLaunchKernelGGL(casclb_wide_init, dim3(slot_blocks(p)), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_wide_check(const WideParams& p, hipStream_t s) {
    hipLaunchKernelGGL(casclb_wide_reset_active, dim3(1), dim3(64), 0, s, p);
    hipLaunchKernelGGL(casclb_wide_check, dim3(slot_blocks(p)), dim3(256), 0, s, p);
    hipLaunchKernelGGL(casclb_wide_advance, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_wide_close(const WideParams& p, int64_t steps, hipStream_t s) {
    hipLaunchKernelGGL(casclb_wide_close, dim3(slot_blocks(p)), dim3(256), 0, s, p, steps);
    return hipGetLastError();
}

hipError_t launch_wide_gather(bool f64, const WideParams& p, int ntiles, hipStream_t s) {
    if (ntiles < 1) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(casclb_wide_gather<double>, dim3(ntiles), dim3(kWideBlock), 0, s, p);
    else
        hipLaunchKernelGGL(casclb_wide_gather<float>, dim3(ntiles), dim3(kWideBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_batch(bool f64, const BatchParams& bp, int grid, int block, size_t lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL(casclb_batch_reset, dim3(1), dim3(64), 0, s, bp.queue);
    if (f64)
        hipLaunchKernelGGL((casclb_batch<double, double>), dim3(grid), dim3(block), lds_bytes, s, bp);
    else
        hipLaunchKernelGGL((casclb_batch<float, float>), dim3(grid), dim3(block), lds_bytes, s, bp);
    return hipGetLastError();
}

hipError_t batch_set_lds_limit(bool f64, size_t lds_bytes) {
    if (f64)
        return hipFuncSetAttribute((const void*)casclb_batch<double, double>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    return hipFuncSetAttribute((const void*)casclb_batch<float, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds_bytes);
}

hipError_t launch_batch_moments(bool f64, const BatchParams& bp, int id, int n, double* rho, double* u,
                                hipStream_t s) {
    const int blocks = (n + 255) / 256;
    if (f64)
        hipLaunchKernelGGL((casclb_batch_moments<double, double>), dim3(blocks), dim3(256), 0, s, bp, id, rho, u);
    else
        hipLaunchKernelGGL((casclb_batch_moments<float, float>), dim3(blocks), dim3(256), 0, s, bp, id, rho, u);
    return hipGetLastError();
}

hipError_t launch_batch_zero(bool f64, void* pool, int64_t n, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (f64)
        hipLaunchKernelGGL(casclb_batch_zero<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)pool, n);
    else
        hipLaunchKernelGGL(casclb_batch_zero<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)pool, n);
    return hipGetLastError();
}

}  // namespace casclb
