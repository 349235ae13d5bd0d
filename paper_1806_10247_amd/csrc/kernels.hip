// Kernels of the casclb library (gfx950, wave64).
//
// Layout in HBM: structure of arrays.  Population a of node n lives at
// buf[a * plane + n], n = x + nx*(y + ny*z); flow planes first, then the five
// D2Q5 planes of the scalar lattice.  `plane` >= N is padded so that the
// planes do not all start at the same HBM channel offset.  Two buffers A/B:
// a step pulls from one and writes the other, so it is race-free.
//
// Launch shape of the per-node kernels: 1D grid, blockDim.x threads along x
// (a multiple of 64, so a wavefront never spans two rows); block b covers
// x-chunk (b % x_blocks) of row b / x_blocks, row = y + ny*z.  Row
// coordinates and wall decisions are block-uniform (scalar registers); only
// the x wrap of the +-1 shifted loads is per lane.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "lattice.hpp"

// Multiply-adds are fused only within one source expression.  With fusion
// across statements the backend decides per basic block, so the kernel
// variants of one lattice (rows or x-adjacent nodes per thread, residual
// steps) would round differently; this way every launch shape gives
// bit-identical results.
#pragma clang fp contract(on)

namespace casclb {

template <class T>
__device__ __forceinline__ T ld_stream(const T* p) {
    return __builtin_nontemporal_load(p);
}
template <class T>
__device__ __forceinline__ void st_stream(T* p, T v) {
    __builtin_nontemporal_store(v, p);
}

template <class Real, class Store>
__device__ __forceinline__ Real to_real(Store v) {
    return static_cast<Real>(v);
}
template <class Store, class Real>
__device__ __forceinline__ Store to_store(Real v) {
    return static_cast<Store>(v);
}

// ---------------------------------------------------------------------------
// float16 storage with stochastic rounding
// ---------------------------------------------------------------------------
// The per-step force kick F.e/<e_x|e_x> of a weakly forced lattice (5.6e-9 on
// D3Q27 at F = 1e-7) lies far below half a float16 unit of the stored
// deviations (the smallest subnormal is 6e-8), so rounding to nearest drops it
// at every store and a lattice started from rest never moves.  Stochastic
// rounding takes the float16 neighbour above or below with probabilities in
// proportion to the distances, so the expected stored value is the float32
// value and the kicks survive on average.  The random bits come from a
// counter-based hash of (node, population, step), so every launch shape gives
// the same result.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Per-population salt added to a node's key (distinct odd multiples of the
// 32-bit golden ratio): over the nodes every bit of key + salt stays uniform.
__device__ __forceinline__ constexpr uint32_t sr_salt(int plane) { return (uint32_t)(plane + 1) * 0x9E3779B9u; }

// float32 -> float16 with stochastic rounding in one instruction
// (v_cvt_sr_f16_f32): the neighbour above or below with probabilities in
// proportion to the distances, the random 32 bits r choosing; exact on
// float16 values, subnormals included (spacing 2^-24).  The pair form packs
// two (low, high) into one word.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_halves_sr(float lo, float hi, uint32_t rlo, uint32_t rhi) {
    half2_t o = {(_Float16)0.0f, (_Float16)0.0f};
    o = __builtin_amdgcn_cvt_sr_f16_f32(o, lo, rlo, false);
    o = __builtin_amdgcn_cvt_sr_f16_f32(o, hi, rhi, true);
    return __builtin_bit_cast(uint32_t, o);
}
__device__ __forceinline__ _Float16 half_sr(float v, uint32_t r) {
    half2_t o = {(_Float16)0.0f, (_Float16)0.0f};
    o = __builtin_amdgcn_cvt_sr_f16_f32(o, v, r, false);
    return o[0];
}

struct RowPos {
    int y, z;            // block-uniform
    int64_t row;         // block-uniform: nx*(y + ny*z)
    bool active;
    uint32_t x, xm, xp;  // per lane: x (clamped), x-1 and x+1 wrapped periodically
    int64_t node;        // row + x
};

__device__ __forceinline__ uint32_t logical_block(const Geometry& g) {
    const uint32_t b = blockIdx.x;
    if (g.xcd_remap) {
        // blocks are dispatched to the 8 XCDs round-robin; hand XCD k the
        // contiguous range [k*G/8, (k+1)*G/8) of logical blocks
        const uint32_t per = (uint32_t)(g.grid_blocks >> 3);
        return (b & 7u) * per + (b >> 3);
    }
    return b;
}

// Position of this thread's node in row k (0 <= k < g.rows) of the group of
// rows of logical block lb.  A row past the last one is clamped and marked
// inactive.
__device__ __forceinline__ RowPos row_position_at(const Geometry& g, uint32_t lb, int k = 0) {
    RowPos p;
    const uint32_t group = g.div_xb.div(lb);
    const int xb = (int)(lb - group * (uint32_t)g.x_blocks);
    uint32_t row = group * (uint32_t)g.rows + (uint32_t)k;
    const bool row_ok = row < (uint32_t)g.nrows;
    if (!row_ok) row = (uint32_t)g.nrows - 1;
    const uint32_t z = g.div_ny.div(row);
    p.y = (int)(row - z * (uint32_t)g.ny);
    p.z = (int)z;
    p.row = (int64_t)g.nx * row;
    const int x = xb * (int)blockDim.x + (int)threadIdx.x;
    p.active = row_ok && x < g.nx;
    const int xc = p.active ? x : g.nx - 1;
    p.x = (uint32_t)xc;
    p.xm = (uint32_t)(xc == 0 ? g.nx - 1 : xc - 1);
    p.xp = (uint32_t)(xc == g.nx - 1 ? 0 : xc + 1);
    p.node = p.row + xc;
    return p;
}

// Position of this thread's node in row k of its own block's group of rows.
__device__ __forceinline__ RowPos row_position(const Geometry& g, int k = 0) {
    return row_position_at(g, logical_block(g), k);
}

// Pull of the population in plane `plane_self` with velocity (EX, EY, EZ)
// (eq. 22b): read node x - e of the stored state, wrapped on periodic axes.
// A link whose source lies in a wall returns the opposite population
// (`plane_opp`) of the same node (halfway bounce-back).  The row part of the
// address and the y/z wall decisions are block-uniform, so each load is a
// uniform base pointer plus one of the three per-lane offsets x, x-1, x+1.
// XWALL: walls on the x axis too (then the x decision is per lane).
template <int EX, int EY, int EZ, bool XWALL, class Store>
__device__ __forceinline__ Store pull(const Store* __restrict__ src, const Geometry& g, const RowPos& p,
                                      int plane_self, int plane_opp) {
    bool wall = false;
    int sy = p.y - EY, sz = p.z - EZ;
    if constexpr (EY != 0) {
        if (sy < 0) { wall |= g.bb[1] != 0; sy += g.ny; }
        if (sy >= g.ny) { wall |= g.bb[1] != 0; sy -= g.ny; }
    }
    if constexpr (EZ != 0) {
        if (sz < 0) { wall |= g.bb[2] != 0; sz += g.nz; }
        if (sz >= g.nz) { wall |= g.bb[2] != 0; sz -= g.nz; }
    }
    const int64_t src_row = (int64_t)g.nx * ((int64_t)sy + (int64_t)g.ny * sz);
    const Store* own = src + (int64_t)plane_opp * g.plane + p.row;       // bounce-back source row
    const Store* base = wall ? own : src + (int64_t)plane_self * g.plane + src_row;
    uint32_t off = EX == 0 ? p.x : (EX > 0 ? p.xm : p.xp);
    if (wall) off = p.x;
    if constexpr (XWALL && EX != 0) {
        const bool lane_wall = g.bb[0] != 0 && (EX > 0 ? p.x == 0 : p.x == (uint32_t)g.nx - 1);
        const Store* q = lane_wall ? own + p.x : base + off;
        return ld_stream(q);
    } else {
        return ld_stream(base + off);
    }
}

template <int D, bool XWALL, class Real, class Store>
__device__ __forceinline__ void gather_flow(const Store* __restrict__ src, const Geometry& g, const RowPos& p,
                                            Real (&m)[Flow<D>::Q]) {
    static_for<Flow<D>::Q>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        constexpr int EX = Flow<D>::velocity(A, 0), EY = Flow<D>::velocity(A, 1), EZ = Flow<D>::velocity(A, 2);
        m[Flow<D>::grid_of(A)] = to_real<Real>(pull<EX, EY, EZ, XWALL>(src, g, p, A, Flow<D>::opposite(A)));
    });
}

template <bool XWALL, class Real, class Store>
__device__ __forceinline__ void gather_scalar(const Store* __restrict__ src, int first_plane, const Geometry& g,
                                              const RowPos& p, Real (&s)[5]) {
    static_for<5>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        s[A] = to_real<Real>(pull<d2q5_velocity(A, 0), d2q5_velocity(A, 1), 0, XWALL>(
            src, g, p, first_plane + A, first_plane + d2q5_opposite(A)));
    });
}

template <int D, class Real>
__device__ __forceinline__ void node_force(const StepArgs& a, const RowPos& p, Real (&fb)[3]) {
    // uniform components first, then the field (if any) replaces them; written
    // without a branch between two stores into fb, which would keep fb (and the
    // force argument) in private memory for float64
    const Real* ff = reinterpret_cast<const Real*>(a.force_field);
    const bool field = ff != nullptr;
    const int64_t off = p.row + p.x;
    const Real f0 = field ? ld_stream(ff + off) : Real(a.fx);
    const Real f1 = field ? ld_stream(ff + a.geo.plane + off) : Real(a.fy);
    Real f2 = Real(0);
    if constexpr (D == 3) f2 = field ? ld_stream(ff + 2 * a.geo.plane + off) : Real(a.fz);
    fb[0] = f0;
    fb[1] = f1;
    fb[2] = f2;
}

// FP64 sum over the block of kDiagSlots values; thread 0 of the block gets the result.
__device__ __forceinline__ void block_sum(double (&v)[kDiagSlots], double* out) {
    __shared__ double red[kMaxBlock / 64][kDiagSlots];
    static_for<kDiagSlots>([&](auto cc) {
        constexpr int C = decltype(cc)::value;
        double s = v[C];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        v[C] = s;
    });
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        static_for<kDiagSlots>([&](auto cc) {   // compile-time indices keep v in registers
            constexpr int C = decltype(cc)::value;
            red[wave][C] = v[C];
        });
    __syncthreads();
    if (threadIdx.x < kDiagSlots) {
        double s = 0.0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// the fused step
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// per-lattice constants: dimension, populations per node, and the velocity /
// opposite of population a in the ABI order
// ---------------------------------------------------------------------------
template <int LAT>
struct Lat {
    static constexpr int D = LAT == kD2Q9 || LAT == kD2Q9D2Q5 ? 2 : 3;
    static constexpr int Q = LAT == kD3Q15 ? 15 : Flow<D>::Q;
    __device__ static constexpr int velocity(int a, int axis) {
        if constexpr (LAT == kD3Q15) return D3Q15::velocity(a, axis);
        else return Flow<D>::velocity(a, axis);
    }
    __device__ static constexpr int opposite(int a) {
        if constexpr (LAT == kD3Q15) return D3Q15::opposite(a);
        else return Flow<D>::opposite(a);
    }
};

// ---------------------------------------------------------------------------
// walls with a velocity / a fixed scalar value, viscous heating (2D lattices)
// ---------------------------------------------------------------------------
// Side crossed first (axis x, then y) by the pull of velocity (EX, EY) at p:
// 2*axis + (0 low, 1 high), or -1 when the link stays in the fluid.
template <int EX, int EY>
__device__ __forceinline__ int crossed_side(const Geometry& g, const RowPos& p) {
    int side = -1;
    if constexpr (EY != 0) {
        const int sy = p.y - EY;
        if (g.bb[1] && sy < 0) side = 2;
        if (g.bb[1] && sy >= g.ny) side = 3;
    }
    if constexpr (EX != 0) {
        const int sx = (int)p.x - EX;
        if (g.bb[0] && sx < 0) side = 0;
        if (g.bb[0] && sx >= g.nx) side = 1;
    }
    return side;
}

__device__ __forceinline__ double wall_u_of(const StepArgs& a, int side, int c) { return a.walls[2 * side + c]; }
__device__ __forceinline__ bool phi_fixed_of(const StepArgs& a, int side) { return a.walls[8 + side] != 0.0; }
__device__ __forceinline__ double phi_wall_of(const StepArgs& a, int side) { return a.walls[12 + side]; }

// Moving-wall bounce-back: a link from a wall of velocity u_w brings the
// opposite population plus 6 w_a rho0 (e_a . u_w) (m in grid order).
template <class Real>
__device__ __forceinline__ void moving_walls(const StepArgs& a, const RowPos& p, Real (&m)[9]) {
    static_for<9>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        constexpr int EX = Flow<2>::velocity(A, 0), EY = Flow<2>::velocity(A, 1);
        const int side = crossed_side<EX, EY>(a.geo, p);
        if (side >= 0) {
            const double eu = EX * wall_u_of(a, side, 0) + EY * wall_u_of(a, side, 1);
            m[Flow<2>::grid_of(A)] += Real(6.0 * rest_weight<2>(A) * a.rho0 * eu);
        }
    });
}

// S:S of the strain rate from the second raw moments (deviations kxx, kyy,
// kxy of the streamed populations) and the half-forced velocity: with
// Pi_ab = sum f e_a e_b - rho u_a u_b - rho/3 delta_ab,
// S_xy = -3 w_shear/(2 rho0) Pi_xy, S_xx - S_yy = -3 w_shear/(2 rho0)(Pi_xx - Pi_yy),
// S_xx + S_yy = -3 w_bulk/(2 rho0)(Pi_xx + Pi_yy) (Sec. 6, thermal Couette flow).
template <class Real>
__device__ __forceinline__ Real strain_rate_squared(const StepArgs& a, Real kxx, Real kyy, Real kxy, Real rho,
                                                    const Real (&u)[3]) {
    const Real drho3 = (rho - Real(a.rho0)) * Real(1.0 / 3.0);
    const Real pxx = kxx - rho * u[0] * u[0] - drho3;
    const Real pyy = kyy - rho * u[1] * u[1] - drho3;
    const Real pxy = kxy - rho * u[0] * u[1];
    const Real cs = Real(-1.5 * a.w_shear / a.rho0), cb = Real(-1.5 * a.w_bulk / a.rho0);
    const Real sxy = cs * pxy, dif = cs * (pxx - pyy), tr = cb * (pxx + pyy);
    const Real sxx = Real(0.5) * (tr + dif), syy = Real(0.5) * (tr - dif);
    return sxx * sxx + syy * syy + Real(2) * sxy * sxy;
}

// Fixed-value scalar walls (anti-bounce-back with the source the collision
// adds to every population, S_tot/5, restored on the reflected link):
// g_a = -g^p_opp(a) + phi_w (1/3 + u_w,k^2) + 2 S_tot/5, k the axis of a.
template <class Real>
__device__ __forceinline__ void scalar_walls(const StepArgs& a, const RowPos& p, Real stot, Real (&sc)[5]) {
    static_for<5>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        constexpr int EX = d2q5_velocity(A, 0), EY = d2q5_velocity(A, 1);
        if constexpr (EX != 0 || EY != 0) {
            const int side = crossed_side<EX, EY>(a.geo, p);
            if (side >= 0 && phi_fixed_of(a, side)) {
                const double uk = wall_u_of(a, side, EX != 0 ? 0 : 1);
                sc[A] = -sc[A] + Real(phi_wall_of(a, side) * (1.0 / 3.0 + uk * uk)) + Real(0.4) * stot;
            }
        }
    });
}

// Collision, both half steps and (DIAG) residual terms of one node whose
// streamed populations `raw` / `raw_sc` have been loaded: m (grid order, ABI
// order for D3Q15) and sc receive the populations to store.
template <int LAT, class Real, class Store, bool DIAG, bool EXT = false>
__device__ __forceinline__ void collide_node(const StepArgs& a, const RowPos& p, const Store (&raw)[Lat<LAT>::Q],
                                             const Store (&raw_sc)[5], double (&v)[kDiagSlots],
                                             Real (&m)[Lat<LAT>::Q], Real (&sc)[5]) {
    constexpr int D = Lat<LAT>::D;
    constexpr int Q = Lat<LAT>::Q;
    const Geometry& g = a.geo;
    static_for<Q>([&](auto kk) {
        constexpr int K = decltype(kk)::value;
        m[K] = to_real<Real>(raw[K]);
    });
    Real kxx = Real(0), kyy = Real(0), kxy = Real(0);
    if constexpr (EXT && D == 2) {
        moving_walls<Real>(a, p, m);
        if constexpr (LAT == kD2Q9D2Q5) {
            static_for<Q>([&](auto kk) {
                constexpr int K = decltype(kk)::value;
                constexpr int EX = grid_velocity(K, 0), EY = grid_velocity(K, 1);
                if constexpr (EX != 0) kxx += m[K];
                if constexpr (EY != 0) kyy += m[K];
                if constexpr (EX * EY != 0) kxy += Real(EX * EY) * m[K];
            });
        }
    }
    Real fb[3];
    node_force<D, Real>(a, p, fb);
    const Real cpre = Real(a.f_pre), ctot = Real(a.f_tot);
    Real fpre[3] = {cpre * fb[0], cpre * fb[1], cpre * fb[2]};
    Real ftot[3] = {ctot * fb[0], ctot * fb[1], ctot * fb[2]};
    if constexpr (D == 2) {
        if (a.lorentz != 0.0) {
            // velocity-dependent x-force F_x - s u_x (Hartmann flow, Sec. 6) by the implicit midpoint
            // rule: rho u_x = j_x + (F_pre,x - s u_x)/2, the step's force F_x - s u_x with that u_x
            Real drho = Real(0), jx = Real(0);
            static_for<Q>([&](auto kk) {
                constexpr int K = decltype(kk)::value;
                drho += m[K];
                jx += Real(grid_velocity(K, 0)) * m[K];
            });
            const Real rho = Real(a.rho0) + drho, sl = Real(a.lorentz);
            const Real ux = (jx + Real(0.5) * fpre[0]) / (rho + Real(0.5) * sl);
            fpre[0] = fpre[0] - sl * ux;
            ftot[0] = ftot[0] - sl * ux;
        }
    }
    const FlowRates<Real> w{Real(a.w_shear), Real(a.w_bulk), Real(a.w_third), Real(a.w_fourth)};
    Real rho, u[3];
    if constexpr (LAT == kD3Q15)
        collide_d3q15<Real>(m, Real(a.rho0), fpre, ftot, w, rho, u);   // m in ABI order
    else
        collide_flow<D, Real>(m, Real(a.rho0), fpre, ftot, w, rho, u);

    Real phi_post = Real(0), phi_star = Real(0);
    if constexpr (LAT == kD2Q9D2Q5) {
        static_for<5>([&](auto kk) {
            constexpr int K = decltype(kk)::value;
            sc[K] = to_real<Real>(raw_sc[K]);
        });
        Real sb = Real(a.source);
        if (a.source_field) sb = ld_stream(reinterpret_cast<const Real*>(a.source_field) + p.row + p.x);
        Real spre = Real(a.s_pre) * sb, stot = Real(a.s_tot) * sb;
        if constexpr (EXT) {
            const Real sr = Real(a.heat) * strain_rate_squared<Real>(a, kxx, kyy, kxy, rho, u);
            spre += sr;
            stot += sr;
            scalar_walls<Real>(a, p, stot, sc);
        }
        const ScalarRates<Real> ws{Real(a.w_phi), Real(a.w_phi_high)};
        const Real phi_o = collide_scalar<Real>(sc, u, spre, stot, ws);
        phi_post = phi_o + stot;                  // scalar of the written state
        phi_star = phi_o + Real(0.5) * spre;      // half-sourced scalar (the u* analogue)
    }

    if constexpr (DIAG) {
        if (p.active) {
            Real* up = reinterpret_cast<Real*>(a.u_prev) + p.row;
            double du2 = 0.0, u2 = 0.0;
            bool finite = isfinite((double)rho);
            static_for<D>([&](auto ax) {
                constexpr int AX = decltype(ax)::value;
                Real* slot = up + (int64_t)AX * g.plane + p.x;
                const double old = (double)*slot;
                const double now = (double)u[AX];
                *slot = u[AX];
                du2 += (now - old) * (now - old);
                u2 += now * now;
                finite = finite && isfinite(now);
            });
            v[0] += du2;
            v[1] += u2;
            v[2] += (double)(rho - Real(a.rho0));
            // momentum of the written state: j + F_tot = rho u - F_pre/2 + F_tot
            static_for<D>([&](auto ax) {
                constexpr int AX = decltype(ax)::value;
                v[3 + AX] += (double)rho * (double)u[AX] - 0.5 * (double)fpre[AX] + (double)ftot[AX];
            });
            v[6] += (double)phi_post;
            if constexpr (LAT == kD2Q9D2Q5) {
                Real* slot = up + (int64_t)D * g.plane + p.x;
                const double old = (double)*slot;
                const double now = (double)phi_star;
                *slot = phi_star;
                v[8] += (now - old) * (now - old);
                v[9] += now * now;
                finite = finite && isfinite(now);
            }
            v[7] += finite ? 0.0 : 1.0;
        }
    }
}

// Random key of one node's stores in this step (stochastic rounding).
__device__ __forceinline__ uint32_t sr_node_key(const StepArgs& a, const RowPos& p) {
    return mix32(((uint32_t)p.node * 0x9E3779B1u) ^ a.sr_seed);
}

// Collision and store of one node (see collide_node).
template <int LAT, class Real, class Store, bool DIAG, bool EXT = false, bool SR = false>
__device__ __forceinline__ void update_node(const StepArgs& a, const RowPos& p, Store* __restrict__ dst,
                                            const Store (&raw)[Lat<LAT>::Q],
                                            const Store (&raw_sc)[5], double (&v)[kDiagSlots]) {
    constexpr int D = Lat<LAT>::D;
    constexpr int Q = Lat<LAT>::Q;
    const Geometry& g = a.geo;
    Real m[Q], sc[5];
    collide_node<LAT, Real, Store, DIAG, EXT>(a, p, raw, raw_sc, v, m, sc);
    if (p.active) {
        Store* __restrict__ out = dst + p.row;
        if constexpr (std::is_same_v<Store, _Float16> && SR) {
            const uint32_t key = sr_node_key(a, p);
            static_for<Q>([&](auto aa) {
                constexpr int A = decltype(aa)::value;
                constexpr int slot = LAT == kD3Q15 ? A : Flow<D>::grid_of(A);
                st_stream(out + (int64_t)A * g.plane + p.x, half_sr(m[slot], key + sr_salt(A)));
            });
            if constexpr (LAT == kD2Q9D2Q5) {
                static_for<5>([&](auto aa) {
                    constexpr int A = decltype(aa)::value;
                    st_stream(out + (int64_t)(Q + A) * g.plane + p.x, half_sr(sc[A], key + sr_salt(Q + A)));
                });
            }
            return;
        }
        static_for<Q>([&](auto aa) {
            constexpr int A = decltype(aa)::value;
            constexpr int slot = LAT == kD3Q15 ? A : Flow<D>::grid_of(A);
            st_stream(out + (int64_t)A * g.plane + p.x, to_store<Store>(m[slot]));
        });
        if constexpr (LAT == kD2Q9D2Q5) {
            static_for<5>([&](auto aa) {
                constexpr int A = decltype(aa)::value;
                st_stream(out + (int64_t)(Q + A) * g.plane + p.x, to_store<Store>(sc[A]));
            });
        }
    }
}

// One step of ROWS rows per thread: all loads of all rows are issued before
// the first collision, so a wave keeps ROWS times the bytes in flight.
template <int LAT, class Real, class Store, bool DIAG, bool XWALL, int ROWS, bool EXT, bool SR = false>
__global__ void __launch_bounds__(kMaxBlock) casclb_step(const StepArgs a) {
    constexpr int D = Lat<LAT>::D;
    constexpr int Q = Lat<LAT>::Q;
    const Geometry& g = a.geo;
    const Store* __restrict__ src = reinterpret_cast<const Store*>(a.src);
    Store* __restrict__ dst = reinterpret_cast<Store*>(a.dst);

    static_assert(ROWS == 1 || ROWS == 2, "one or two rows per thread");
    // (two named rows rather than an array indexed by row: the compiler may
    // otherwise merge the two updates into a loop over a private-memory array)
    auto gather = [&](const RowPos& p, Store (&raw)[Q], Store (&raw_sc)[5]) {
        static_for<Q>([&](auto aa) {
            constexpr int A = decltype(aa)::value;
            constexpr int EX = Lat<LAT>::velocity(A, 0), EY = Lat<LAT>::velocity(A, 1), EZ = Lat<LAT>::velocity(A, 2);
            constexpr int slot = LAT == kD3Q15 ? A : Flow<D>::grid_of(A);
            raw[slot] = pull<EX, EY, EZ, XWALL>(src, g, p, A, Lat<LAT>::opposite(A));
        });
        if constexpr (LAT == kD2Q9D2Q5) {
            static_for<5>([&](auto aa) {
                constexpr int A = decltype(aa)::value;
                raw_sc[A] = pull<d2q5_velocity(A, 0), d2q5_velocity(A, 1), 0, XWALL>(src, g, p, Q + A,
                                                                                    Q + d2q5_opposite(A));
            });
        }
    };
    const RowPos p0 = row_position(g, 0);
    Store raw0[Q], raw0_sc[5];
    gather(p0, raw0, raw0_sc);
    double v[kDiagSlots] = {};
    if constexpr (ROWS == 2) {
        const RowPos p1 = row_position(g, 1);
        Store raw1[Q], raw1_sc[5];
        gather(p1, raw1, raw1_sc);
        update_node<LAT, Real, Store, DIAG, EXT, SR>(a, p0, dst, raw0, raw0_sc, v);
        update_node<LAT, Real, Store, DIAG, EXT, SR>(a, p1, dst, raw1, raw1_sc, v);
    } else {
        update_node<LAT, Real, Store, DIAG, EXT, SR>(a, p0, dst, raw0, raw0_sc, v);
    }
    if constexpr (DIAG) block_sum(v, a.partials + logical_block(g) * kDiagSlots);
}

// ---------------------------------------------------------------------------
// 16-bit storage, two x-adjacent nodes per thread
// ---------------------------------------------------------------------------
// With 2-byte populations a wave of one-node threads moves 128 bytes per load
// instruction.  Here thread t of a row updates nodes 2t and 2t+1 and reads
// and writes each population plane as aligned 32-bit words (word t holds
// nodes 2t, 2t+1): a population pulled along x (e_x = +-1) needs the high
// half of one word and the low half of the next, so it takes two word loads,
// the others one.  Needs nx even, x periodic, an even plane stride and 4-byte
// aligned buffers (checked by the host).  The arithmetic per node is
// collide_node's, so results are bit-identical to one node per thread.
struct PairPos {
    RowPos n0, n1;           // the two nodes (x = 2t, 2t + 1)
    uint32_t t, tm, tp;      // word index in the row and its periodic neighbours
    int64_t row_words;       // row / 2
};

__device__ __forceinline__ PairPos pair_position(const Geometry& g) {
    PairPos q;
    const uint32_t lb = logical_block(g);
    const uint32_t row0 = g.div_xb.div(lb);
    const int xb = (int)(lb - row0 * (uint32_t)g.x_blocks);
    const bool row_ok = row0 < (uint32_t)g.nrows;
    const uint32_t row = row_ok ? row0 : (uint32_t)g.nrows - 1;
    const uint32_t z = g.div_ny.div(row);
    const int words = g.nx >> 1;
    const int t = xb * (int)blockDim.x + (int)threadIdx.x;
    const bool active = row_ok && t < words;
    const int tc = active ? t : words - 1;
    q.t = (uint32_t)tc;
    q.tm = (uint32_t)(tc == 0 ? words - 1 : tc - 1);
    q.tp = (uint32_t)(tc == words - 1 ? 0 : tc + 1);
    q.row_words = (int64_t)words * row;
    RowPos p;
    p.y = (int)(row - z * (uint32_t)g.ny);
    p.z = (int)z;
    p.row = (int64_t)g.nx * row;
    p.active = active;
    p.x = (uint32_t)(2 * tc);
    p.xm = p.x == 0 ? (uint32_t)g.nx - 1 : p.x - 1;
    p.xp = p.x + 1;
    p.node = p.row + p.x;
    q.n0 = p;
    p.x += 1;
    p.xm = p.x - 1;
    p.xp = p.x == (uint32_t)g.nx - 1 ? 0 : p.x + 1;
    p.node += 1;
    q.n1 = p;
    return q;
}

__device__ __forceinline__ _Float16 half_lo(uint32_t w) { return __builtin_bit_cast(_Float16, (uint16_t)w); }
__device__ __forceinline__ _Float16 half_hi(uint32_t w) {
    return __builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

// The pull (eq. 22b, halfway bounce-back at y / z walls) of population
// `plane_self` with velocity (EX, EY, EZ) for both nodes of the pair.
template <int EX, int EY, int EZ>
__device__ __forceinline__ void pull_pair(const uint32_t* __restrict__ src, const Geometry& g, const PairPos& q,
                                          int plane_self, int plane_opp, _Float16& v0, _Float16& v1) {
    const RowPos& p = q.n0;
    bool wall = false;
    int sy = p.y - EY, sz = p.z - EZ;
    if constexpr (EY != 0) {
        if (sy < 0) { wall |= g.bb[1] != 0; sy += g.ny; }
        if (sy >= g.ny) { wall |= g.bb[1] != 0; sy -= g.ny; }
    }
    if constexpr (EZ != 0) {
        if (sz < 0) { wall |= g.bb[2] != 0; sz += g.nz; }
        if (sz >= g.nz) { wall |= g.bb[2] != 0; sz -= g.nz; }
    }
    const int64_t half_plane = g.plane >> 1;
    const int64_t words = g.nx >> 1;
    const uint32_t* own = src + (int64_t)plane_opp * half_plane + q.row_words;   // bounce-back: same nodes
    const uint32_t* base =
        wall ? own : src + (int64_t)plane_self * half_plane + words * ((int64_t)sy + (int64_t)g.ny * sz);
    // ordinary (temporal) word loads: the words next to a wave's range, which the
    // neighbouring wave also reads, then stay in L2 longer (about 1% faster on the
    // 256^3 duct than non-temporal loads; the stores stay non-temporal)
    if constexpr (EX == 0) {
        const uint32_t w = base[q.t];
        v0 = half_lo(w);
        v1 = half_hi(w);
    } else {
        // e_x = +1: nodes 2t, 2t+1 pull from 2t-1, 2t (high half of word t-1,
        // low half of word t); e_x = -1: from 2t+1, 2t+2 (high half of word t,
        // low half of word t+1); at a wall both take word t of `own`
        const uint32_t ia = wall ? q.t : (EX > 0 ? q.tm : q.t);
        const uint32_t ib = wall ? q.t : (EX > 0 ? q.t : q.tp);
        const uint32_t wa = base[ia];
        const uint32_t wb = base[ib];
        v0 = wall ? half_lo(wa) : half_hi(wa);
        v1 = wall ? half_hi(wb) : half_lo(wb);
    }
}

__device__ __forceinline__ uint32_t pack_halves(float lo, float hi) {
    const uint16_t a = __builtin_bit_cast(uint16_t, static_cast<_Float16>(lo));
    const uint16_t b = __builtin_bit_cast(uint16_t, static_cast<_Float16>(hi));
    return (uint32_t)a | ((uint32_t)b << 16);
}

template <int LAT, bool DIAG, bool EXT, bool SR>
__global__ void __launch_bounds__(kMaxBlock) casclb_step_xpair(const StepArgs a) {
    using Real = float;
    using Store = _Float16;
    constexpr int D = Lat<LAT>::D;
    constexpr int Q = Lat<LAT>::Q;
    const Geometry& g = a.geo;
    const uint32_t* __restrict__ src = reinterpret_cast<const uint32_t*>(a.src);
    uint32_t* __restrict__ dst = reinterpret_cast<uint32_t*>(a.dst);
    const PairPos q = pair_position(g);
    Store raw0[Q], raw1[Q], raw0_sc[5], raw1_sc[5];
    static_for<Q>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        constexpr int EX = Lat<LAT>::velocity(A, 0), EY = Lat<LAT>::velocity(A, 1), EZ = Lat<LAT>::velocity(A, 2);
        constexpr int slot = LAT == kD3Q15 ? A : Flow<D>::grid_of(A);
        pull_pair<EX, EY, EZ>(src, g, q, A, Lat<LAT>::opposite(A), raw0[slot], raw1[slot]);
    });
    if constexpr (LAT == kD2Q9D2Q5) {
        static_for<5>([&](auto aa) {
            constexpr int A = decltype(aa)::value;
            pull_pair<d2q5_velocity(A, 0), d2q5_velocity(A, 1), 0>(src, g, q, Q + A, Q + d2q5_opposite(A),
                                                                  raw0_sc[A], raw1_sc[A]);
        });
    }
    double v[kDiagSlots] = {};
    Real m0[Q], m1[Q], sc0[5], sc1[5];
    collide_node<LAT, Real, Store, DIAG, EXT>(a, q.n0, raw0, raw0_sc, v, m0, sc0);
    collide_node<LAT, Real, Store, DIAG, EXT>(a, q.n1, raw1, raw1_sc, v, m1, sc1);
    // the rounding is a template choice: a kernel that carries both store paths
    // schedules its loads worse (measured 43.6 against 49.2 GLUPS on the duct)
    if (SR && q.n0.active) {
        const int64_t half_plane = g.plane >> 1;
        uint32_t* __restrict__ out = dst + q.row_words + q.t;
        const uint32_t key0 = sr_node_key(a, q.n0), key1 = sr_node_key(a, q.n1);
        static_for<Q>([&](auto aa) {
            constexpr int A = decltype(aa)::value;
            constexpr int slot = LAT == kD3Q15 ? A : Flow<D>::grid_of(A);
            st_stream(out + (int64_t)A * half_plane,
                      pack_halves_sr(m0[slot], m1[slot], key0 + sr_salt(A), key1 + sr_salt(A)));
        });
        if constexpr (LAT == kD2Q9D2Q5) {
            static_for<5>([&](auto aa) {
                constexpr int A = decltype(aa)::value;
                st_stream(out + (int64_t)(Q + A) * half_plane,
                          pack_halves_sr(sc0[A], sc1[A], key0 + sr_salt(Q + A), key1 + sr_salt(Q + A)));
            });
        }
    } else if (!SR && q.n0.active) {
        const int64_t half_plane = g.plane >> 1;
        uint32_t* __restrict__ out = dst + q.row_words + q.t;
        static_for<Q>([&](auto aa) {
            constexpr int A = decltype(aa)::value;
            constexpr int slot = LAT == kD3Q15 ? A : Flow<D>::grid_of(A);
            st_stream(out + (int64_t)A * half_plane, pack_halves(m0[slot], m1[slot]));
        });
        if constexpr (LAT == kD2Q9D2Q5) {
            static_for<5>([&](auto aa) {
                constexpr int A = decltype(aa)::value;
                st_stream(out + (int64_t)(Q + A) * half_plane, pack_halves(sc0[A], sc1[A]));
            });
        }
    }
    if constexpr (DIAG) block_sum(v, a.partials + logical_block(g) * kDiagSlots);
}

// Deterministic second pass: sums `blocks` partial records of kDiagSlots in
// a fixed order into out[0..kDiagSlots).
__global__ void __launch_bounds__(256) casclb_reduce_partials(const double* __restrict__ partials, int64_t blocks,
                                                              double* __restrict__ out) {
    __shared__ double red[256][kDiagSlots];
    double acc[kDiagSlots] = {};
    for (int64_t b = threadIdx.x; b < blocks; b += 256)
        for (int c = 0; c < kDiagSlots; ++c) acc[c] += partials[b * kDiagSlots + c];
    for (int c = 0; c < kDiagSlots; ++c) red[threadIdx.x][c] = acc[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < kDiagSlots; ++c) red[threadIdx.x][c] += red[threadIdx.x + s][c];
        __syncthreads();
    }
    if (threadIdx.x < kDiagSlots) out[threadIdx.x] = red[0][threadIdx.x];
}

// ---------------------------------------------------------------------------
// initial equilibrium
// ---------------------------------------------------------------------------
// Equilibrium of (rho = rho0 + drho, u, phi): the flow populations as
// deviations from the rest populations w_a rho0 (ABI order) and the scalar
// populations (D2Q9+D2Q5).
template <int LAT, class Real>
__device__ __forceinline__ void equilibrium_node(Real drho, Real rho, const Real (&u)[3], Real phi,
                                                 Real (&f)[Lat<LAT>::Q], Real (&g)[5]) {
    constexpr int D = Lat<LAT>::D;
    constexpr int Q = Lat<LAT>::Q;
    if constexpr (LAT == kD3Q15) {
        // second-order equilibrium w rho (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u), as a deviation from w rho0
        const Real uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        static_for<Q>([&](auto aa) {
            constexpr int A = decltype(aa)::value;
            const Real eu = Real(D3Q15::velocity(A, 0)) * u[0] + Real(D3Q15::velocity(A, 1)) * u[1] +
                            Real(D3Q15::velocity(A, 2)) * u[2];
            const Real dev = drho + rho * (Real(3) * eu + Real(4.5) * eu * eu - Real(1.5) * uu);
            f[A] = Real(D3Q15::weight(A)) * dev;
        });
    } else {
        static_for<Q>([&](auto aa) {
            constexpr int A = decltype(aa)::value;
            const int e[3] = {Flow<D>::velocity(A, 0), Flow<D>::velocity(A, 1), Flow<D>::velocity(A, 2)};
            f[A] = equilibrium_deviation<D, Real>(e, drho, rho, u);
        });
    }
    if constexpr (LAT == kD2Q9D2Q5) {
        const Real ux = u[0], uy = u[1], third = Real(1) / Real(3);
        g[0] = phi * (third - ux * ux - uy * uy);
        g[1] = Real(0.5) * phi * (third + ux * ux + ux);
        g[2] = Real(0.5) * phi * (third + uy * uy + uy);
        g[3] = Real(0.5) * phi * (third + ux * ux - ux);
        g[4] = Real(0.5) * phi * (third + uy * uy - uy);
    }
}

template <int LAT, class Real, class Store>
__global__ void __launch_bounds__(256) casclb_init(Geometry g, void* buf, const double* rho_in, const double* u_in,
                                                   const double* phi_in, double rho0, int64_t n_nodes) {
    constexpr int D = Lat<LAT>::D;
    constexpr int Q = Lat<LAT>::Q;
    const RowPos p = row_position(g);
    if (!p.active) return;
    Store* out = reinterpret_cast<Store*>(buf);
    const Real rho = rho_in ? Real(rho_in[p.node]) : Real(rho0);
    const Real drho = rho_in ? Real(rho_in[p.node] - rho0) : Real(0);
    Real u[3] = {Real(0), Real(0), Real(0)};
    if (u_in)
        for (int i = 0; i < D; ++i) u[i] = Real(u_in[(int64_t)i * n_nodes + p.node]);
    const Real phi = phi_in ? Real(phi_in[p.node]) : Real(0);
    Real f[Q], sc[5];
    equilibrium_node<LAT, Real>(drho, rho, u, phi, f, sc);
    static_for<Q>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        out[(int64_t)A * g.plane + p.node] = to_store<Store>(f[A]);
    });
    if constexpr (LAT == kD2Q9D2Q5)
        for (int A = 0; A < 5; ++A) out[(int64_t)(Q + A) * g.plane + p.node] = to_store<Store>(sc[A]);
}

// Moment reset of the stored state: every node's populations are shifted by
// the equilibrium of the target (rho_in, u_in, phi_in) minus the equilibrium
// of their own moments (rho = rho0 + sum of the flow deviations, u = their
// first moment / rho, phi = sum of the scalar populations), so the node takes
// the target's moments and keeps its non-equilibrium part f - f_eq.
template <int LAT, class Real, class Store>
__global__ void __launch_bounds__(256) casclb_reset(Geometry g, void* buf, const double* rho_in, const double* u_in,
                                                    const double* phi_in, double rho0, int64_t n_nodes) {
    constexpr int D = Lat<LAT>::D;
    constexpr int Q = Lat<LAT>::Q;
    const RowPos p = row_position(g);
    if (!p.active) return;
    Store* st = reinterpret_cast<Store*>(buf);
    Real f[Q], sc[5];
    Real drho = Real(0), j[3] = {Real(0), Real(0), Real(0)}, phi = Real(0);
    static_for<Q>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        f[A] = to_real<Real>(st[(int64_t)A * g.plane + p.node]);
        drho += f[A];
        static_for<D>([&](auto ax) {
            constexpr int AX = decltype(ax)::value;
            constexpr int E = Lat<LAT>::velocity(A, AX);
            if constexpr (E != 0) j[AX] += Real(E) * f[A];
        });
    });
    if constexpr (LAT == kD2Q9D2Q5) {
        for (int A = 0; A < 5; ++A) {
            sc[A] = to_real<Real>(st[(int64_t)(Q + A) * g.plane + p.node]);
            phi += sc[A];
        }
    }
    const Real rho = Real(rho0) + drho;
    const Real u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    Real fc[Q], gc[5];
    equilibrium_node<LAT, Real>(drho, rho, u, phi, fc, gc);
    const Real rho_t = Real(rho_in[p.node]);
    const Real drho_t = Real(rho_in[p.node] - rho0);
    Real ut[3] = {Real(0), Real(0), Real(0)};
    for (int i = 0; i < D; ++i) ut[i] = Real(u_in[(int64_t)i * n_nodes + p.node]);
    const Real phi_t = phi_in ? Real(phi_in[p.node]) : Real(0);
    Real ft[Q], gt[5];
    equilibrium_node<LAT, Real>(drho_t, rho_t, ut, phi_t, ft, gt);
    static_for<Q>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        st[(int64_t)A * g.plane + p.node] = to_store<Store>(f[A] - fc[A] + ft[A]);
    });
    if constexpr (LAT == kD2Q9D2Q5)
        for (int A = 0; A < 5; ++A)
            st[(int64_t)(Q + A) * g.plane + p.node] = to_store<Store>(sc[A] - gc[A] + gt[A]);
}

// ---------------------------------------------------------------------------
// macroscopic readout (pull + moments), float64 outputs
// ---------------------------------------------------------------------------
template <int LAT, class Real, class Store>
__global__ void __launch_bounds__(256) casclb_moments(StepArgs a, int kind, double* rho_out, double* u_out,
                                                      double* phi_out, int64_t n_nodes) {
    constexpr int D = Lat<LAT>::D;
    constexpr int Q = Lat<LAT>::Q;
    const Geometry& g = a.geo;
    const RowPos p = row_position(g);
    if (!p.active) return;
    const Store* src = reinterpret_cast<const Store*>(a.src);
    if constexpr (LAT == kD3Q15) {
        Real drho = Real(0), j[3] = {Real(0), Real(0), Real(0)};
        static_for<Q>([&](auto aa) {
            constexpr int A = decltype(aa)::value;
            constexpr int EX = D3Q15::velocity(A, 0), EY = D3Q15::velocity(A, 1), EZ = D3Q15::velocity(A, 2);
            const Real v = to_real<Real>(pull<EX, EY, EZ, true>(src, g, p, A, D3Q15::opposite(A)));
            drho += v;
            j[0] += Real(EX) * v;
            j[1] += Real(EY) * v;
            j[2] += Real(EZ) * v;
        });
        Real fb[3];
        node_force<3, Real>(a, p, fb);
        const Real rho = Real(a.rho0) + drho;
        if (rho_out) rho_out[p.node] = (double)rho;
        if (u_out)
            for (int i = 0; i < 3; ++i) {
                const Real ji = kind == 1 ? j[i] + Real(0.5) * Real(a.f_pre) * fb[i] : j[i];
                u_out[(int64_t)i * n_nodes + p.node] = (double)(ji / rho);
            }
        return;
    } else {
    Real m[Q];
    gather_flow<D, true, Real, Store>(src, g, p, m);
    if constexpr (D == 2) {
        if (a.ext) moving_walls<Real>(a, p, m);
    }
    raw_moments<D>(m);
    Real fb[3];
    node_force<D, Real>(a, p, fb);
    const Real rho = Real(a.rho0) + m[0];
    if (rho_out) rho_out[p.node] = (double)rho;
    if (u_out) {
        for (int i = 0; i < D; ++i) {
            const int slot = i == 0 ? 1 : (i == 1 ? 3 : 9);
            Real j = m[slot];
            Real r = rho;
            if (kind == 1) {
                j = j + Real(0.5) * Real(a.f_pre) * fb[i];
                if (i == 0 && a.lorentz != 0.0) r = rho + Real(0.5) * Real(a.lorentz);   // implicit half step
            }
            u_out[(int64_t)i * n_nodes + p.node] = (double)(j / r);
        }
    }
    if constexpr (LAT == kD2Q9D2Q5) {
        if (phi_out) {
            Real sc[5];
            gather_scalar<true, Real, Store>(src, Q, g, p, sc);
            Real sb = Real(a.source);
            if (a.source_field) sb = reinterpret_cast<const Real*>(a.source_field)[p.node];
            Real spre = Real(a.s_pre) * sb;
            if (a.ext) {
                // the step's scalar source and wall rule (heating from the half-forced velocity)
                const Real uh[3] = {(m[1] + Real(0.5) * Real(a.f_pre) * fb[0]) / rho,
                                    (m[3] + Real(0.5) * Real(a.f_pre) * fb[1]) / rho, Real(0)};
                const Real sr = Real(a.heat) * strain_rate_squared<Real>(a, m[2], m[6], m[4], rho, uh);
                spre += sr;
                scalar_walls<Real>(a, p, Real(a.s_tot) * sb + sr, sc);
            }
            Real phi = sc[0] + (sc[1] + sc[3]) + (sc[2] + sc[4]);
            if (kind == 1) phi = phi + Real(0.5) * spre;
            phi_out[p.node] = (double)phi;
        }
    }
    }
}

// ---------------------------------------------------------------------------
// totals of the stored state (no pull), float64
// ---------------------------------------------------------------------------
template <int LAT, class Real, class Store>
__global__ void __launch_bounds__(256) casclb_totals(Geometry g, const void* buf, double* partials) {
    constexpr int Q = Lat<LAT>::Q;
    const RowPos p = row_position(g);
    const Store* s = reinterpret_cast<const Store*>(buf);
    double v[kDiagSlots] = {};
    if (p.active) {
        static_for<Q>([&](auto aa) {
            constexpr int A = decltype(aa)::value;
            const double f = (double)to_real<Real>(s[(int64_t)A * g.plane + p.node]);
            v[0] += f;
            v[1] += Lat<LAT>::velocity(A, 0) * f;
            v[2] += Lat<LAT>::velocity(A, 1) * f;
            v[3] += Lat<LAT>::velocity(A, 2) * f;
        });
        if constexpr (LAT == kD2Q9D2Q5)
            for (int A = 0; A < 5; ++A) v[4] += (double)to_real<Real>(s[(int64_t)(Q + A) * g.plane + p.node]);
    }
    block_sum(v, partials + logical_block(g) * kDiagSlots);
}

// The same totals with a bounded number of partial records: block b sums the
// nodes of logical blocks b, b + records, b + 2 records, ... (grid-stride), so
// the partial records fit a fixed scratch area whatever the lattice size.
template <int LAT, class Real, class Store>
__global__ void __launch_bounds__(256) casclb_totals_strided(Geometry g, const void* buf, double* partials,
                                                              int64_t records) {
    constexpr int Q = Lat<LAT>::Q;
    const Store* s = reinterpret_cast<const Store*>(buf);
    double v[kDiagSlots] = {};
    for (int64_t lb = blockIdx.x; lb < g.grid_blocks; lb += records) {
        const RowPos p = row_position_at(g, (uint32_t)lb);
        if (!p.active) continue;
        static_for<Q>([&](auto aa) {
            constexpr int A = decltype(aa)::value;
            const double f = (double)to_real<Real>(s[(int64_t)A * g.plane + p.node]);
            v[0] += f;
            v[1] += Lat<LAT>::velocity(A, 0) * f;
            v[2] += Lat<LAT>::velocity(A, 1) * f;
            v[3] += Lat<LAT>::velocity(A, 2) * f;
        });
        if constexpr (LAT == kD2Q9D2Q5)
            for (int A = 0; A < 5; ++A) v[4] += (double)to_real<Real>(s[(int64_t)(Q + A) * g.plane + p.node]);
    }
    block_sum(v, partials + (int64_t)blockIdx.x * kDiagSlots);
}

// out[0..5) = mass (rest mass `mass_offset` plus the deviations), momentum, scalar.
__global__ void casclb_totals_finish(const double* __restrict__ sums, double mass_offset, double* __restrict__ out) {
    if (threadIdx.x == 0) {
        out[0] = mass_offset + sums[0];
        for (int k = 1; k < 5; ++k) out[k] = sums[k];
    }
}

// ---------------------------------------------------------------------------
// conversions between storage and float64 (host transfers go through these)
// ---------------------------------------------------------------------------
template <class Store>
__global__ void casclb_plane_to_f64(const Store* __restrict__ in, double* __restrict__ out, int64_t n, double offset) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)in[i] + offset;
}

template <class Store>
__global__ void casclb_plane_from_f64(const double* __restrict__ in, Store* __restrict__ out, int64_t n, double offset) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = static_cast<Store>(in[i] - offset);
}

template <class Store>
__global__ void casclb_box_to_f64(const Store* __restrict__ in, double* __restrict__ out, Geometry g, int64_t lo0,
                                  int64_t lo1, int64_t lo2, int64_t e0, int64_t e1, int64_t e2, double offset) {
    const int64_t bn = e0 * e1 * e2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bn; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t bx = i % e0, by = (i / e0) % e1, bz = i / (e0 * e1);
        const int64_t x = ((lo0 + bx) % g.nx + g.nx) % g.nx;
        const int64_t y = ((lo1 + by) % g.ny + g.ny) % g.ny;
        const int64_t z = ((lo2 + bz) % g.nz + g.nz) % g.nz;
        out[i] = (double)in[x + g.nx * (y + g.ny * z)] + offset;
    }
}

// field conversion from float64 into the arithmetic type, [c][n] -> [c][plane]
template <class Real>
__global__ void casclb_field_from_f64(const double* __restrict__ in, Real* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = static_cast<Real>(in[i]);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Streaming copy: each thread moves 4 x 16 bytes, all four loads issued
// before the stores; one block covers 16 KiB.
constexpr int kCopyUnroll = 4;
__global__ void __launch_bounds__(256) casclb_copy(const u32x4* __restrict__ in, u32x4* __restrict__ out, int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * (256 * kCopyUnroll) + threadIdx.x;
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int k = 0; k < kCopyUnroll; ++k) {
        const int64_t i = base + k * 256;
        if (i < n) v[k] = __builtin_nontemporal_load(in + i);
    }
#pragma unroll
    for (int k = 0; k < kCopyUnroll; ++k) {
        const int64_t i = base + k * 256;
        if (i < n) __builtin_nontemporal_store(v[k], out + i);
    }
}

// Fill of a buffer with one 16-bit pattern (the debug poison of lb_step).
__global__ void __launch_bounds__(256) casclb_fill_u16(uint16_t* __restrict__ out, int64_t n, uint16_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = value;
}

// Streaming kernels for the bandwidth ceiling: read-only, write-only and copy
// over n vectors of V (8- or 16-byte) elements, non-temporal, 4 vectors per
// thread per pass.  blocks_fixed = 0: one pass, each block covers 4 x 256
// vectors; otherwise a grid-stride loop over that many blocks.  The read kernel
// folds what it loads into one vector per block (out[block]) so the loads
// cannot be dropped.
template <class V>
__global__ void __launch_bounds__(256) casclb_stream_read(const V* __restrict__ in, V* __restrict__ out, int64_t n) {
    V acc = {};
    const int64_t step = (int64_t)gridDim.x * 256 * kCopyUnroll;
    for (int64_t base = (int64_t)blockIdx.x * (256 * kCopyUnroll) + threadIdx.x; base < n; base += step) {
        V v[kCopyUnroll];
#pragma unroll
        for (int k = 0; k < kCopyUnroll; ++k) {
            const int64_t i = base + k * 256;
            v[k] = i < n ? __builtin_nontemporal_load(in + i) : V{};
        }
#pragma unroll
        for (int k = 0; k < kCopyUnroll; ++k) acc ^= v[k];
    }
    // one value per block: xor over the block's lanes via LDS
    __shared__ V red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] ^= red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

template <class V>
__global__ void __launch_bounds__(256) casclb_stream_write(V* __restrict__ out, int64_t n) {
    const int64_t step = (int64_t)gridDim.x * 256 * kCopyUnroll;
    for (int64_t base = (int64_t)blockIdx.x * (256 * kCopyUnroll) + threadIdx.x; base < n; base += step) {
#pragma unroll
        for (int k = 0; k < kCopyUnroll; ++k) {
            const int64_t i = base + k * 256;
            if (i < n) __builtin_nontemporal_store(V{}, out + i);
        }
    }
}

template <class V>
__global__ void __launch_bounds__(256) casclb_stream_copy(const V* __restrict__ in, V* __restrict__ out, int64_t n) {
    const int64_t step = (int64_t)gridDim.x * 256 * kCopyUnroll;
    for (int64_t base = (int64_t)blockIdx.x * (256 * kCopyUnroll) + threadIdx.x; base < n; base += step) {
        V v[kCopyUnroll];
#pragma unroll
        for (int k = 0; k < kCopyUnroll; ++k) {
            const int64_t i = base + k * 256;
            if (i < n) v[k] = __builtin_nontemporal_load(in + i);
        }
#pragma unroll
        for (int k = 0; k < kCopyUnroll; ++k) {
            const int64_t i = base + k * 256;
            if (i < n) __builtin_nontemporal_store(v[k], out + i);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
template <int LAT, class Real, class Store, bool EXT, bool SR>
hipError_t launch_step_e(const StepArgs& a, int block, bool diag, hipStream_t s) {
    const dim3 grid((unsigned)a.geo.grid_blocks), blk((unsigned)block);
    const bool xwall = a.geo.bb[0] != 0;
    if constexpr (std::is_same_v<Store, _Float16>) {
        if (a.geo.xpair) {
            if (xwall) return hipErrorInvalidValue;
            if (diag)
                hipLaunchKernelGGL((casclb_step_xpair<LAT, true, EXT, SR>), grid, blk, 0, s, a);
            else
                hipLaunchKernelGGL((casclb_step_xpair<LAT, false, EXT, SR>), grid, blk, 0, s, a);
            return hipGetLastError();
        }
    }
    if (xwall) {
        // walls across x: the per-lane wall handling, one row per thread
        if (diag)
            hipLaunchKernelGGL((casclb_step<LAT, Real, Store, true, true, 1, EXT, SR>), grid, blk, 0, s, a);
        else
            hipLaunchKernelGGL((casclb_step<LAT, Real, Store, false, true, 1, EXT, SR>), grid, blk, 0, s, a);
    } else if (a.geo.rows == 2) {
        if (diag)
            hipLaunchKernelGGL((casclb_step<LAT, Real, Store, true, false, 2, EXT, SR>), grid, blk, 0, s, a);
        else
            hipLaunchKernelGGL((casclb_step<LAT, Real, Store, false, false, 2, EXT, SR>), grid, blk, 0, s, a);
    } else {
        if (diag)
            hipLaunchKernelGGL((casclb_step<LAT, Real, Store, true, false, 1, EXT, SR>), grid, blk, 0, s, a);
        else
            hipLaunchKernelGGL((casclb_step<LAT, Real, Store, false, false, 1, EXT, SR>), grid, blk, 0, s, a);
    }
    return hipGetLastError();
}

// Stochastic rounding exists for float16 storage only.
template <int LAT, class Real, class Store, bool EXT>
hipError_t launch_step_r(const StepArgs& a, int block, bool diag, hipStream_t s) {
    if constexpr (std::is_same_v<Store, _Float16>) {
        if (a.sr) return launch_step_e<LAT, Real, Store, EXT, true>(a, block, diag, s);
    }
    return launch_step_e<LAT, Real, Store, EXT, false>(a, block, diag, s);
}

// EXT kernels (moving walls, fixed-value scalar walls, viscous heating) exist
// for the 2D lattices only; the API rejects those settings on D3Q27.
template <int LAT, class Real, class Store>
hipError_t launch_step_t(const StepArgs& a, int block, bool diag, hipStream_t s) {
    if constexpr (Lat<LAT>::D == 2) {
        if (a.ext) return launch_step_r<LAT, Real, Store, true>(a, block, diag, s);
    }
    return launch_step_r<LAT, Real, Store, false>(a, block, diag, s);
}

}  // namespace

hipError_t launch_step(int lat, int storage, const StepArgs& a, int block, bool diag, hipStream_t s) {
    switch (lat * 3 + storage) {
        case kD2Q9 * 3 + kF64: return launch_step_t<kD2Q9, double, double>(a, block, diag, s);
        case kD2Q9 * 3 + kF32Dev: return launch_step_t<kD2Q9, float, float>(a, block, diag, s);
        case kD2Q9 * 3 + kF16Dev: return launch_step_t<kD2Q9, float, _Float16>(a, block, diag, s);
        case kD2Q9D2Q5 * 3 + kF64: return launch_step_t<kD2Q9D2Q5, double, double>(a, block, diag, s);
        case kD2Q9D2Q5 * 3 + kF32Dev: return launch_step_t<kD2Q9D2Q5, float, float>(a, block, diag, s);
        case kD2Q9D2Q5 * 3 + kF16Dev: return launch_step_t<kD2Q9D2Q5, float, _Float16>(a, block, diag, s);
        case kD3Q27 * 3 + kF64: return launch_step_t<kD3Q27, double, double>(a, block, diag, s);
        case kD3Q27 * 3 + kF32Dev: return launch_step_t<kD3Q27, float, float>(a, block, diag, s);
        case kD3Q27 * 3 + kF16Dev: return launch_step_t<kD3Q27, float, _Float16>(a, block, diag, s);
        case kD3Q15 * 3 + kF64: return launch_step_t<kD3Q15, double, double>(a, block, diag, s);
        case kD3Q15 * 3 + kF32Dev: return launch_step_t<kD3Q15, float, float>(a, block, diag, s);
        case kD3Q15 * 3 + kF16Dev: return launch_step_t<kD3Q15, float, _Float16>(a, block, diag, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(const double* partials, int64_t blocks, double* out, hipStream_t s) {
    hipLaunchKernelGGL(casclb_reduce_partials, dim3(1), dim3(256), 0, s, partials, blocks, out);
    return hipGetLastError();
}

#define CASCLB_DISPATCH3(fn, ...)                                                          \
    switch (lat * 3 + storage) {                                                           \
        case kD2Q9 * 3 + kF64: fn<kD2Q9, double, double> __VA_ARGS__; break;               \
        case kD2Q9 * 3 + kF32Dev: fn<kD2Q9, float, float> __VA_ARGS__; break;              \
        case kD2Q9 * 3 + kF16Dev: fn<kD2Q9, float, _Float16> __VA_ARGS__; break;           \
        case kD2Q9D2Q5 * 3 + kF64: fn<kD2Q9D2Q5, double, double> __VA_ARGS__; break;       \
        case kD2Q9D2Q5 * 3 + kF32Dev: fn<kD2Q9D2Q5, float, float> __VA_ARGS__; break;      \
        case kD2Q9D2Q5 * 3 + kF16Dev: fn<kD2Q9D2Q5, float, _Float16> __VA_ARGS__; break;   \
        case kD3Q27 * 3 + kF64: fn<kD3Q27, double, double> __VA_ARGS__; break;             \
        case kD3Q27 * 3 + kF32Dev: fn<kD3Q27, float, float> __VA_ARGS__; break;            \
        case kD3Q27 * 3 + kF16Dev: fn<kD3Q27, float, _Float16> __VA_ARGS__; break;         \
        case kD3Q15 * 3 + kF64: fn<kD3Q15, double, double> __VA_ARGS__; break;             \
        case kD3Q15 * 3 + kF32Dev: fn<kD3Q15, float, float> __VA_ARGS__; break;            \
        case kD3Q15 * 3 + kF16Dev: fn<kD3Q15, float, _Float16> __VA_ARGS__; break;         \
        default: return hipErrorInvalidValue;                                              \
    }

namespace {
template <int LAT, class Real, class Store>
void init_t(const Geometry& g, void* buf, const double* rho, const double* u, const double* phi, double rho0,
            int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((casclb_init<LAT, Real, Store>), dim3((unsigned)g.grid_blocks), dim3(256), 0, s, g, buf, rho,
                       u, phi, rho0, n);
}
template <int LAT, class Real, class Store>
void reset_t(const Geometry& g, void* buf, const double* rho, const double* u, const double* phi, double rho0,
             int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((casclb_reset<LAT, Real, Store>), dim3((unsigned)g.grid_blocks), dim3(256), 0, s, g, buf, rho,
                       u, phi, rho0, n);
}
template <int LAT, class Real, class Store>
void moments_t(const StepArgs& a, int kind, double* rho, double* u, double* phi, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((casclb_moments<LAT, Real, Store>), dim3((unsigned)a.geo.grid_blocks), dim3(256), 0, s, a,
                       kind, rho, u, phi, n);
}
template <int LAT, class Real, class Store>
void totals_strided_t(const Geometry& g, const void* buf, double* partials, int64_t records, hipStream_t s) {
    hipLaunchKernelGGL((casclb_totals_strided<LAT, Real, Store>), dim3((unsigned)records), dim3(256), 0, s, g, buf,
                       partials, records);
}
template <int LAT, class Real, class Store>
void totals_t(const Geometry& g, const void* buf, double* partials, hipStream_t s) {
    hipLaunchKernelGGL((casclb_totals<LAT, Real, Store>), dim3((unsigned)g.grid_blocks), dim3(256), 0, s, g, buf,
                       partials);
}
}  // namespace

hipError_t launch_init(int lat, int storage, const Geometry& g256, void* buf, const double* rho, const double* u,
                       const double* phi, double rho0, int64_t n, hipStream_t s) {
    CASCLB_DISPATCH3(init_t, (g256, buf, rho, u, phi, rho0, n, s))
    return hipGetLastError();
}

hipError_t launch_reset(int lat, int storage, const Geometry& g256, void* buf, const double* rho, const double* u,
                        const double* phi, double rho0, int64_t n, hipStream_t s) {
    CASCLB_DISPATCH3(reset_t, (g256, buf, rho, u, phi, rho0, n, s))
    return hipGetLastError();
}

hipError_t launch_moments(int lat, int storage, const StepArgs& a256, int kind, double* rho, double* u, double* phi,
                          int64_t n, hipStream_t s) {
    CASCLB_DISPATCH3(moments_t, (a256, kind, rho, u, phi, n, s))
    return hipGetLastError();
}

hipError_t launch_totals(int lat, int storage, const Geometry& g256, const void* buf, double* partials,
                         hipStream_t s) {
    CASCLB_DISPATCH3(totals_t, (g256, buf, partials, s))
    return hipGetLastError();
}

static unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_totals_bounded(int lat, int storage, const Geometry& g256, const void* buf, double* scratch,
                                 int64_t records, double mass_offset, double* out5, hipStream_t s) {
    if (records < 1 || records > g256.grid_blocks) return hipErrorInvalidValue;
    CASCLB_DISPATCH3(totals_strided_t, (g256, buf, scratch, records, s))
    double* sums = scratch + records * kDiagSlots;
    hipLaunchKernelGGL(casclb_reduce_partials, dim3(1), dim3(256), 0, s, scratch, records, sums);
    hipLaunchKernelGGL(casclb_totals_finish, dim3(1), dim3(64), 0, s, sums, mass_offset, out5);
    return hipGetLastError();
}

hipError_t launch_plane_to_f64(int storage, const void* in, double* out, int64_t n, double offset, hipStream_t s) {
    switch (storage) {
        case kF64: hipLaunchKernelGGL(casclb_plane_to_f64<double>, dim3(grid_for(n)), dim3(256), 0, s, (const double*)in, out, n, offset); break;
        case kF32Dev: hipLaunchKernelGGL(casclb_plane_to_f64<float>, dim3(grid_for(n)), dim3(256), 0, s, (const float*)in, out, n, offset); break;
        case kF16Dev: hipLaunchKernelGGL(casclb_plane_to_f64<_Float16>, dim3(grid_for(n)), dim3(256), 0, s, (const _Float16*)in, out, n, offset); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_plane_from_f64(int storage, const double* in, void* out, int64_t n, double offset, hipStream_t s) {
    switch (storage) {
        case kF64: hipLaunchKernelGGL(casclb_plane_from_f64<double>, dim3(grid_for(n)), dim3(256), 0, s, in, (double*)out, n, offset); break;
        case kF32Dev: hipLaunchKernelGGL(casclb_plane_from_f64<float>, dim3(grid_for(n)), dim3(256), 0, s, in, (float*)out, n, offset); break;
        case kF16Dev: hipLaunchKernelGGL(casclb_plane_from_f64<_Float16>, dim3(grid_for(n)), dim3(256), 0, s, in, (_Float16*)out, n, offset); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_box_to_f64(int storage, const void* plane, double* out, const Geometry& g, const int64_t lo[3],
                             const int64_t ext[3], double offset, hipStream_t s) {
    const int64_t bn = ext[0] * ext[1] * ext[2];
    switch (storage) {
        case kF64: hipLaunchKernelGGL(casclb_box_to_f64<double>, dim3(grid_for(bn)), dim3(256), 0, s, (const double*)plane, out, g, lo[0], lo[1], lo[2], ext[0], ext[1], ext[2], offset); break;
        case kF32Dev: hipLaunchKernelGGL(casclb_box_to_f64<float>, dim3(grid_for(bn)), dim3(256), 0, s, (const float*)plane, out, g, lo[0], lo[1], lo[2], ext[0], ext[1], ext[2], offset); break;
        case kF16Dev: hipLaunchKernelGGL(casclb_box_to_f64<_Float16>, dim3(grid_for(bn)), dim3(256), 0, s, (const _Float16*)plane, out, g, lo[0], lo[1], lo[2], ext[0], ext[1], ext[2], offset); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_field_from_f64(bool f64, const double* in, void* out, int64_t n, hipStream_t s) {
    if (f64)
        hipLaunchKernelGGL(casclb_field_from_f64<double>, dim3(grid_for(n)), dim3(256), 0, s, in, (double*)out, n);
    else
        hipLaunchKernelGGL(casclb_field_from_f64<float>, dim3(grid_for(n)), dim3(256), 0, s, in, (float*)out, n);
    return hipGetLastError();
}

hipError_t launch_fill_u16(void* dst, size_t count, uint16_t value, hipStream_t s) {
    hipLaunchKernelGGL(casclb_fill_u16, dim3(grid_for((int64_t)count)), dim3(256), 0, s, (uint16_t*)dst,
                       (int64_t)count, value);
    return hipGetLastError();
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

namespace {
template <class V>
hipError_t launch_stream_t(void* dst, const void* src, size_t bytes, int mode, int64_t blocks_fixed, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / sizeof(V));
    int64_t blocks = blocks_fixed > 0 ? blocks_fixed : (n + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll);
    if (blocks < 1) blocks = 1;
    if (blocks > (1LL << 31) - 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), blk(256);
    if (mode == 0)
        hipLaunchKernelGGL(casclb_stream_copy<V>, grid, blk, 0, s, (const V*)src, (V*)dst, n);
    else if (mode == 1)
        hipLaunchKernelGGL(casclb_stream_read<V>, grid, blk, 0, s, (const V*)src, (V*)dst, n);
    else
        hipLaunchKernelGGL(casclb_stream_write<V>, grid, blk, 0, s, (V*)dst, n);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_stream(void* dst, const void* src, size_t bytes, int mode, int width, int64_t blocks,
                         hipStream_t s) {
    if (mode < 0 || mode > 2 || (width != 8 && width != 16)) return hipErrorInvalidValue;
    return width == 16 ? launch_stream_t<u32x4>(dst, src, bytes, mode, blocks, s)
                       : launch_stream_t<u32x2>(dst, src, bytes, mode, blocks, s);
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 16);
    int64_t blocks = (n + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll);
    if (blocks < 1) blocks = 1;
    if (blocks > (1LL << 31) - 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(casclb_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, n);
    return hipGetLastError();
}

}  // namespace casclb
