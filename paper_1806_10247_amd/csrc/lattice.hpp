// Per-node arithmetic of the cascaded (central-moment) LB update with
// symmetrized operator-split forcing, written for registers on gfx950.
//
// The flow lattices are tensor products of the one-dimensional three-velocity
// set {0, +1, -1}: D2Q9 and D3Q27.  A node's 9 or 27 values live in a
// register array in "grid order" k = i0 + 3 i1 + 9 i2.  For populations the
// digit i_a selects the velocity component along axis a (0 -> 0, 1 -> +1,
// 2 -> -1); for moments it is the power of that component.  Every transform
// is a product of one-dimensional 3x3 transforms applied as sweeps along the
// axes, so a full moment transform costs O(Q) operations, not O(Q^2).
//
// The update works on deviations from the rest state (f - w rho0) and on the
// non-equilibrium part of the moments, so that in float32 the small force
// increments (F/18 ~ 1e-8 per step) are not lost against O(1) values:
//   A     = M df                      raw moments of the deviations
//   E     = m_eq(rho, u) - m_w        raw moments of the equilibrium at
//                                     (rho, u), minus those of the rest state,
//                                     formed factor by factor (no cancellation)
//   kneq  = T(u) (A - E + d1)         non-equilibrium central moments; d1 =
//                                     F_pre/2 in the first-order slots, i.e.
//                                     the first raw moments are taken as
//                                     rho u (the half-forced velocity), as the
//                                     printed D2Q9 collision does
//   df'   = M^-1 ( A - T(-u) R kneq + K_F )
// where T(u) is the binomial shift to central moments, R applies the
// relaxation rates per moment group (so R kneq is what the collision removes)
// and K_F are the raw moments of the post-collision half force step
// F_tot e_a / <e_x|e_x>.  Zeroth and first-order slots of the result are set
// exactly to drho and j + F_tot (eq. 27).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "common.hpp"

namespace casclb {

template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (N > 0) {
        static_for<N - 1>(f);
        f(std::integral_constant<int, N - 1>{});
    }
}

// ---------------------------------------------------------------------------
// lattice tables (compile-time)
// ---------------------------------------------------------------------------

__host__ __device__ constexpr int digit(int k, int axis) {
    return axis == 0 ? k % 3 : (axis == 1 ? (k / 3) % 3 : (k / 9) % 3);
}
__host__ __device__ constexpr int digit_velocity(int d) { return d == 0 ? 0 : (d == 1 ? 1 : -1); }
__host__ __device__ constexpr int grid_velocity(int k, int axis) { return digit_velocity(digit(k, axis)); }
__host__ __device__ constexpr int grid_opposite(int k) {
    return (digit(k, 0) == 0 ? 0 : 3 - digit(k, 0)) + 3 * (digit(k, 1) == 0 ? 0 : 3 - digit(k, 1)) +
           9 * (digit(k, 2) == 0 ? 0 : 3 - digit(k, 2));
}

template <int D>
struct Flow {
    static constexpr int Q = (D == 2) ? 9 : 27;
    // ABI population order -> grid index.  D2Q9 uses the order of eq. (15):
    // (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
    __host__ __device__ static constexpr int grid_of(int a) {
        if constexpr (D == 2) {
            return a == 0 ? 0 : a == 1 ? 1 : a == 2 ? 3 : a == 3 ? 2 : a == 4 ? 6 : a == 5 ? 4 : a == 6 ? 5 : a == 7 ? 8 : 7;
        } else {
            return a;
        }
    }
    __host__ __device__ static constexpr int abi_of(int g) {
        if constexpr (D == 2) {
            return g == 0 ? 0 : g == 1 ? 1 : g == 3 ? 2 : g == 2 ? 3 : g == 6 ? 4 : g == 4 ? 5 : g == 5 ? 6 : g == 8 ? 7 : 8;
        } else {
            return g;
        }
    }
    __host__ __device__ static constexpr int velocity(int a, int axis) {
        return axis < D ? grid_velocity(grid_of(a), axis) : 0;
    }
    __host__ __device__ static constexpr int opposite(int a) { return abi_of(grid_opposite(grid_of(a))); }
    // moment order of grid slot k
    __host__ __device__ static constexpr int order(int k) {
        return digit(k, 0) + digit(k, 1) + (D == 3 ? digit(k, 2) : 0);
    }
    static constexpr int first_slot(int axis) { return axis == 0 ? 1 : (axis == 1 ? 3 : 9); }
};

// D2Q5 scalar lattice, order of eq. (34): (0,0) (1,0) (0,1) (-1,0) (0,-1)
__host__ __device__ constexpr int d2q5_velocity(int a, int axis) {
    return axis == 0 ? (a == 1 ? 1 : (a == 3 ? -1 : 0)) : (axis == 1 ? (a == 2 ? 1 : (a == 4 ? -1 : 0)) : 0);
}
__host__ __device__ constexpr int d2q5_opposite(int a) { return a == 0 ? 0 : (a == 1 ? 3 : a == 2 ? 4 : a == 3 ? 1 : 2); }

// ---------------------------------------------------------------------------
// one-dimensional sweeps
// ---------------------------------------------------------------------------

template <int D, int AX, class Real, class Op>
__device__ __forceinline__ void sweep(Real (&m)[Flow<D>::Q], Op op) {
    constexpr int S = AX == 0 ? 1 : (AX == 1 ? 3 : 9);
    static_for<Flow<D>::Q / 3>([&](auto t) {
        constexpr int T = decltype(t)::value;
        constexpr int b = (T / S) * 3 * S + (T % S);
        op(m[b], m[b + S], m[b + 2 * S]);
    });
}

// populations (v = 0, +1, -1) -> raw moments (power 0, 1, 2)
template <int D, class Real>
__device__ __forceinline__ void raw_moments(Real (&m)[Flow<D>::Q]) {
    auto op = [](Real& a0, Real& a1, Real& a2) {
        const Real s = a1 + a2, d = a1 - a2;
        a0 = a0 + s;
        a1 = d;
        a2 = s;
    };
    sweep<D, 0>(m, op);
    sweep<D, 1>(m, op);
    if constexpr (D == 3) sweep<D, 2>(m, op);
}

// raw moments -> populations
template <int D, class Real>
__device__ __forceinline__ void populations(Real (&m)[Flow<D>::Q]) {
    auto op = [](Real& m0, Real& m1, Real& m2) {
        const Real plus = Real(0.5) * (m2 + m1);
        m0 = m0 - m2;
        m2 = plus - m1;
        m1 = plus;
    };
    sweep<D, 0>(m, op);
    sweep<D, 1>(m, op);
    if constexpr (D == 3) sweep<D, 2>(m, op);
}

// raw-type moments -> moments about velocity u (sign = +1) or back (sign = -1)
template <int D, int SIGN, class Real>
__device__ __forceinline__ void shift(Real (&m)[Flow<D>::Q], const Real (&u)[3]) {
    static_for<D>([&](auto ax) {
        constexpr int AX = decltype(ax)::value;
        const Real v = SIGN > 0 ? -u[AX] : u[AX];
        const Real v2 = v * v, tv = v + v;
        sweep<D, AX>(m, [&](Real& a0, Real& a1, Real& a2) {
            const Real b1 = a1;
            a1 = a1 + v * a0;
            a2 = a2 + tv * b1 + v2 * a0;
        });
    });
}

// Raw moment k of (equilibrium at (rho, u)) - (rest equilibrium at rho0),
// with per-axis factors b = (1, 0, 1/3) (rest) and c = (1, u, 1/3 + u^2):
// E = drho * prod b + rho * (prod c - prod b), the bracket telescoped axis by
// axis so no two O(1) numbers are subtracted.
template <int D, int K, class Real>
__device__ __forceinline__ Real eq_deviation(Real drho, Real rho, const Real (&u)[3], const Real (&usq)[3]) {
    Real pc = Real(1), diff = Real(0);
    Real pb = Real(1);
    static_for<D>([&](auto ax) {
        constexpr int AX = decltype(ax)::value;
        constexpr int p = digit(K, AX);
        if constexpr (p == 0) {
            // b = c = 1: nothing changes
        } else if constexpr (p == 1) {
            diff = pc * u[AX];  // b = 0
            pc = pc * u[AX];
            pb = Real(0);
        } else {
            const Real third = Real(1) / Real(3);
            diff = diff * third + pc * usq[AX];
            pc = pc * (third + usq[AX]);
            pb = pb * third;
        }
    });
    return drho * pb + rho * diff;
}

// Coefficient of F_tot[axis] in raw moment K of the kick F_tot . e_a / <e_x|e_x>:
// nonzero when the power along `axis` is 1 and all others are even; equals
// prod over the other axes of (1 for power 0, 2/3 for power 2).
template <int D, int K, int AXIS>
__host__ __device__ constexpr int kick_twothirds_power() {
    int n = 0;
    for (int a = 0; a < D; ++a)
        if (a != AXIS && digit(K, a) == 2) ++n;
    return n;
}
template <int D, int K, int AXIS>
__host__ __device__ constexpr bool kick_nonzero() {
    if (digit(K, AXIS) != 1) return false;
    for (int a = 0; a < D; ++a)
        if (a != AXIS && digit(K, a) == 1) return false;
    return true;
}

template <class Real>
struct FlowRates {
    Real shear, bulk, third, fourth;
};

// Collision with both half force steps.  On entry m holds the deviation
// populations (grid order) of the streamed state; on exit the deviation
// post-collision populations.  fpre: force averaged over the pre-collision
// half step; ftot: momentum change of the whole step.  Returns rho and the
// half-forced velocity u (eq. 25 / 8A).
template <int D, class Real>
__device__ __forceinline__ void collide_flow(Real (&m)[Flow<D>::Q], Real rho0, const Real (&fpre)[3],
                                             const Real (&ftot)[3], const FlowRates<Real>& w, Real& rho_out,
                                             Real (&u)[3]) {
    constexpr int Q = Flow<D>::Q;
    raw_moments<D>(m);
    const Real drho = m[0];
    const Real rho = rho0 + drho;
    const Real inv_rho = Real(1) / rho;
    Real j[3] = {Real(0), Real(0), Real(0)};
    Real usq[3] = {Real(0), Real(0), Real(0)};
    u[0] = u[1] = u[2] = Real(0);
    static_for<D>([&](auto ax) {
        constexpr int AX = decltype(ax)::value;
        j[AX] = m[Flow<D>::first_slot(AX)];
        u[AX] = (j[AX] + Real(0.5) * fpre[AX]) * inv_rho;
        usq[AX] = u[AX] * u[AX];
    });
    rho_out = rho;
    // b: non-equilibrium raw moments, first-order moments taken as rho u
    // (their slots are exact zeros: j - rho u + F_pre/2 = 0, and so is slot 0)
    Real b[Q];
    static_for<Q>([&](auto kk) {
        constexpr int K = decltype(kk)::value;
        if constexpr (Flow<D>::order(K) >= 2)
            b[K] = m[K] - eq_deviation<D, K>(drho, rho, u, usq);
        else
            b[K] = Real(0);
    });
    shift<D, +1>(b, u);
    // b <- R b: the part of each non-equilibrium central moment that the
    // collision removes (trace with omega_bulk, deviators and off-diagonal
    // second-order moments with omega_shear, third order with omega_third,
    // higher orders with omega_fourth; conserved moments untouched)
    {
        if constexpr (D == 3) {
            const Real mean = (b[2] + b[6] + b[18]) * (Real(1) / Real(3));
            const Real wm = w.bulk * mean;
            b[2] = wm + w.shear * (b[2] - mean);
            b[6] = wm + w.shear * (b[6] - mean);
            b[18] = wm + w.shear * (b[18] - mean);
        } else {
            const Real mean = Real(0.5) * (b[2] + b[6]);
            const Real half_dev = Real(0.5) * (b[2] - b[6]);
            b[2] = w.bulk * mean + w.shear * half_dev;
            b[6] = w.bulk * mean - w.shear * half_dev;
        }
        static_for<Q>([&](auto kk) {
            constexpr int K = decltype(kk)::value;
            constexpr int ord = Flow<D>::order(K);
            constexpr bool diag2 = (K == 2 || K == 6 || K == 18);
            if constexpr (ord <= 1) {
                b[K] = Real(0);
            } else if constexpr (ord == 2 && !diag2) {
                b[K] = w.shear * b[K];
            } else if constexpr (ord == 3) {
                b[K] = w.third * b[K];
            } else if constexpr (ord >= 4) {
                b[K] = w.fourth * b[K];
            }
        });
    }
    shift<D, -1>(b, u);
    // post-collision deviation raw moments A - T(-u) R kneq, with the
    // post-collision half force step
    static_for<Q>([&](auto kk) {
        constexpr int K = decltype(kk)::value;
        if constexpr (Flow<D>::order(K) >= 2) {
            Real v = m[K] - b[K];
            static_for<D>([&](auto ax) {
                constexpr int AX = decltype(ax)::value;
                if constexpr (kick_nonzero<D, K, AX>()) {
                    constexpr int n23 = kick_twothirds_power<D, K, AX>();
                    const Real c = n23 == 0 ? Real(1) : (n23 == 1 ? Real(2) / Real(3) : Real(4) / Real(9));
                    v = v + c * ftot[AX];
                }
            });
            m[K] = v;
        }
    });
    m[0] = drho;
    static_for<D>([&](auto ax) {
        constexpr int AX = decltype(ax)::value;
        m[Flow<D>::first_slot(AX)] = j[AX] + ftot[AX];
    });
    populations<D>(m);
}

template <class Real>
struct ScalarRates {
    Real diff, high;
};

// D2Q5 scalar collision with both half source steps.  g: streamed
// populations (order of eq. 34), overwritten with the post-collision ones.
// u: the flow's half-forced velocity at the node.  The central moments of
// eq. (37) about u, with the source-kicked phi (eq. 43) as zeroth moment,
// relax towards eq. (39); the post-collision half source step adds S_tot/5 to
// every population (eq. 47, 48).  Returns phi^o (eq. 42).
template <class Real>
__device__ __forceinline__ Real collide_scalar(Real (&g)[5], const Real (&u)[3], Real spre, Real stot,
                                               const ScalarRates<Real>& w) {
    const Real phi_o = g[0] + (g[1] + g[3]) + (g[2] + g[4]);
    const Real phi = phi_o + Real(0.5) * spre;
    const Real kx = g[1] - g[3], ky = g[2] - g[4];
    const Real kxx = g[1] + g[3], kyy = g[2] + g[4];
    const Real ux = u[0], uy = u[1];
    const Real third = Real(1) / Real(3);
    // non-equilibrium central moments
    const Real cx = kx - ux * phi;
    const Real cy = ky - uy * phi;
    const Real cxx = kxx - (ux + ux) * kx + ux * ux * phi - third * phi;
    const Real cyy = kyy - (uy + uy) * ky + uy * uy * phi - third * phi;
    // changes under relaxation
    const Real dcx = -w.diff * cx, dcy = -w.diff * cy;
    const Real tr = cxx + cyy, dv = cxx - cyy;
    const Real dcxx = Real(-0.5) * (w.high * tr + w.high * dv);
    const Real dcyy = Real(-0.5) * (w.high * tr - w.high * dv);
    // back to raw moments (zeroth moment unchanged by collision)
    const Real dkx = dcx, dky = dcy;
    const Real dkxx = dcxx + (ux + ux) * dcx;
    const Real dkyy = dcyy + (uy + uy) * dcy;
    const Real s5 = Real(0.2) * stot;
    g[0] = g[0] - (dkxx + dkyy) + s5;
    g[1] = g[1] + Real(0.5) * (dkxx + dkx) + s5;
    g[3] = g[3] + Real(0.5) * (dkxx - dkx) + s5;
    g[2] = g[2] + Real(0.5) * (dkyy + dky) + s5;
    g[4] = g[4] + Real(0.5) * (dkyy - dky) + s5;
    return phi_o;
}

// Deviation of the product-form equilibrium from the rest state for one
// population with velocity (e0, e1, e2):
//   rho prod psi(e_i, u_i) - rho0 prod psi(e_i, 0),
//   psi(0, u) = 2/3 - u^2, psi(+-1, u) = (1/3 + u^2 +- u)/2,
// telescoped factor by factor.
template <int D, class Real>
__device__ __forceinline__ Real equilibrium_deviation(const int (&e)[3], Real drho, Real rho, const Real (&u)[3]) {
    Real pc = Real(1), pb = Real(1), diff = Real(0);
    for (int a = 0; a < D; ++a) {
        const Real b = e[a] == 0 ? Real(2) / Real(3) : Real(1) / Real(6);
        const Real d = e[a] == 0 ? -u[a] * u[a] : Real(0.5) * (u[a] * u[a] + Real(e[a]) * u[a]);
        diff = diff * b + pc * d;
        pc = pc * (b + d);
        pb = pb * b;
    }
    return drho * pb + rho * diff;
}

// Rest-state weight w_a (product of 2/3 and 1/6 factors).
template <int D>
__host__ __device__ constexpr double rest_weight(int a) {
    double w = 1.0;
    for (int i = 0; i < D; ++i) w *= Flow<D>::velocity(a, i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
    return w;
}

// ---------------------------------------------------------------------------
// D3Q15 (Appendix A): velocity set of eq. (A1) in the paper's order, the
// orthogonal basis of eq. (2A), and the cascaded collision of eq. (6A) with
// the half force steps (8A), (13A).  Not a tensor-product lattice, so the
// update works on the 15 populations directly.
// ---------------------------------------------------------------------------
struct D3Q15 {
    static constexpr int Q = 15;
    __host__ __device__ static constexpr int velocity(int a, int axis) {
        constexpr int ex[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
        constexpr int ey[15] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
        constexpr int ez[15] = {0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
        return axis == 0 ? ex[a] : (axis == 1 ? ey[a] : ez[a]);
    }
    // pairs 1-2, 3-4, 5-6 and a <-> 21 - a among the diagonals 7..14
    __host__ __device__ static constexpr int opposite(int a) {
        return a == 0 ? 0 : (a <= 6 ? (a % 2 == 1 ? a + 1 : a - 1) : 21 - a);
    }
    // rest weights of the second-order equilibrium (2/9, 1/9, 1/72)
    __host__ __device__ static constexpr double weight(int a) { return a == 0 ? 2.0 / 9.0 : (a <= 6 ? 1.0 / 9.0 : 1.0 / 72.0); }
    // K_beta(alpha) of eq. (2A)
    __host__ __device__ static constexpr int basis(int b, int a) {
        const int x = velocity(a, 0), y = velocity(a, 1), z = velocity(a, 2), e2 = x * x + y * y + z * z;
        switch (b) {
            case 0: return 1;
            case 1: return x;
            case 2: return y;
            case 3: return z;
            case 4: return x * y;
            case 5: return x * z;
            case 6: return y * z;
            case 7: return x * x - y * y;
            case 8: return e2 - 3 * z * z;
            case 9: return e2 - 2;
            case 10: return 5 * x * e2 - 13 * x;
            case 11: return 5 * y * e2 - 13 * y;
            case 12: return 5 * z * e2 - 13 * z;
            case 13: return x * y * z;
            default: return 30 * (x * x * y * y + x * x * z * z + y * y * z * z) - 40 * e2 + 32;
        }
    }
};

// Deviations df_a = f_a - w_a rho0 in, post-collision deviations out (eq. 6A
// relaxation, g_1..3 = F_tot/10, f^p = f + K g).  Readings: the trace relaxes
// to rho (3 c_s^2 rho); rho/9 is the fourth-order equilibrium of g_14.
// Every bracket is written with deviation moments (sum w e.. rho0 removed
// analytically), so float32 keeps the O(1e-8) force increments.
template <class Real>
__device__ __forceinline__ void collide_d3q15(Real (&f)[15], Real rho0, const Real (&fpre)[3], const Real (&ftot)[3],
                                              const FlowRates<Real>& w, Real& rho_out, Real (&u)[3]) {
    Real drho = Real(0), jx = Real(0), jy = Real(0), jz = Real(0);
    Real axy = Real(0), axz = Real(0), ayz = Real(0), dxx = Real(0), dyy = Real(0), dzz = Real(0);
    Real txyy = Real(0), txxy = Real(0), txxz = Real(0), txyz = Real(0), qxxyy = Real(0);
    static_for<15>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        constexpr int X = D3Q15::velocity(A, 0), Y = D3Q15::velocity(A, 1), Z = D3Q15::velocity(A, 2);
        const Real v = f[A];
        drho += v;
        if constexpr (X != 0) { jx += Real(X) * v; dxx += v; }
        if constexpr (Y != 0) { jy += Real(Y) * v; dyy += v; }
        if constexpr (Z != 0) { jz += Real(Z) * v; dzz += v; }
        if constexpr (X * Y != 0) { axy += Real(X * Y) * v; txyy += Real(X) * v; txxy += Real(Y) * v; qxxyy += v; }
        if constexpr (X * Z != 0) { axz += Real(X * Z) * v; txxz += Real(Z) * v; }
        if constexpr (Y * Z != 0) ayz += Real(Y * Z) * v;
        if constexpr (X * Y * Z != 0) txyz += Real(X * Y * Z) * v;
    });
    const Real rho = rho0 + drho;
    const Real ux = (jx + Real(0.5) * fpre[0]) / rho, uy = (jy + Real(0.5) * fpre[1]) / rho,
               uz = (jz + Real(0.5) * fpre[2]) / rho;
    const Real third = Real(1.0 / 3.0);
    const Real kxx = third * rho0 + dxx, kyy = third * rho0 + dyy;   // raw second moments
    const Real ws = w.shear, wb = w.bulk, w3 = w.third, w4 = w.fourth;
    Real g[15];
    g[0] = Real(0);
    g[1] = Real(0.1) * ftot[0];
    g[2] = Real(0.1) * ftot[1];
    g[3] = Real(0.1) * ftot[2];
    g[4] = ws * Real(0.125) * (-axy + rho * ux * uy);
    g[5] = ws * Real(0.125) * (-axz + rho * ux * uz);
    g[6] = ws * Real(0.125) * (-ayz + rho * uy * uz);
    g[7] = ws * Real(0.25) * (-(dxx - dyy) + rho * (ux * ux - uy * uy));
    g[8] = ws * Real(1.0 / 12.0) * (-(dxx + dyy - Real(2) * dzz) + rho * (ux * ux + uy * uy - Real(2) * uz * uz));
    g[9] = wb * Real(1.0 / 18.0) * (drho - (dxx + dyy + dzz) + rho * (ux * ux + uy * uy + uz * uz));
    const Real c789 = g[8] + Real(3) * g[9];
    g[10] = w3 * Real(0.0625) * (-txyy + Real(2) * uy * axy + ux * kyy - Real(2) * rho * ux * uy * uy) + uy * g[4] +
            Real(0.125) * ux * (c789 - g[7]);
    g[11] = w3 * Real(0.0625) * (-txxy + Real(2) * ux * axy + uy * kxx - Real(2) * rho * ux * ux * uy) + ux * g[4] +
            Real(0.125) * uy * (c789 + g[7]);
    g[12] = w3 * Real(0.0625) * (-txxz + Real(2) * ux * axz + uz * kxx - Real(2) * rho * ux * ux * uz) + ux * g[5] +
            Real(0.125) * uz * (c789 + g[7]);
    g[13] = w3 * Real(0.125) * (-txyz + ux * ayz + uy * axz + uz * axy - Real(2) * rho * ux * uy * uz) + uz * g[4] +
            uy * g[5] + ux * g[6];
    const Real ux2 = ux * ux, uy2 = uy * uy;
    g[14] = w4 * Real(0.0625) * (-qxxyy + Real(2) * ux * txyy + Real(2) * uy * txxy - ux2 * kyy - uy2 * kxx -
                                 Real(4) * ux * uy * axy + drho * Real(1.0 / 9.0) + Real(3) * rho * ux2 * uy2) -
            Real(2) * ux * uy * g[4] + Real(0.125) * (ux2 - uy2) * g[7] - Real(0.125) * (ux2 + uy2) * g[8] +
            (Real(-0.375) * (ux2 + uy2) - Real(0.5)) * g[9] + Real(2) * ux * g[10] + Real(2) * uy * g[11];
    static_for<15>([&](auto aa) {
        constexpr int A = decltype(aa)::value;
        Real d = Real(0);
        static_for<14>([&](auto bb) {
            constexpr int B = decltype(bb)::value + 1;
            constexpr int k = D3Q15::basis(B, A);
            if constexpr (k != 0) d += Real(k) * g[B];
        });
        f[A] += d;
    });
    rho_out = rho;
    u[0] = ux;
    u[1] = uy;
    u[2] = uz;
}

}  // namespace casclb
