// Types shared by the host API and the kernels of the casclb library.
#pragma once

#include <stdint.h>

namespace casclb {

enum Lattice : int { kD2Q9 = 0, kD2Q9D2Q5 = 1, kD3Q27 = 2, kD3Q15 = 3 };
enum Storage : int { kF64 = 0, kF32Dev = 1, kF16Dev = 2 };

// du2, u2, drho, momentum x/y/z, scalar, non-finite count, dphi2, phi2
constexpr int kDiagSlots = 10;
constexpr int kMaxBlock = 256;  // largest block of any kernel

// Division of n < 2^31 by a fixed divisor d >= 1 as a multiply-high and a
// shift (round-up method for invariant divisors): q = (mulhi(n, m) + n) >> s
// with s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1.  Lets a kernel
// decode its block index with scalar integer ops instead of an emulated
// division.
struct FastDiv {
    uint32_t d, m, s;
    FastDiv() : d(1), m(1), s(0) {}
    explicit FastDiv(uint32_t div) : d(div), m(0), s(0) {
        while ((1ull << s) < div) ++s;
        m = (uint32_t)((((1ull << s) - div) << 32) / div + 1);
    }
#ifdef __HIPCC__
    __host__ __device__
#endif
    uint32_t div(uint32_t n) const {
        const uint32_t hi = (uint32_t)(((uint64_t)n * m) >> 32);
        return (hi + n) >> s;
    }
};

// Lattice geometry seen by a kernel.
struct Geometry {
    int32_t nx, ny, nz;
    int32_t bb[3];        // 1: halfway bounce-back walls at both ends of the axis
    int64_t plane;        // elements between population planes
    int32_t x_blocks;     // blocks along x per row
    int32_t xcd_remap;    // 1: give each XCD a contiguous range of rows
    int64_t grid_blocks;  // total blocks of the launch (< 2^31)
    int32_t rows;         // rows per thread (1 or 2): a thread updates node x of `rows` consecutive rows
    int32_t nrows;        // ny * nz
    int32_t xpair;        // 1: 16-bit storage, a thread updates nodes 2t, 2t+1 (x_blocks counts pairs)
    FastDiv div_xb;       // division by x_blocks
    FastDiv div_ny;       // division by ny
};

// Arguments of the fused step kernel (passed by value).
struct StepArgs {
    Geometry geo;
    const void* src;   // stored state (flow planes, then scalar planes)
    void* dst;         // next state
    double rho0;
    double w_shear, w_bulk, w_third, w_fourth;  // flow relaxation rates
    double w_phi, w_phi_high;                    // scalar relaxation rates
    // force: uniform components or a [dims][plane] field in the arithmetic type
    double fx, fy, fz;   // separate fields: an indexed array here ends up in scratch
    const void* force_field;
    double f_pre, f_tot;   // time factors: pre-collision half step, whole step
    // source (scalar lattice only)
    double source;
    const void* source_field;
    double s_pre, s_tot;
    // residual check (DIAG kernels only)
    void* u_prev;          // [dims][plane] previous check's velocity, arithmetic type
    double* partials;      // [grid_blocks][kDiagSlots]
    // walls of 2D lattices (EXT kernels only), side index 2*axis + (0 low,
    // 1 high), axis 0 = x, 1 = y, as a device table (indexed by a run-time
    // side; an array among the kernel arguments would be copied to scratch):
    // [0..8) wall velocity (x, y) per side, [8..12) 1 = scalar held fixed,
    // [12..16) the fixed scalar value
    const double* walls;
    double heat;           // viscous-heating coefficient c_h of the scalar source c_h (S:S)
    int32_t ext;           // walls move, a scalar wall is fixed, or heat != 0
    // float16 storage: 1 = stores rounded stochastically with random bits from a
    // hash of (node, population, sr_seed), sr_seed a hash of the step number;
    // 0 = rounded to nearest
    int32_t sr;
    uint32_t sr_seed;
    double lorentz;        // 2D lattices: s of the velocity-dependent x-force -s u_x (0: none)
};
constexpr int kWallTable = 16;

}  // namespace casclb
