// Types shared by the host API and the kernels of the casclb library.
#pragma once

#include <stdint.h>

namespace casclb {

enum Lattice : int { kD2Q9 = 0, kD2Q9D2Q5 = 1, kD3Q27 = 2 };
enum Storage : int { kF64 = 0, kF32Dev = 1, kF16Dev = 2 };

constexpr int kDiagSlots = 8;  // du2, u2, drho, momentum x/y/z, scalar, non-finite count
constexpr int kMaxBlock = 256;  // largest block of any kernel

// Lattice geometry seen by a kernel.
struct Geometry {
    int32_t nx, ny, nz;
    int32_t bb[3];        // 1: halfway bounce-back walls at both ends of the axis
    int64_t plane;        // elements between population planes
    int32_t x_blocks;     // blocks along x per row
    int32_t xcd_remap;    // 1: give each XCD a contiguous range of rows
    int64_t grid_blocks;  // total blocks of the launch
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
    double force[3];
    const void* force_field;
    double f_pre, f_tot;   // time factors: pre-collision half step, whole step
    // source (scalar lattice only)
    double source;
    const void* source_field;
    double s_pre, s_tot;
    // residual check (DIAG kernels only)
    void* u_prev;          // [dims][plane] previous check's velocity, arithmetic type
    double* partials;      // [grid_blocks][kDiagSlots]
};

}  // namespace casclb
