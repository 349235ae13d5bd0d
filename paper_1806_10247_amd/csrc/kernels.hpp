// Host-side launchers of the casclb kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace casclb {

// Fused step: one launch of a.geo.grid_blocks blocks of `block` threads.
// diag = true also updates the residual record (u_prev, partials).
hipError_t launch_step(int lattice, int storage, const StepArgs& a, int block, bool diag, hipStream_t s);
// Sums `blocks` diagnostic partial records into out[kDiagSlots].
hipError_t launch_reduce(const double* partials, int64_t blocks, double* out, hipStream_t s);
// The following take a Geometry laid out for 256-thread blocks.
hipError_t launch_init(int lattice, int storage, const Geometry& g256, void* buf, const double* rho, const double* u,
                       const double* phi, double rho0, int64_t n, hipStream_t s);
// Shifts the stored state (buf) to the moments (rho, u, phi), keeping f - f_eq per node.
hipError_t launch_reset(int lattice, int storage, const Geometry& g256, void* buf, const double* rho, const double* u,
                        const double* phi, double rho0, int64_t n, hipStream_t s);
hipError_t launch_moments(int lattice, int storage, const StepArgs& a256, int kind, double* rho, double* u,
                          double* phi, int64_t n, hipStream_t s);
hipError_t launch_totals(int lattice, int storage, const Geometry& g256, const void* buf, double* partials,
                         hipStream_t s);
// Totals of the stored state (buf) into out5 (device, 5 doubles: mass incl.
// mass_offset, momentum x/y/z, scalar) with `records` partial records
// (1 <= records <= g256.grid_blocks) in scratch, which must hold
// (records + 1) * kDiagSlots doubles; no allocation.
hipError_t launch_totals_bounded(int lattice, int storage, const Geometry& g256, const void* buf, double* scratch,
                                 int64_t records, double mass_offset, double* out5, hipStream_t s);
hipError_t launch_plane_to_f64(int storage, const void* in, double* out, int64_t n, double offset, hipStream_t s);
hipError_t launch_plane_from_f64(int storage, const double* in, void* out, int64_t n, double offset, hipStream_t s);
hipError_t launch_box_to_f64(int storage, const void* plane, double* out, const Geometry& g, const int64_t lo[3],
                             const int64_t ext[3], double offset, hipStream_t s);
hipError_t launch_field_from_f64(bool f64, const double* in, void* out, int64_t n, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// Streaming read (mode 1), write (2) or copy (0) of `bytes` in `width`-byte
// (8 or 16) vectors; blocks = 0: one pass, otherwise a grid-stride loop over
// that many 256-thread blocks.  Read mode writes one vector per block to dst.
hipError_t launch_stream(void* dst, const void* src, size_t bytes, int mode, int width, int64_t blocks,
                         hipStream_t s);
// Fills `count` 16-bit words at dst with `value` (a kernel, not a memset node).
hipError_t launch_fill_u16(void* dst, size_t count, uint16_t value, hipStream_t s);

}  // namespace casclb
