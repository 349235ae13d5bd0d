// Types and launchers of the batched multi-domain D2Q9 solver (batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace casclb {

enum BatchStatus : int {
    kBatchNotRun = 0,
    kBatchConverged = 1,   // residual below tol
    kBatchStationary = 2,  // u did not change at all over K steps (storage precision reached)
    kBatchMaxSteps = 3,    // step limit reached first
    kBatchNonFinite = 4,   // NaN or infinity found
};

struct BatchDomain {
    int32_t nx, ny;
    int64_t offset;        // element offset of the domain's first buffer in the pool ([9][n], then [9][n])
    int64_t uprev_offset;  // element offset of its [2][n] previous-check velocity
    double w_shear;        // 1 / (3 nu + 1/2)
    double force_x;        // F_b
    double lorentz;        // s: force -s u_x
};

struct BatchParams {
    const BatchDomain* domains;
    const int32_t* order;  // processing order (indices into domains)
    int32_t ndomains;
    int32_t check_interval;  // K >= 1
    void* pool;
    void* uprev;
    int* queue;
    int64_t max_steps;
    double tol;
    double rho0, w_bulk, w_third, w_fourth;
    int32_t lds_nodes;     // domains with at most this many nodes run in LDS
    int64_t* out_steps;
    double* out_residual;
    int32_t* out_status;
};

// Routed domains: stepped together by ordinary (non-persistent) launches, one
// per time step, each domain tiled over workgroups of kWideBlock nodes.  The
// state of slot r: 0 running, 1 running with a previous check, >= 2 stopped.
constexpr int kWideBlock = 256;

struct WideParams {
    const BatchDomain* domains;
    const int32_t* ids;          // slot -> domain id
    const int4* tiles;           // per workgroup: x = slot, y = first node
    const int32_t* tile_first;   // per slot: its first tile (tiles of a slot are consecutive)
    const int32_t* tile_count;   // per slot
    int32_t* state;              // per slot
    double* partials;            // [tile][3]: sums of |u - u_prev|^2, |u|^2, non-finite values
    int64_t* step;               // steps taken by the slots still running
    int32_t* active;             // slots still running after the latest check
    void* pool;
    void* uprev;
    int32_t nslots;
    int32_t check_interval;
    double tol;
    double rho0, w_bulk, w_third, w_fourth;
    int64_t* out_steps;
    double* out_residual;
    int32_t* out_status;
};

// One step of every running slot from buffer `parity` (0: first) to the other;
// with check, the residual partials of the step.
hipError_t launch_wide_step(bool f64, const WideParams& p, int ntiles, int parity, bool check, hipStream_t s);
// Before a run: every slot running without a previous check, residual +inf, steps 0.
hipError_t launch_wide_init(const WideParams& p, hipStream_t s);
// After a check step: per slot residual and stopping rule (the persistent
// kernel's), steps of the stopping slots; `active` counts the others; the step
// counter advances by K.
hipError_t launch_wide_check(const WideParams& p, hipStream_t s);
// Slots still running after `steps` steps stop at the step limit.
hipError_t launch_wide_close(const WideParams& p, int64_t steps, hipStream_t s);
// Final states into each domain's first buffer (after an odd number of steps
// they are in the second).
hipError_t launch_wide_gather(bool f64, const WideParams& p, int ntiles, hipStream_t s);

hipError_t launch_batch(bool f64, const BatchParams& bp, int grid, int block, size_t lds_bytes, hipStream_t s);
hipError_t batch_set_lds_limit(bool f64, size_t lds_bytes);
hipError_t launch_batch_moments(bool f64, const BatchParams& bp, int id, int n, double* rho, double* u,
                                hipStream_t s);
hipError_t launch_batch_zero(bool f64, void* pool, int64_t n, hipStream_t s);

}  // namespace casclb
