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

hipError_t launch_batch(bool f64, const BatchParams& bp, int grid, int block, size_t lds_bytes, hipStream_t s);
hipError_t batch_set_lds_limit(bool f64, size_t lds_bytes);
hipError_t launch_batch_moments(bool f64, const BatchParams& bp, int id, int n, double* rho, double* u,
                                hipStream_t s);
hipError_t launch_batch_zero(bool f64, void* pool, int64_t n, hipStream_t s);

}  // namespace casclb
