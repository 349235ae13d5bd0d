// C ABI of the batched multi-domain solver: domain table and pools, the
// captured-graph persistent launch, results, readback and the autotuner.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "batch.hpp"
#include "casclb.h"
#include "lattice.hpp"

using namespace casclb;

struct lb_batch {
    lb_batch_config cfg;
    bool f64 = false;
    int elem = 4;
    int32_t nd = 0;
    std::vector<lb_batch_domain> dom;
    std::vector<BatchDomain> ddom;
    BatchDomain* d_dom = nullptr;
    int32_t* d_order = nullptr;
    void* pool = nullptr;
    void* uprev = nullptr;
    int64_t pool_elems = 0, uprev_elems = 0;
    int* queue = nullptr;
    int64_t* d_steps = nullptr;
    double* d_res = nullptr;
    int32_t* d_status = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int cus = 0;
    size_t lds_max = 0;       // bytes of dynamic LDS one workgroup may use
    int block = 512;
    int lds_policy = 0;
    // captured graph of (queue reset, persistent kernel) for the current parameters
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t g_steps = -1;
    double g_tol = -1;
    int g_block = -1, g_policy = -1;
    // (max_steps, tol) the device-side domain order was computed for
    int64_t o_steps = -1;
    double o_tol = -1;
    double* staging = nullptr;
    size_t staging_bytes = 0;
    std::string err;
};

static thread_local std::string g_batch_create_error;

static int bfail(lb_batch* b, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (b)
        b->err = buf;
    else
        g_batch_create_error = buf;
    return code;
}

#define BHIP(b, call)                                                                                 \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) return bfail((b), LB_EHIP, "%s: %s", #call, hipGetErrorString(e_));     \
    } while (0)

static void bfree(lb_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    void* ptrs[] = {b->d_dom, b->d_order, b->pool, b->uprev, b->queue, b->d_steps, b->d_res, b->d_status, b->staging};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

extern "C" {

void lb_batch_config_default(lb_batch_config* c) {
    if (!c) return;
    memset(c, 0, sizeof(*c));
    c->abi_version = LB_ABI_VERSION;
    c->storage = LB_STORE_F32_DEV;
    c->check_interval = 100;
    c->rho0 = 1.0;
    c->omega_bulk = c->omega_third = c->omega_fourth = 1.0;
    c->block = 0;
}

int lb_batch_create(lb_batch** out, const lb_batch_config* cfg, const lb_batch_domain* domains, int32_t nd) {
    if (!out) return bfail(nullptr, LB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg || !domains) return bfail(nullptr, LB_EINVAL, "cfg and domains are required");
    if (cfg->abi_version != LB_ABI_VERSION) return bfail(nullptr, LB_EINVAL, "abi_version mismatch");
    if (cfg->storage != LB_STORE_F64 && cfg->storage != LB_STORE_F32_DEV)
        return bfail(nullptr, LB_EINVAL, "batch storage must be LB_STORE_F64 or LB_STORE_F32_DEV");
    if (nd < 1) return bfail(nullptr, LB_EINVAL, "ndomains must be >= 1");
    if (cfg->check_interval < 1) return bfail(nullptr, LB_EINVAL, "check_interval must be >= 1");
    if (!(cfg->rho0 > 0.0)) return bfail(nullptr, LB_EINVAL, "rho0 must be > 0");
    const double ws[3] = {cfg->omega_bulk, cfg->omega_third, cfg->omega_fourth};
    for (double w : ws)
        if (!(w > 0.0 && w < 2.0)) return bfail(nullptr, LB_EINVAL, "relaxation rates must lie in (0, 2)");
    if (cfg->block != 0 && (cfg->block < 64 || cfg->block > 1024 || cfg->block % 64))
        return bfail(nullptr, LB_EINVAL, "block must be 0 or a multiple of 64 in [64, 1024]");
    if (cfg->lds_policy != 0 && cfg->lds_policy != 1) return bfail(nullptr, LB_EINVAL, "lds_policy must be 0 or 1");
    if (cfg->lds_bytes < 0 || cfg->reserved != 0) return bfail(nullptr, LB_EINVAL, "lds_bytes >= 0, reserved = 0");
    for (int32_t i = 0; i < nd; ++i) {
        const lb_batch_domain& d = domains[i];
        if (d.nx < 1 || d.ny < 1 || (int64_t)d.nx * d.ny > (1 << 20))
            return bfail(nullptr, LB_EINVAL, "domain %d: size %d x %d out of range", i, d.nx, d.ny);
        if (!(d.nu > 0.0) || !isfinite(d.nu) || !isfinite(d.force_x) || !(d.lorentz >= 0.0) || !isfinite(d.lorentz))
            return bfail(nullptr, LB_EINVAL, "domain %d: nu > 0, finite force and lorentz >= 0 required", i);
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return bfail(nullptr, LB_EHIP, "no HIP device available");
    if (cfg->device < 0 || cfg->device >= ndev) return bfail(nullptr, LB_EINVAL, "device out of range");
    if (hipSetDevice(cfg->device) != hipSuccess) return bfail(nullptr, LB_EHIP, "hipSetDevice failed");

    lb_batch* b = new (std::nothrow) lb_batch();
    if (!b) return bfail(nullptr, LB_ENOMEM, "host allocation failed");
    b->cfg = *cfg;
    b->f64 = cfg->storage == LB_STORE_F64;
    b->elem = b->f64 ? 8 : 4;
    b->nd = nd;
    b->dom.assign(domains, domains + nd);
    b->block = cfg->block ? cfg->block : 512;
    b->lds_policy = cfg->lds_policy;
    int rc = LB_OK;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, cfg->device);
    if (e != hipSuccess) {
        rc = bfail(nullptr, LB_EHIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
        goto error;
    }
    b->cus = prop.multiProcessorCount;
    {
        // leave room for the kernel's static LDS (queue slot and reduction buffer)
        size_t avail = prop.sharedMemPerBlock > 4096 ? prop.sharedMemPerBlock - 4096 : 0;
        b->lds_max = cfg->lds_bytes ? std::min((size_t)cfg->lds_bytes, avail) : avail;
    }
    {
        // domain table: pools are laid out domain after domain
        b->ddom.resize(nd);
        int64_t off = 0, uoff = 0;
        for (int32_t i = 0; i < nd; ++i) {
            const lb_batch_domain& d = domains[i];
            const int64_t n = (int64_t)d.nx * d.ny;
            BatchDomain& q = b->ddom[i];
            q.nx = d.nx;
            q.ny = d.ny;
            q.offset = off;
            q.uprev_offset = uoff;
            q.w_shear = 1.0 / (3.0 * d.nu + 0.5);
            q.force_x = d.force_x;
            q.lorentz = d.lorentz;
            off += 18 * n;
            uoff += 2 * n;
        }
        b->pool_elems = off;
        b->uprev_elems = uoff;
#define BALLOC(ptr, bytes)                                                                               \
        e = hipMalloc((void**)&(ptr), (bytes));                                                          \
        if (e != hipSuccess) {                                                                           \
            rc = bfail(nullptr, LB_ENOMEM, "hipMalloc(%zu): %s", (size_t)(bytes), hipGetErrorString(e)); \
            goto error;                                                                                  \
        }
        BALLOC(b->d_dom, sizeof(BatchDomain) * nd);
        BALLOC(b->d_order, sizeof(int32_t) * nd);
        BALLOC(b->pool, (size_t)b->pool_elems * b->elem);
        BALLOC(b->uprev, (size_t)b->uprev_elems * b->elem);
        BALLOC(b->queue, sizeof(int) * 64);
        BALLOC(b->d_steps, sizeof(int64_t) * nd);
        BALLOC(b->d_res, sizeof(double) * nd);
        BALLOC(b->d_status, sizeof(int32_t) * nd);
#undef BALLOC
        if (cfg->stream) {
            b->stream = (hipStream_t)cfg->stream;
        } else {
            e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                rc = bfail(nullptr, LB_EHIP, "hipStreamCreate: %s", hipGetErrorString(e));
                goto error;
            }
            b->own_stream = true;
        }
        e = hipMemcpy(b->d_dom, b->ddom.data(), sizeof(BatchDomain) * nd, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            rc = bfail(nullptr, LB_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
            goto error;
        }
    }
    *out = b;
    return LB_OK;
error:
    bfree(b);
    delete b;
    return rc;
}

void lb_batch_destroy(lb_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->cfg.device);
    (void)hipStreamSynchronize(b->stream);
    bfree(b);
    delete b;
}

const char* lb_batch_last_error(const lb_batch* b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

int lb_batch_init(lb_batch* b) {
    if (!b) return LB_EINVAL;
    BHIP(b, hipSetDevice(b->cfg.device));
    BHIP(b, launch_batch_zero(b->f64, b->pool, b->pool_elems, b->stream));
    BHIP(b, hipMemsetAsync(b->d_steps, 0, sizeof(int64_t) * b->nd, b->stream));
    BHIP(b, hipMemsetAsync(b->d_status, 0, sizeof(int32_t) * b->nd, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return LB_OK;
}

static BatchParams params_of(lb_batch* b, int64_t max_steps, double tol, int lds_policy, int block) {
    BatchParams p{};
    p.domains = b->d_dom;
    p.order = b->d_order;
    p.ndomains = b->nd;
    p.check_interval = b->cfg.check_interval;
    p.pool = b->pool;
    p.uprev = b->uprev;
    p.queue = b->queue;
    p.max_steps = max_steps;
    p.tol = tol;
    p.rho0 = b->cfg.rho0;
    p.w_bulk = b->cfg.omega_bulk;
    p.w_third = b->cfg.omega_third;
    p.w_fourth = b->cfg.omega_fourth;
    p.lds_nodes = lds_policy == 0 ? (int32_t)(b->lds_max / (18 * (size_t)b->elem)) : 0;
    p.out_steps = b->d_steps;
    p.out_residual = b->d_res;
    p.out_status = b->d_status;
    (void)block;
    return p;
}

// Workgroups of the persistent launch: as many as fit on the device at once
// (LDS-resident runs: one per CU for the full LDS budget).
static int grid_of(const lb_batch* b, int block, size_t lds) {
    int per_cu = 2048 / block;
    if (lds > 0) {
        int by_lds = (int)(163840 / (lds + 4096));
        if (by_lds < 1) by_lds = 1;
        per_cu = std::min(per_cu, by_lds);
    }
    if (per_cu < 1) per_cu = 1;
    return b->cus * per_cu;
}

// Order in which workgroups take the domains: largest expected work first, so
// that the longest domains do not start last.  Expected steps of a domain are
// max_steps, or fewer when tol > 0: the time for its slowest mode (decay rate
// pi^2 nu / (4 L^2) + s per step, L = ny/2) to fall by 1/tol.
static int upload_order(lb_batch* b, int64_t max_steps, double tol) {
    if (b->o_steps == max_steps && b->o_tol == tol) return LB_OK;
    std::vector<int32_t> order(b->nd);
    std::vector<double> work(b->nd);
    for (int32_t i = 0; i < b->nd; ++i) {
        order[i] = i;
        const lb_batch_domain& d = b->dom[i];
        const double L = 0.5 * d.ny;
        const double rate = d.nu * 9.869604401089358 / (4.0 * L * L) + d.lorentz;
        double steps = (double)max_steps;
        if (tol > 0.0) steps = std::min(steps, std::log(1.0 / tol) / rate);
        work[i] = (double)d.nx * d.ny * steps;
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return work[a] > work[c]; });
    // synchronous copy: the order is read by the (possibly graph-replayed) launch
    // that follows on the stream, and the host vector dies at return
    BHIP(b, hipStreamSynchronize(b->stream));
    BHIP(b, hipMemcpy(b->d_order, order.data(), sizeof(int32_t) * b->nd, hipMemcpyHostToDevice));
    b->o_steps = max_steps;
    b->o_tol = tol;
    return LB_OK;
}

static int launch_run(lb_batch* b, int64_t max_steps, double tol, int block, int policy, bool use_graph) {
    {
        const int rc = upload_order(b, max_steps, tol);
        if (rc) return rc;
    }
    const BatchParams p = params_of(b, max_steps, tol, policy, block);
    const size_t lds = policy == 0 ? (size_t)p.lds_nodes * 18 * b->elem : 0;
    if (lds) BHIP(b, batch_set_lds_limit(b->f64, lds));
    const int grid = grid_of(b, block, lds);
    if (!use_graph) {
        BHIP(b, launch_batch(b->f64, p, grid, block, lds, b->stream));
        return LB_OK;
    }
    if (!b->exec || b->g_steps != max_steps || b->g_tol != tol || b->g_block != block || b->g_policy != policy) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_batch(b->f64, p, grid, block, lds, b->stream);
        hipError_t e2 = hipStreamEndCapture(b->stream, &b->graph);
        if (e != hipSuccess) return bfail(b, LB_EHIP, "batch launch during capture: %s", hipGetErrorString(e));
        if (e2 != hipSuccess) return bfail(b, LB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
        BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->g_steps = max_steps;
        b->g_tol = tol;
        b->g_block = block;
        b->g_policy = policy;
    }
    BHIP(b, hipGraphLaunch(b->exec, b->stream));
    return LB_OK;
}

int lb_batch_run(lb_batch* b, int64_t max_steps, double tol) {
    if (!b) return LB_EINVAL;
    if (max_steps < 1) return bfail(b, LB_EINVAL, "max_steps must be >= 1");
    if (!(tol >= 0.0)) return bfail(b, LB_EINVAL, "tol must be >= 0");
    BHIP(b, hipSetDevice(b->cfg.device));
    return launch_run(b, max_steps, tol, b->block, b->lds_policy, true);
}

int lb_batch_results(lb_batch* b, int64_t* steps, double* residual, int32_t* status) {
    if (!b) return LB_EINVAL;
    BHIP(b, hipSetDevice(b->cfg.device));
    BHIP(b, hipStreamSynchronize(b->stream));
    if (steps) BHIP(b, hipMemcpy(steps, b->d_steps, sizeof(int64_t) * b->nd, hipMemcpyDeviceToHost));
    if (residual) BHIP(b, hipMemcpy(residual, b->d_res, sizeof(double) * b->nd, hipMemcpyDeviceToHost));
    if (status) BHIP(b, hipMemcpy(status, b->d_status, sizeof(int32_t) * b->nd, hipMemcpyDeviceToHost));
    return LB_OK;
}

static int bstaging(lb_batch* b, size_t bytes) {
    if (b->staging_bytes >= bytes) return LB_OK;
    if (b->staging) (void)hipFree(b->staging);
    b->staging = nullptr;
    b->staging_bytes = 0;
    hipError_t e = hipMalloc((void**)&b->staging, bytes);
    if (e != hipSuccess) return bfail(b, LB_ENOMEM, "staging: %s", hipGetErrorString(e));
    b->staging_bytes = bytes;
    return LB_OK;
}

int lb_batch_read_moments(lb_batch* b, int32_t id, double* rho, double* u) {
    if (!b) return LB_EINVAL;
    if (id < 0 || id >= b->nd) return bfail(b, LB_EINVAL, "domain %d out of range", id);
    BHIP(b, hipSetDevice(b->cfg.device));
    const int n = b->dom[id].nx * b->dom[id].ny;
    int rc = bstaging(b, sizeof(double) * 3 * n);
    if (rc) return rc;
    const BatchParams p = params_of(b, 1, 0.0, 1, b->block);
    BHIP(b, launch_batch_moments(b->f64, p, id, n, b->staging, b->staging + n, b->stream));
    if (rho) BHIP(b, hipMemcpyAsync(rho, b->staging, sizeof(double) * n, hipMemcpyDeviceToHost, b->stream));
    if (u) BHIP(b, hipMemcpyAsync(u, b->staging + n, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return LB_OK;
}

int lb_batch_read_populations(lb_batch* b, int32_t id, double* f) {
    if (!b || !f) return LB_EINVAL;
    if (id < 0 || id >= b->nd) return bfail(b, LB_EINVAL, "domain %d out of range", id);
    BHIP(b, hipSetDevice(b->cfg.device));
    BHIP(b, hipStreamSynchronize(b->stream));
    const int64_t n = (int64_t)b->dom[id].nx * b->dom[id].ny;
    std::vector<char> tmp((size_t)(9 * n * b->elem));
    BHIP(b, hipMemcpy(tmp.data(), (char*)b->pool + b->ddom[id].offset * b->elem, tmp.size(), hipMemcpyDeviceToHost));
    for (int a = 0; a < 9; ++a) {
        const double w = rest_weight<2>(a) * b->cfg.rho0;
        for (int64_t i = 0; i < n; ++i) {
            const double v = b->f64 ? ((const double*)tmp.data())[a * n + i] : (double)((const float*)tmp.data())[a * n + i];
            f[a * n + i] = v + w;
        }
    }
    return LB_OK;
}

int lb_batch_write_populations(lb_batch* b, int32_t id, const double* f) {
    if (!b || !f) return LB_EINVAL;
    if (id < 0 || id >= b->nd) return bfail(b, LB_EINVAL, "domain %d out of range", id);
    BHIP(b, hipSetDevice(b->cfg.device));
    BHIP(b, hipStreamSynchronize(b->stream));
    const int64_t n = (int64_t)b->dom[id].nx * b->dom[id].ny;
    std::vector<char> tmp((size_t)(9 * n * b->elem));
    for (int a = 0; a < 9; ++a) {
        const double w = rest_weight<2>(a) * b->cfg.rho0;
        for (int64_t i = 0; i < n; ++i) {
            const double v = f[a * n + i] - w;
            if (b->f64)
                ((double*)tmp.data())[a * n + i] = v;
            else
                ((float*)tmp.data())[a * n + i] = (float)v;
        }
    }
    BHIP(b, hipMemcpy((char*)b->pool + b->ddom[id].offset * b->elem, tmp.data(), tmp.size(), hipMemcpyHostToDevice));
    return LB_OK;
}

int lb_batch_autotune(lb_batch* b, int64_t sample_steps, int32_t* block_out, int32_t* lds_out, double* best_ms) {
    if (!b) return LB_EINVAL;
    if (sample_steps < 1) return bfail(b, LB_EINVAL, "sample_steps must be >= 1");
    BHIP(b, hipSetDevice(b->cfg.device));
    BHIP(b, hipStreamSynchronize(b->stream));
    // save the state (pool) so that the trials leave it unchanged
    void* saved = nullptr;
    const size_t bytes = (size_t)b->pool_elems * b->elem;
    BHIP(b, hipMalloc(&saved, bytes));
    hipError_t e = hipMemcpy(saved, b->pool, bytes, hipMemcpyDeviceToDevice);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    double best = INFINITY;
    int best_block = b->block, best_policy = b->lds_policy;
    const int blocks[3] = {256, 512, 1024};
    for (int bi = 0; bi < 3 && e == hipSuccess; ++bi) {
        for (int policy = 0; policy < 2 && e == hipSuccess; ++policy) {
            e = hipMemcpyAsync(b->pool, saved, bytes, hipMemcpyDeviceToDevice, b->stream);
            if (e != hipSuccess) break;
            e = hipEventRecord(t0, b->stream);
            if (e != hipSuccess) break;
            if (launch_run(b, sample_steps, 0.0, blocks[bi], policy, false) != LB_OK) {
                e = hipErrorUnknown;
                break;
            }
            e = hipEventRecord(t1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e == hipSuccess && ms < best) {
                best = ms;
                best_block = blocks[bi];
                best_policy = policy;
            }
        }
    }
    hipError_t e2 = hipMemcpy(b->pool, saved, bytes, hipMemcpyDeviceToDevice);
    (void)hipFree(saved);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (e != hipSuccess) return bfail(b, LB_EHIP, "autotune: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return bfail(b, LB_EHIP, "autotune restore: %s", hipGetErrorString(e2));
    b->block = best_block;
    b->lds_policy = best_policy;
    if (block_out) *block_out = best_block;
    if (lds_out) *lds_out = best_policy;
    if (best_ms) *best_ms = best;
    // results of the trials are not results of a run
    BHIP(b, hipMemsetAsync(b->d_steps, 0, sizeof(int64_t) * b->nd, b->stream));
    BHIP(b, hipMemsetAsync(b->d_status, 0, sizeof(int32_t) * b->nd, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return LB_OK;
}

}  // extern "C"
