// C ABI of the batched multi-domain solver: domain table and pools, the
// captured-graph persistent launch, results, readback and the autotuner.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <thread>
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
    // routed domains (the `routed` largest by expected work): each an ordinary
    // lattice context with its own stream, stepped by a host thread while the
    // persistent launch runs the others
    std::vector<int32_t> route_ids;            // domain ids, largest work first
    std::vector<char> routed_mask;             // per domain
    std::vector<lb_ctx*> route_ctx;
    std::vector<hipStream_t> route_stream;
    std::vector<int64_t> route_steps;
    std::vector<double> route_res;
    std::vector<int32_t> route_status;
    std::thread driver;
    int driver_rc = LB_OK;
    std::string driver_err;
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

// Waits for the host thread that steps the routed domains (if one runs).
static int join_driver(lb_batch* b) {
    if (b->driver.joinable()) b->driver.join();
    if (b->driver_rc != LB_OK) {
        const int rc = b->driver_rc;
        b->driver_rc = LB_OK;
        b->err = b->driver_err;
        return rc;
    }
    return LB_OK;
}

static void bfree(lb_batch* b) {
    (void)join_driver(b);
    for (lb_ctx* c : b->route_ctx)
        if (c) lb_destroy(c);
    b->route_ctx.clear();
    for (hipStream_t st : b->route_stream)
        if (st) (void)hipStreamDestroy(st);
    b->route_stream.clear();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    void* ptrs[] = {b->d_dom, b->d_order, b->pool, b->uprev, b->queue, b->d_steps, b->d_res, b->d_status, b->staging};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

// Expected work of a domain up to a residual tolerance: nodes times the
// steps its slowest mode (decay rate pi^2 nu / (4 L^2) + s, L = ny / 2) needs,
// up to a factor common to all domains.
static double domain_work(const lb_batch_domain& d) {
    const double L = 0.5 * d.ny;
    return (double)d.nx * d.ny / (d.nu * 9.869604401089358 / (4.0 * L * L) + d.lorentz);
}

// The `routed` domains of largest expected work as ordinary lattice contexts
// (D2Q9, x periodic, halfway bounce-back walls on y, the batch's storage and
// rates, the domain's viscosity, force and Lorentz coefficient), each on a
// stream of its own.
static int create_routes(lb_batch* b) {
    std::vector<int32_t> ids(b->nd);
    for (int32_t i = 0; i < b->nd; ++i) ids[i] = i;
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int32_t x, int32_t y) { return domain_work(b->dom[x]) > domain_work(b->dom[y]); });
    b->route_ids.assign(ids.begin(), ids.begin() + b->cfg.routed);
    b->routed_mask.assign(b->nd, 0);
    for (int32_t id : b->route_ids) b->routed_mask[id] = 1;
    for (int32_t id : b->route_ids) {
        const lb_batch_domain& d = b->dom[id];
        hipStream_t st = nullptr;
        BHIP(b, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        b->route_stream.push_back(st);
        lb_config c;
        lb_config_default(&c);
        c.lattice = LB_D2Q9;
        c.storage = b->cfg.storage;
        c.device = b->cfg.device;
        c.nx = d.nx;
        c.ny = d.ny;
        c.nz = 1;
        c.bc[0] = LB_PERIODIC;
        c.bc[1] = LB_HALFWAY_BB;
        c.bc[2] = LB_PERIODIC;
        c.residual_interval = b->cfg.check_interval;
        c.nu = d.nu;
        c.omega_bulk = b->cfg.omega_bulk;
        c.omega_third = b->cfg.omega_third;
        c.omega_fourth = b->cfg.omega_fourth;
        c.rho0 = b->cfg.rho0;
        c.stream = st;
        lb_ctx* ctx = nullptr;
        if (lb_create(&ctx, &c) != LB_OK) return bfail(b, LB_EHIP, "routed domain %d: %s", id, lb_last_error(nullptr));
        b->route_ctx.push_back(ctx);
        if (lb_set_force_uniform(ctx, d.force_x, 0.0, 0.0) != LB_OK || lb_set_lorentz(ctx, d.lorentz) != LB_OK ||
            lb_init_equilibrium(ctx, nullptr, nullptr, nullptr) != LB_OK)
            return bfail(b, LB_EHIP, "routed domain %d: %s", id, lb_last_error(ctx));
    }
    const size_t r = b->route_ids.size();
    b->route_steps.assign(r, 0);
    b->route_res.assign(r, INFINITY);
    b->route_status.assign(r, LB_BATCH_NOT_RUN);
    return LB_OK;
}

// Host thread of a run: steps every routed context K steps at a time (all of
// them enqueued before any result is read) and applies the batch's stopping
// rule to each context's own residual check.
static void drive_routes(lb_batch* b, int64_t max_steps, double tol) {
    if (hipSetDevice(b->cfg.device) != hipSuccess) {
        b->driver_rc = LB_EHIP;
        b->driver_err = "routed domains: hipSetDevice failed";
        return;
    }
    const size_t r = b->route_ctx.size();
    const int64_t K = b->cfg.check_interval;
    std::vector<char> active(r, 1);
    std::vector<int64_t> done(r, 0);
    std::vector<double> res(r, INFINITY);
    for (size_t i = 0; i < r; ++i) b->route_status[i] = LB_BATCH_MAX_STEPS;
    size_t left = r;
    while (left > 0) {
        for (size_t i = 0; i < r; ++i) {
            if (!active[i]) continue;
            const int64_t n = std::min(K - lb_get_step(b->route_ctx[i]) % K, max_steps - done[i]);
            const int rc = lb_step(b->route_ctx[i], n);
            if (rc == LB_ENONFINITE) {
                b->route_status[i] = LB_BATCH_NONFINITE;
                active[i] = 0;
                --left;
            } else if (rc != LB_OK) {
                b->driver_rc = rc;
                b->driver_err = std::string("routed domain: ") + lb_last_error(b->route_ctx[i]);
                return;
            } else {
                done[i] += n;
            }
        }
        for (size_t i = 0; i < r; ++i) {
            if (!active[i]) continue;
            int64_t at = -1;
            double ri = INFINITY;
            const int rc = lb_residual(b->route_ctx[i], &ri, &at, nullptr);
            int stop = 0;
            if (rc == LB_ENONFINITE) {
                stop = LB_BATCH_NONFINITE;
            } else if (rc != LB_OK) {
                b->driver_rc = rc;
                b->driver_err = std::string("routed domain: ") + lb_last_error(b->route_ctx[i]);
                return;
            } else if (at == lb_get_step(b->route_ctx[i])) {   // a check ran at this step
                res[i] = ri;
                if (ri == 0.0)
                    stop = LB_BATCH_STATIONARY;
                else if (ri < tol)
                    stop = LB_BATCH_CONVERGED;
            }
            if (!stop && done[i] >= max_steps) stop = LB_BATCH_MAX_STEPS;
            if (stop) {
                b->route_status[i] = stop;
                active[i] = 0;
                --left;
            }
        }
    }
    for (size_t i = 0; i < r; ++i) {
        b->route_steps[i] = done[i];
        b->route_res[i] = res[i];
    }
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
    if (cfg->lds_bytes < 0) return bfail(nullptr, LB_EINVAL, "lds_bytes must be >= 0");
    if (cfg->routed < 0 || cfg->routed > nd || cfg->routed > 64)
        return bfail(nullptr, LB_EINVAL, "routed must lie in [0, min(ndomains, 64)]");
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
    if (cfg->routed > 0) {
        rc = create_routes(b);
        if (rc) {
            g_batch_create_error = b->err;
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
    {
        const int rc = join_driver(b);
        if (rc) return rc;
    }
    BHIP(b, hipSetDevice(b->cfg.device));
    for (size_t i = 0; i < b->route_ctx.size(); ++i) {
        if (lb_init_equilibrium(b->route_ctx[i], nullptr, nullptr, nullptr) != LB_OK)
            return bfail(b, LB_EHIP, "routed domain: %s", lb_last_error(b->route_ctx[i]));
        b->route_steps[i] = 0;
        b->route_res[i] = INFINITY;
        b->route_status[i] = LB_BATCH_NOT_RUN;
    }
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
    p.ndomains = b->nd - (int32_t)b->route_ids.size();   // the order lists the persistent launch's domains
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
    // routed domains are not in the persistent launch's queue
    if (!b->routed_mask.empty())
        order.erase(std::remove_if(order.begin(), order.end(), [&](int32_t i) { return b->routed_mask[i] != 0; }),
                    order.end());
    // synchronous copy: the order is read by the (possibly graph-replayed) launch
    // that follows on the stream, and the host vector dies at return
    BHIP(b, hipStreamSynchronize(b->stream));
    if (!order.empty())
        BHIP(b, hipMemcpy(b->d_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice));
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
    if (p.ndomains == 0) return LB_OK;
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
    {
        const int rc = join_driver(b);
        if (rc) return rc;
    }
    BHIP(b, hipSetDevice(b->cfg.device));
    const int rc = launch_run(b, max_steps, tol, b->block, b->lds_policy, true);
    if (rc) return rc;
    if (!b->route_ctx.empty()) b->driver = std::thread(drive_routes, b, max_steps, tol);
    return LB_OK;
}

int lb_batch_results(lb_batch* b, int64_t* steps, double* residual, int32_t* status) {
    if (!b) return LB_EINVAL;
    {
        const int rc = join_driver(b);
        if (rc) return rc;
    }
    BHIP(b, hipSetDevice(b->cfg.device));
    BHIP(b, hipStreamSynchronize(b->stream));
    if (steps) BHIP(b, hipMemcpy(steps, b->d_steps, sizeof(int64_t) * b->nd, hipMemcpyDeviceToHost));
    if (residual) BHIP(b, hipMemcpy(residual, b->d_res, sizeof(double) * b->nd, hipMemcpyDeviceToHost));
    if (status) BHIP(b, hipMemcpy(status, b->d_status, sizeof(int32_t) * b->nd, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < b->route_ids.size(); ++i) {
        const int32_t id = b->route_ids[i];
        if (steps) steps[id] = b->route_steps[i];
        if (residual) residual[id] = b->route_res[i];
        if (status) status[id] = b->route_status[i];
    }
    return LB_OK;
}

// Index of domain id among the routed ones, or -1.
static int route_index(const lb_batch* b, int32_t id) {
    for (size_t i = 0; i < b->route_ids.size(); ++i)
        if (b->route_ids[i] == id) return (int)i;
    return -1;
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
    {
        const int rc = join_driver(b);
        if (rc) return rc;
    }
    const int ri = route_index(b, id);
    if (ri >= 0) {
        if (lb_read_moments(b->route_ctx[ri], LB_MOMENTS_HALF_FORCED, rho, u, nullptr) != LB_OK)
            return bfail(b, LB_EHIP, "routed domain %d: %s", id, lb_last_error(b->route_ctx[ri]));
        return LB_OK;
    }
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
    {
        const int rc = join_driver(b);
        if (rc) return rc;
    }
    const int ri = route_index(b, id);
    if (ri >= 0) {
        if (lb_read_populations(b->route_ctx[ri], f, nullptr) != LB_OK)
            return bfail(b, LB_EHIP, "routed domain %d: %s", id, lb_last_error(b->route_ctx[ri]));
        return LB_OK;
    }
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
    {
        const int rc = join_driver(b);
        if (rc) return rc;
    }
    const int ri = route_index(b, id);
    if (ri >= 0) {
        if (lb_write_populations(b->route_ctx[ri], f, nullptr) != LB_OK)
            return bfail(b, LB_EHIP, "routed domain %d: %s", id, lb_last_error(b->route_ctx[ri]));
        return LB_OK;
    }
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
    {
        const int rc = join_driver(b);
        if (rc) return rc;
    }
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
