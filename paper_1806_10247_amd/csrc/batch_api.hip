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
    // routed domains (the `routed` of longest expected time in the persistent
    // launch): stepped together by ordinary launches, one per step, on their
    // own stream, driven by a host thread while the persistent launch runs the
    // others; their results go to the same per-domain arrays
    std::vector<int32_t> route_ids;            // slot -> domain id
    std::vector<char> routed_mask;             // per domain
    int32_t* w_ids = nullptr;
    int4* w_tiles = nullptr;
    int32_t* w_tile_first = nullptr;
    int32_t* w_tile_count = nullptr;
    int32_t* w_state = nullptr;
    double* w_partials = nullptr;
    int64_t* w_step = nullptr;
    int32_t* w_active = nullptr;
    int32_t* h_active = nullptr;               // pinned host copy of w_active
    int w_ntiles = 0;                          // tiles of the slots in the tile list
    int w_ntiles_all = 0;                      // tiles of all slots
    hipStream_t wstream = nullptr;
    static constexpr int kWideInFlight = 4;    // captured check intervals queued ahead of the host
    hipEvent_t w_events[kWideInFlight] = {};
    hipGraph_t wgraph[2] = {nullptr, nullptr};  // K steps + check from buffer parity p
    hipGraphExec_t wexec[2] = {nullptr, nullptr};
    double wg_tol[2] = {-1.0, -1.0};
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
    for (int p = 0; p < 2; ++p) {
        if (b->wexec[p]) (void)hipGraphExecDestroy(b->wexec[p]);
        if (b->wgraph[p]) (void)hipGraphDestroy(b->wgraph[p]);
    }
    for (hipEvent_t e : b->w_events)
        if (e) (void)hipEventDestroy(e);
    if (b->wstream) (void)hipStreamDestroy(b->wstream);
    if (b->h_active) (void)hipHostFree(b->h_active);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    void* ptrs[] = {b->d_dom, b->d_order, b->pool, b->uprev, b->queue, b->d_steps, b->d_res, b->d_status, b->staging,
                    b->w_ids, b->w_tiles, b->w_tile_first, b->w_tile_count, b->w_state, b->w_partials, b->w_step,
                    b->w_active};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

// Expected time of a domain in the persistent launch, up to a common factor:
// the steps its slowest mode needs (decay rate pi^2 nu / (4 L^2) + s per
// step, L = ny / 2) times the time of one of its steps on one workgroup, a
// fixed latency (about four passes over the workgroup's threads) plus one
// pass per 1024 nodes.
static double persistent_time(const lb_batch_domain& d) {
    const double L = 0.5 * d.ny;
    const double rate = d.nu * 9.869604401089358 / (4.0 * L * L) + d.lorentz;
    return (4.0 + (double)d.nx * d.ny / 1024.0) / rate;
}

// Tiles of kWideBlock nodes of the slots marked `running`, slot after slot
// (a stopped slot keeps no tile); invalidates the captured intervals.  The
// wide stream must be idle.
static int upload_tiles(lb_batch* b, const std::vector<char>& running) {
    const int r = (int)b->route_ids.size();
    std::vector<int4> tiles;
    std::vector<int32_t> first(r, 0), count(r, 0);
    for (int s = 0; s < r; ++s) {
        first[s] = (int32_t)tiles.size();
        if (!running[s]) continue;
        const int n = b->dom[b->route_ids[s]].nx * b->dom[b->route_ids[s]].ny;
        for (int node = 0; node < n; node += kWideBlock) tiles.push_back(make_int4(s, node, 0, 0));
        count[s] = (int32_t)tiles.size() - first[s];
    }
    b->w_ntiles = (int)tiles.size();
    if (!tiles.empty())
        BHIP(b, hipMemcpy(b->w_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->w_tile_first, first.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->w_tile_count, count.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice));
    for (int p = 0; p < 2; ++p) {
        if (b->wexec[p]) (void)hipGraphExecDestroy(b->wexec[p]);
        if (b->wgraph[p]) (void)hipGraphDestroy(b->wgraph[p]);
        b->wexec[p] = nullptr;
        b->wgraph[p] = nullptr;
    }
    return LB_OK;
}

// The `routed` domains of longest expected time, as slots of the wide launch:
// tiles of kWideBlock nodes, slot after slot.
static int create_routes(lb_batch* b) {
    std::vector<int32_t> ids(b->nd);
    for (int32_t i = 0; i < b->nd; ++i) ids[i] = i;
    std::stable_sort(ids.begin(), ids.end(), [&](int32_t x, int32_t y) {
        return persistent_time(b->dom[x]) > persistent_time(b->dom[y]);
    });
    b->route_ids.assign(ids.begin(), ids.begin() + b->cfg.routed);
    b->routed_mask.assign(b->nd, 0);
    for (int32_t id : b->route_ids) b->routed_mask[id] = 1;
    const int r = (int)b->route_ids.size();
    int64_t ntiles = 0;
    for (int32_t id : b->route_ids) ntiles += ((int64_t)b->dom[id].nx * b->dom[id].ny + kWideBlock - 1) / kWideBlock;
    b->w_ntiles_all = (int)ntiles;
#define WALLOC(ptr, bytes) BHIP(b, hipMalloc((void**)&(ptr), (bytes)))
    WALLOC(b->w_ids, sizeof(int32_t) * r);
    WALLOC(b->w_tiles, sizeof(int4) * ntiles);
    WALLOC(b->w_tile_first, sizeof(int32_t) * r);
    WALLOC(b->w_tile_count, sizeof(int32_t) * r);
    WALLOC(b->w_state, sizeof(int32_t) * r);
    WALLOC(b->w_partials, sizeof(double) * 3 * ntiles);
    WALLOC(b->w_step, sizeof(int64_t));
    WALLOC(b->w_active, sizeof(int32_t));
#undef WALLOC
    BHIP(b, hipHostMalloc((void**)&b->h_active, sizeof(int32_t), hipHostMallocDefault));
    BHIP(b, hipMemcpy(b->w_ids, b->route_ids.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice));
    BHIP(b, hipStreamCreateWithFlags(&b->wstream, hipStreamNonBlocking));
    {
        const int rc = upload_tiles(b, std::vector<char>(r, 1));
        if (rc) return rc;
    }
    for (hipEvent_t& e : b->w_events) BHIP(b, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return LB_OK;
}

static WideParams wide_params(const lb_batch* b, double tol) {
    WideParams p{};
    p.domains = b->d_dom;
    p.ids = b->w_ids;
    p.tiles = b->w_tiles;
    p.tile_first = b->w_tile_first;
    p.tile_count = b->w_tile_count;
    p.state = b->w_state;
    p.partials = b->w_partials;
    p.step = b->w_step;
    p.active = b->w_active;
    p.pool = b->pool;
    p.uprev = b->uprev;
    p.nslots = (int32_t)b->route_ids.size();
    p.check_interval = b->cfg.check_interval;
    p.tol = tol;
    p.rho0 = b->cfg.rho0;
    p.w_bulk = b->cfg.omega_bulk;
    p.w_third = b->cfg.omega_third;
    p.w_fourth = b->cfg.omega_fourth;
    p.out_steps = b->d_steps;
    p.out_residual = b->d_res;
    p.out_status = b->d_status;
    return p;
}

// The graph of one check interval of the routed slots from buffer parity p:
// K - 1 plain steps, the check step, the residuals and stopping rule.
static int wide_graph(lb_batch* b, const WideParams& w, int p, hipGraphExec_t* out) {
    if (b->wexec[p] && b->wg_tol[p] == w.tol) {
        *out = b->wexec[p];
        return LB_OK;
    }
    if (b->wexec[p]) (void)hipGraphExecDestroy(b->wexec[p]);
    if (b->wgraph[p]) (void)hipGraphDestroy(b->wgraph[p]);
    b->wexec[p] = nullptr;
    b->wgraph[p] = nullptr;
    const int K = b->cfg.check_interval;
    BHIP(b, hipStreamBeginCapture(b->wstream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int i = 0; i < K && e == hipSuccess; ++i)
        e = launch_wide_step(b->f64, w, b->w_ntiles, (p + i) & 1, i == K - 1, b->wstream);
    if (e == hipSuccess) e = launch_wide_check(w, b->wstream);
    hipError_t e2 = hipStreamEndCapture(b->wstream, &b->wgraph[p]);
    if (e != hipSuccess) return bfail(b, LB_EHIP, "routed step capture: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return bfail(b, LB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    BHIP(b, hipGraphInstantiate(&b->wexec[p], b->wgraph[p], nullptr, nullptr, 0));
    b->wg_tol[p] = w.tol;
    *out = b->wexec[p];
    return LB_OK;
}

static int drive_wide_run(lb_batch* b, int64_t max_steps, double tol) {
    BHIP(b, hipSetDevice(b->cfg.device));
    const WideParams w = wide_params(b, tol);
    const int64_t K = b->cfg.check_interval;
    const int r = w.nslots;
    // every slot starts with its tiles (an interrupted run may have left fewer)
    BHIP(b, hipStreamSynchronize(b->wstream));
    if (b->w_ntiles != b->w_ntiles_all) {
        const int rc = upload_tiles(b, std::vector<char>(r, 1));
        if (rc) return rc;
    }
    BHIP(b, launch_wide_init(w, b->wstream));
    int64_t launched = 0, head = 0, tail = 0;
    int tiled = r;   // slots that have tiles
    bool finished = false;
    while (!finished && launched + K <= max_steps) {
        if (head - tail == lb_batch::kWideInFlight) {
            BHIP(b, hipEventSynchronize(b->w_events[tail % lb_batch::kWideInFlight]));
            ++tail;
            // the count only falls: a later interval's copy can only be smaller
            int active = __atomic_load_n(b->h_active, __ATOMIC_ACQUIRE);
            if (active == 0) {
                finished = true;
                break;
            }
            if (2 * active <= tiled) {
                // half the tiled slots have stopped: drop their tiles (their
                // workgroups would only return at once, but each still costs a
                // dispatch every step)
                BHIP(b, hipStreamSynchronize(b->wstream));
                tail = head;
                std::vector<int32_t> state(r);
                BHIP(b, hipMemcpy(state.data(), b->w_state, sizeof(int32_t) * r, hipMemcpyDeviceToHost));
                std::vector<char> running(r);
                active = 0;
                for (int s = 0; s < r; ++s) active += (running[s] = state[s] < 2);
                if (active == 0) {
                    finished = true;
                    break;
                }
                const int rc = upload_tiles(b, running);
                if (rc) return rc;
                tiled = active;
            }
        }
        hipGraphExec_t ge = nullptr;
        const int rc = wide_graph(b, w, (int)(launched & 1), &ge);
        if (rc) return rc;
        BHIP(b, hipGraphLaunch(ge, b->wstream));
        BHIP(b, hipMemcpyAsync(b->h_active, b->w_active, sizeof(int32_t), hipMemcpyDeviceToHost, b->wstream));
        BHIP(b, hipEventRecord(b->w_events[head % lb_batch::kWideInFlight], b->wstream));
        ++head;
        launched += K;
    }
    BHIP(b, hipStreamSynchronize(b->wstream));
    if (!finished) {
        const int active = head > 0 ? __atomic_load_n(b->h_active, __ATOMIC_ACQUIRE) : w.nslots;
        if (active > 0) {
            // the steps short of a check up to the limit, then the limit's status
            for (int64_t s = launched; s < max_steps; ++s)
                BHIP(b, launch_wide_step(b->f64, w, b->w_ntiles, (int)(s & 1), false, b->wstream));
            BHIP(b, launch_wide_close(w, max_steps, b->wstream));
        }
    }
    if (b->w_ntiles != b->w_ntiles_all) {   // the stopped slots' tiles back for the gather
        const int rc = upload_tiles(b, std::vector<char>(r, 1));
        if (rc) return rc;
    }
    BHIP(b, launch_wide_gather(b->f64, w, b->w_ntiles, b->wstream));
    BHIP(b, hipStreamSynchronize(b->wstream));
    return LB_OK;
}

// Host thread of a run: the routed slots, interval by interval.
static void drive_routes(lb_batch* b, int64_t max_steps, double tol) {
    const int rc = drive_wide_run(b, max_steps, tol);
    if (rc != LB_OK) {
        b->driver_err = b->err;
        b->driver_rc = rc;
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
    if (cfg->routed < 0 || cfg->routed > nd) return bfail(nullptr, LB_EINVAL, "routed must lie in [0, ndomains]");
    if (cfg->routed_cus < 0) return bfail(nullptr, LB_EINVAL, "routed_cus must be >= 0");
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
    if (cfg->routed > 0 && cfg->routed_cus >= b->cus) {
        rc = bfail(nullptr, LB_EINVAL, "routed_cus must be below the device's %d compute units", b->cus);
        goto error;
    }
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
    // with routed domains, routed_cus compute units are left to their launches
    const int cus = b->cfg.routed > 0 ? b->cus - b->cfg.routed_cus : b->cus;
    return cus * per_cu;
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
    if (!b->route_ids.empty()) {
        // the routed slots start from the state the batch's stream holds when the
        // run is called (lb_batch_init, written populations): the wide stream waits
        // for the work enqueued so far, not for the persistent launch enqueued next
        hipEvent_t ready = nullptr;
        BHIP(b, hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        hipError_t e = hipEventRecord(ready, b->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->wstream, ready, 0);
        (void)hipEventDestroy(ready);
        if (e != hipSuccess) return bfail(b, LB_EHIP, "stream order: %s", hipGetErrorString(e));
    }
    const int rc = launch_run(b, max_steps, tol, b->block, b->lds_policy, true);
    if (rc) return rc;
    if (!b->route_ids.empty()) b->driver = std::thread(drive_routes, b, max_steps, tol);
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
    {
        const int rc = join_driver(b);
        if (rc) return rc;
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
