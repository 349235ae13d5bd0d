// C ABI of the casclb library: context management, host<->device transfers,
// the step loop with its time factors and residual checks.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "casclb.h"
#include "common.hpp"
#include "kernels.hpp"
#include "lattice.hpp"

using namespace casclb;

struct lb_ctx {
    lb_config cfg;
    int dims = 0, q = 0, qs = 0;
    int64_t n = 0, plane = 0;
    int elem = 0;                 // bytes per stored population
    int real_bytes = 0;           // bytes of the arithmetic type
    int block = 256;              // threads per block of the step kernel
    Geometry geo_step{}, geo_aux{};
    void* buf[2] = {nullptr, nullptr};
    bool own_buf = false;
    int cur = 0;                  // buffer holding the stored state
    bool initialised = false;
    int64_t step = 0;
    hipStream_t stream = nullptr;
    // force
    double force[3] = {0, 0, 0};
    void* force_field = nullptr;
    int force_mode = LB_TIME_CONSTANT;
    double force_omega = 0;
    // source
    double source = 0;
    void* source_field = nullptr;
    int source_mode = LB_TIME_CONSTANT;
    double source_omega = 0;
    // walls of 2D lattices: host copy of the device table (StepArgs::walls)
    double wall_table[kWallTable] = {};
    double* wall_dev = nullptr;
    bool walls_used = false;
    double heat = 0;
    double lorentz = 0;           // s of the velocity-dependent x-force -s u_x (2D lattices)
    // captured runs of plain steps (no residual check): each entry holds n
    // steps starting from buffer parity p, valid while the step arguments
    // equal its args (both parities); least recently used entries are replaced
    hipStream_t cap_stream = nullptr;
    struct StepGraph {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        int p = -1;
        int n = 0;
        uint64_t used = 0;
        StepArgs args[2];
    };
    static constexpr int kGraphCache = 8;
    StepGraph graphs[kGraphCache];
    uint64_t graph_clock = 0;
    // residual checks
    void* u_prev = nullptr;
    double* partials = nullptr;   // [max blocks][kDiagSlots]
    int64_t partial_blocks = 0;
    double* diag_dev = nullptr;   // kDiagSlots doubles
    double* diag_host = nullptr;  // pinned copy of the last completed check
    hipEvent_t diag_event = nullptr;
    bool prev_valid = false;      // u_prev holds the previous check's velocity
    bool check_pending = false;
    bool check_valid = false;     // the latest check had a previous velocity
    int64_t check_step = -1;
    // staging for float64 transfers
    double* staging = nullptr;
    size_t staging_bytes = 0;
    std::string err;
};

static thread_local std::string g_create_error;

// Scratch of lb_totals_noalloc: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends) for at most
// kScratchRecords partial records plus the reduced record.  Host code never
// uses the array's name as an address: lb_create resolves each device's
// address once, with that device current, and the kernels receive it.
static constexpr int64_t kScratchRecords = 1024;
static __device__ __align__(256) double scratch[(kScratchRecords + 1) * kDiagSlots];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch array (the device must be current).
static hipError_t scratch_address(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

static int fail(lb_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_create_error = buf;
    return code;
}

#define HIP_OR_FAIL(ctx, call)                                                                       \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return fail((ctx), LB_EHIP, "%s: %s", #call, hipGetErrorString(e_));   \
    } while (0)

// float16 stores are rounded stochastically unless LB_FLAG_F16_NEAREST asks
// for rounding to nearest.
static bool stochastic_rounding(const lb_ctx* c) {
    return c->cfg.storage == LB_STORE_F16_DEV && !(c->cfg.flags & LB_FLAG_F16_NEAREST);
}

// Random seed of step n's stochastic rounding (splitmix64 finaliser of n).
static uint32_t step_seed(int64_t n) {
    uint64_t z = (uint64_t)n + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (uint32_t)(z >> 32);
}

// Largest change one step's force makes to one population, per unit force
// summed over the axes: the first-order moment change F / <e_x|e_x> (eq. 31:
// 6 on D2Q9, eq. 13A: 10 on D3Q15, 18 on D3Q27) on a population whose
// velocity has every component non-zero.
static double kick_per_force(int lattice) {
    return lattice == LB_D3Q27 ? 1.0 / 18.0 : (lattice == LB_D3Q15 ? 1.0 / 10.0 : 1.0 / 6.0);
}

// With float16 stores rounded to nearest, a kick below half the smallest
// float16 subnormal (2^-25) is lost at every store, so a lattice started from
// rest never moves: such a force or source is refused.
static int check_nearest_kick(lb_ctx* c, double kick, const char* what) {
    if (c->cfg.storage != LB_STORE_F16_DEV || !(c->cfg.flags & LB_FLAG_F16_NEAREST)) return LB_OK;
    if (kick > 0.0 && kick < 0x1p-25)
        return fail(c, LB_EINVAL,
                    "%s: the largest per-step change of a population (%.3g) is below half the smallest float16 "
                    "subnormal; with float16 stores rounded to nearest it would be lost at every step "
                    "(use stochastic rounding, the float16 default)",
                    what, kick);
    return LB_OK;
}

static int dims_of(int lattice) { return lattice == LB_D3Q27 || lattice == LB_D3Q15 ? 3 : 2; }
static int q_of(int lattice) { return lattice == LB_D3Q27 ? 27 : (lattice == LB_D3Q15 ? 15 : 9); }
static int qs_of(int lattice) { return lattice == LB_D2Q9_D2Q5 ? 5 : 0; }
static int elem_of(int storage) { return storage == LB_STORE_F64 ? 8 : (storage == LB_STORE_F32_DEV ? 4 : 2); }
static int real_of(int storage) { return storage == LB_STORE_F64 ? 8 : 4; }

static int64_t plane_of(const lb_config* c, int64_t n, int elem) {
    if (c->plane_pad >= 0) return n + c->plane_pad;
    // round each plane up to 256 bytes, then add 4 KiB + 256 B so that
    // consecutive planes do not start on the same HBM channel/bank offset
    const int64_t per = 256 / elem;
    int64_t p = (n + per - 1) / per * per;
    if (n >= (1 << 20)) p += (4096 + 256) / elem;
    return p;
}

// Two x-adjacent nodes per step-kernel thread, read and written as 32-bit
// words: 16-bit storage only, with an even nx, a periodic x axis and an even
// plane stride (word-aligned planes and rows).
static bool xpair_allowed(const lb_config* c) {
    return c->storage == LB_STORE_F16_DEV && c->nx % 2 == 0 && c->bc[0] == LB_PERIODIC &&
           plane_of(c, c->nx * c->ny * c->nz, 2) % 2 == 0;
}

// Automatic choice, measured on MI355X (float16, GLUPS, one node / x-adjacent pair
// per thread): D3Q27 256^3 duct 35.2 / 49.2, D2Q9 4096^2 131.5 / 145.8,
// D2Q9+D2Q5 4096^2 95.6 / 97.4, D3Q15 256^3 duct 72.0 / 71.0: pairs except on D3Q15.
static int xpairs_of(const lb_config* c) {
    if (c->x_pairs > 0) return c->x_pairs;
    return xpair_allowed(c) && c->rows_per_thread != 2 && c->lattice != LB_D3Q15 ? 2 : 1;
}

// Rows each thread of the step kernel updates.  Two rows keep twice the
// bytes in flight per wave but cost registers; with one node per thread
// that measured faster only for D2Q9 with 16-bit storage (about +5%).
static int rows_of(const lb_config* c) {
    if (c->rows_per_thread > 0) return c->rows_per_thread;
    if (xpairs_of(c) == 2) return 1;
    return (c->lattice == LB_D2Q9 && c->storage == LB_STORE_F16_DEV) ? 2 : 1;
}

static int block_of(const lb_config* c) {
    if (c->block_x > 0) return c->block_x;
    const int64_t threads = xpairs_of(c) == 2 ? c->nx / 2 : c->nx;
    int64_t b = (threads + 63) / 64 * 64;
    if (b > 256) b = 256;
    return (int)b;
}

extern "C" {

void lb_config_default(lb_config* cfg) {
    if (!cfg) return;
    memset(cfg, 0, sizeof(*cfg));
    cfg->abi_version = LB_ABI_VERSION;
    cfg->lattice = LB_D3Q27;
    cfg->storage = LB_STORE_F32_DEV;
    cfg->device = 0;
    cfg->nx = cfg->ny = cfg->nz = 64;
    cfg->bc[0] = cfg->bc[1] = cfg->bc[2] = LB_PERIODIC;
    cfg->residual_interval = 100;
    cfg->nu = 1.0 / 6.0;
    cfg->omega_bulk = cfg->omega_third = cfg->omega_fourth = 1.0;
    cfg->D_phi = 1.0 / 6.0;
    cfg->omega_phi_high = 1.0;
    cfg->rho0 = 1.0;
    cfg->stream = nullptr;
    cfg->plane_pad = -1;
    cfg->block_x = 0;
}

int lb_validate_config(const lb_config* c, char* msg, size_t msg_len) {
    char tmp[256] = "";
    int rc = LB_OK;
#define BAD(...)                               \
    do {                                       \
        snprintf(tmp, sizeof(tmp), __VA_ARGS__); \
        rc = LB_EINVAL;                        \
        goto done;                             \
    } while (0)
    if (!c) BAD("config is NULL");
    if (c->abi_version != LB_ABI_VERSION) BAD("abi_version %d, library has %d", c->abi_version, LB_ABI_VERSION);
    if (c->lattice < LB_D2Q9 || c->lattice > LB_D3Q15) BAD("unknown lattice %d", c->lattice);
    if (c->storage < LB_STORE_F64 || c->storage > LB_STORE_F16_DEV) BAD("unknown storage %d", c->storage);
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) BAD("lattice size must be >= 1 (got %lld x %lld x %lld)",
                                                 (long long)c->nx, (long long)c->ny, (long long)c->nz);
    // each factor < 2^31, so nx*ny fits in int64; the third factor is checked
    // by division before any product that could overflow is formed
    if (c->nx > (1LL << 30) || c->ny > (1LL << 30) || c->nz > (1LL << 30) || c->nx * c->ny > (1LL << 31) - 1 ||
        c->nz > ((1LL << 31) - 1) / (c->nx * c->ny))
        BAD("lattice too large: N must fit in 31 bits");
    for (int i = 0; i < 3; ++i)
        if (c->bc[i] != LB_PERIODIC && c->bc[i] != LB_HALFWAY_BB) BAD("bc[%d] = %d is not a boundary type", i, c->bc[i]);
    if (!(c->nu > 0.0) || !isfinite(c->nu)) BAD("nu must be > 0 (tau > 1/2), got %g", c->nu);
    if (!(c->omega_bulk > 0.0 && c->omega_bulk < 2.0)) BAD("omega_bulk must lie in (0, 2)");
    if (!(c->omega_third > 0.0 && c->omega_third < 2.0)) BAD("omega_third must lie in (0, 2)");
    if (!(c->omega_fourth > 0.0 && c->omega_fourth < 2.0)) BAD("omega_fourth must lie in (0, 2)");
    if (c->lattice == LB_D2Q9_D2Q5) {
        if (!(c->D_phi > 0.0) || !isfinite(c->D_phi)) BAD("D_phi must be > 0, got %g", c->D_phi);
        if (!(c->omega_phi_high > 0.0 && c->omega_phi_high < 2.0)) BAD("omega_phi_high must lie in (0, 2)");
    }
    if (!(c->rho0 > 0.0) || !isfinite(c->rho0)) BAD("rho0 must be > 0");
    if (c->residual_interval < 0) BAD("residual_interval must be >= 0");
    if (c->block_x != 0 && (c->block_x < 64 || c->block_x > kMaxBlock || c->block_x % 64 != 0))
        BAD("block_x must be 0 or a multiple of 64 in [64, %d]", kMaxBlock);
    if (c->rows_per_thread < 0 || c->rows_per_thread > 2) BAD("rows_per_thread must be 0, 1 or 2");
    if (c->x_pairs < 0 || c->x_pairs > 2) BAD("x_pairs must be 0, 1 or 2");
    if (c->x_pairs == 2 && !xpair_allowed(c))
        BAD("x_pairs = 2 needs 16-bit storage, an even nx, a periodic x axis and an even plane stride");
    if (c->x_pairs == 2 && c->rows_per_thread == 2) BAD("x_pairs = 2 updates one row per thread");
    if (c->plane_pad < -1 || c->plane_pad > (1LL << 24)) BAD("plane_pad must be -1 or in [0, 2^24]");
    if (c->flags & ~(LB_FLAG_EXTERNAL_BUFFERS | LB_FLAG_XCD_REMAP | LB_FLAG_DEBUG_POISON | LB_FLAG_F16_NEAREST))
        BAD("unknown flags 0x%x", c->flags);
#undef BAD
done:
    if (msg && msg_len) {
        strncpy(msg, tmp, msg_len - 1);
        msg[msg_len - 1] = 0;
    }
    return rc;
}

size_t lb_required_bytes(const lb_config* c) {
    if (lb_validate_config(c, nullptr, 0) != LB_OK) return 0;
    const int64_t n = c->nx * c->ny * c->nz;
    const int elem = elem_of(c->storage);
    return (size_t)(plane_of(c, n, elem) * (q_of(c->lattice) + qs_of(c->lattice)) * elem);
}

static Geometry make_geometry(const lb_ctx* c, int block, int rows, bool xpair = false) {
    Geometry g{};
    g.nx = (int32_t)c->cfg.nx;
    g.ny = (int32_t)c->cfg.ny;
    g.nz = (int32_t)c->cfg.nz;
    for (int i = 0; i < 3; ++i) g.bb[i] = c->cfg.bc[i] == LB_HALFWAY_BB;
    g.plane = c->plane;
    const int64_t threads = xpair ? c->cfg.nx / 2 : c->cfg.nx;
    g.x_blocks = (int32_t)((threads + block - 1) / block);
    g.xpair = xpair ? 1 : 0;
    g.rows = g.bb[0] || xpair ? 1 : rows;  // the x-wall and x-pair kernels update one row per thread
    g.nrows = (int32_t)(c->cfg.ny * c->cfg.nz);
    g.grid_blocks = (int64_t)g.x_blocks * ((g.nrows + g.rows - 1) / g.rows);
    g.div_xb = FastDiv((uint32_t)g.x_blocks);
    g.div_ny = FastDiv((uint32_t)c->cfg.ny);
    g.xcd_remap = (c->cfg.flags & LB_FLAG_XCD_REMAP) && g.grid_blocks % 8 == 0 ? 1 : 0;
    return g;
}

static int ensure_staging(lb_ctx* c, size_t bytes) {
    if (c->staging_bytes >= bytes) return LB_OK;
    if (c->staging) (void)hipFree(c->staging);
    c->staging = nullptr;
    c->staging_bytes = 0;
    hipError_t e = hipMalloc((void**)&c->staging, bytes);
    if (e != hipSuccess) return fail(c, LB_ENOMEM, "staging allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    c->staging_bytes = bytes;
    return LB_OK;
}

static void release(lb_ctx* c) {
    if (c->own_buf) {
        if (c->buf[0]) (void)hipFree(c->buf[0]);
        if (c->buf[1]) (void)hipFree(c->buf[1]);
    }
    c->buf[0] = c->buf[1] = nullptr;
    if (c->force_field) (void)hipFree(c->force_field);
    if (c->source_field) (void)hipFree(c->source_field);
    if (c->u_prev) (void)hipFree(c->u_prev);
    if (c->partials) (void)hipFree(c->partials);
    if (c->diag_dev) (void)hipFree(c->diag_dev);
    if (c->wall_dev) (void)hipFree(c->wall_dev);
    if (c->diag_host) (void)hipHostFree(c->diag_host);
    if (c->diag_event) (void)hipEventDestroy(c->diag_event);
    if (c->staging) (void)hipFree(c->staging);
    for (auto& g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
        g = lb_ctx::StepGraph{};
    }
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
}

int lb_create(lb_ctx** out, const lb_config* cfg) {
    if (!out) return fail(nullptr, LB_EINVAL, "out is NULL");
    *out = nullptr;
    char msg[256];
    if (lb_validate_config(cfg, msg, sizeof(msg)) != LB_OK) return fail(nullptr, LB_EINVAL, "%s", msg);
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) return fail(nullptr, LB_EHIP, "no HIP device available (%s)", hipGetErrorString(e));
    if (cfg->device < 0 || cfg->device >= ndev) return fail(nullptr, LB_EINVAL, "device %d out of range (%d devices)", cfg->device, ndev);
    e = hipSetDevice(cfg->device);
    if (e != hipSuccess) return fail(nullptr, LB_EHIP, "hipSetDevice: %s", hipGetErrorString(e));

    lb_ctx* c = new (std::nothrow) lb_ctx();
    if (!c) return fail(nullptr, LB_ENOMEM, "host allocation failed");
    c->cfg = *cfg;
    c->dims = dims_of(cfg->lattice);
    c->q = q_of(cfg->lattice);
    c->qs = qs_of(cfg->lattice);
    c->n = cfg->nx * cfg->ny * cfg->nz;
    c->elem = elem_of(cfg->storage);
    c->real_bytes = real_of(cfg->storage);
    c->plane = plane_of(cfg, c->n, c->elem);
    c->block = block_of(cfg);
    c->geo_step = make_geometry(c, c->block, rows_of(cfg), xpairs_of(cfg) == 2);
    c->geo_aux = make_geometry(c, 256, 1);
    c->stream = (hipStream_t)cfg->stream;

    const size_t bytes = lb_required_bytes(cfg);
    int rc = LB_OK;
#define ALLOC(ptr, sz)                                                                                   \
    do {                                                                                                 \
        hipError_t ae_ = hipMalloc((void**)&(ptr), (sz));                                                \
        if (ae_ != hipSuccess) {                                                                         \
            rc = fail(nullptr, LB_ENOMEM, "hipMalloc(%zu) failed: %s", (size_t)(sz), hipGetErrorString(ae_)); \
            goto error;                                                                                  \
        }                                                                                                \
    } while (0)
    if (!(cfg->flags & LB_FLAG_EXTERNAL_BUFFERS)) {
        ALLOC(c->buf[0], bytes);
        ALLOC(c->buf[1], bytes);
        c->own_buf = true;
    }
    {
        const int64_t maxb = c->geo_step.grid_blocks > c->geo_aux.grid_blocks ? c->geo_step.grid_blocks : c->geo_aux.grid_blocks;
        c->partial_blocks = maxb;
        ALLOC(c->partials, (size_t)maxb * kDiagSlots * sizeof(double));
    }
    ALLOC(c->diag_dev, kDiagSlots * sizeof(double));
    ALLOC(c->wall_dev, kWallTable * sizeof(double));
    // previous check's u* (dims planes) and, on the coupled lattice, phi* (one more plane)
    if (cfg->residual_interval > 0)
        ALLOC(c->u_prev, (size_t)c->plane * (c->dims + (c->qs ? 1 : 0)) * c->real_bytes);
#undef ALLOC
    e = hipHostMalloc((void**)&c->diag_host, kDiagSlots * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        rc = fail(nullptr, LB_ENOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
        goto error;
    }
    memset(c->diag_host, 0, kDiagSlots * sizeof(double));
    e = hipMemcpy(c->wall_dev, c->wall_table, sizeof(c->wall_table), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        rc = fail(nullptr, LB_EHIP, "hipMemcpy failed: %s", hipGetErrorString(e));
        goto error;
    }
    e = hipEventCreateWithFlags(&c->diag_event, hipEventDisableTiming);
    if (e != hipSuccess) {
        rc = fail(nullptr, LB_EHIP, "hipEventCreate failed: %s", hipGetErrorString(e));
        goto error;
    }
    {
        double* sp = nullptr;
        e = scratch_address(cfg->device, &sp);
        if (e != hipSuccess) {
            rc = fail(nullptr, LB_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            goto error;
        }
    }
    *out = c;
    return LB_OK;
error:
    release(c);
    delete c;
    return rc;
}

void lb_destroy(lb_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->cfg.device);
    (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
}

const char* lb_last_error(const lb_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int lb_bind_buffers(lb_ctx* c, void* a, void* b, size_t bytes_each) {
    if (!c) return LB_EINVAL;
    if (!a || !b || a == b) return fail(c, LB_EINVAL, "two distinct non-NULL buffers are required");
    if (bytes_each < lb_required_bytes(&c->cfg))
        return fail(c, LB_EINVAL, "buffers of %zu bytes, %zu required", bytes_each, lb_required_bytes(&c->cfg));
    if (((uintptr_t)a | (uintptr_t)b) & 255) return fail(c, LB_EINVAL, "buffers must be 256-byte aligned");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    if (c->own_buf) {
        (void)hipFree(c->buf[0]);
        (void)hipFree(c->buf[1]);
    }
    c->buf[0] = a;
    c->buf[1] = b;
    c->own_buf = false;
    c->cur = 0;
    c->initialised = false;
    c->prev_valid = false;
    return LB_OK;
}

static double rest_weight_of(const lb_ctx* c, int a) {
    if (c->cfg.lattice == LB_D3Q15) return D3Q15::weight(a);
    return c->dims == 3 ? rest_weight<3>(a) : rest_weight<2>(a);
}

static int init_from(lb_ctx* c, const double* d_rho, const double* d_u, const double* d_phi, bool sync) {
    HIP_OR_FAIL(c, launch_init(c->cfg.lattice, c->cfg.storage, c->geo_aux, c->buf[c->cur], d_rho, d_u, d_phi,
                               c->cfg.rho0, c->n, c->stream));
    if (sync) HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->initialised = true;
    c->step = 0;
    c->prev_valid = false;
    c->check_pending = false;
    c->check_step = -1;
    c->diag_host[7] = 0.0;
    return LB_OK;
}

int lb_init_equilibrium(lb_ctx* c, const double* rho, const double* u, const double* phi) {
    if (!c) return LB_EINVAL;
    if (!c->buf[0]) return fail(c, LB_ESTATE, "no population buffers bound");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    const size_t nb = (size_t)c->n * sizeof(double);
    const size_t need = (rho ? nb : 0) + (u ? nb * c->dims : 0) + (phi && c->qs ? nb : 0);
    double *d_rho = nullptr, *d_u = nullptr, *d_phi = nullptr;
    if (need) {
        int rc = ensure_staging(c, need);
        if (rc) return rc;
        double* p = c->staging;
        if (rho) { d_rho = p; p += c->n; }
        if (u) { d_u = p; p += c->n * c->dims; }
        if (phi && c->qs) { d_phi = p; p += c->n; }
        if (d_rho) HIP_OR_FAIL(c, hipMemcpyAsync(d_rho, rho, nb, hipMemcpyHostToDevice, c->stream));
        if (d_u) HIP_OR_FAIL(c, hipMemcpyAsync(d_u, u, nb * c->dims, hipMemcpyHostToDevice, c->stream));
        if (d_phi) HIP_OR_FAIL(c, hipMemcpyAsync(d_phi, phi, nb, hipMemcpyHostToDevice, c->stream));
    }
    return init_from(c, d_rho, d_u, d_phi, true);
}

int lb_init_equilibrium_device(lb_ctx* c, const double* rho, const double* u, const double* phi) {
    if (!c) return LB_EINVAL;
    if (!c->buf[0]) return fail(c, LB_ESTATE, "no population buffers bound");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    return init_from(c, rho, u, c->qs ? phi : nullptr, false);
}

int lb_reset_moments_device(lb_ctx* c, const double* rho, const double* u, const double* phi) {
    if (!c) return LB_EINVAL;
    if (!rho || !u || (c->qs && !phi))
        return fail(c, LB_EINVAL, "rho and u (and phi on the scalar lattice) are required");
    if (!c->buf[0]) return fail(c, LB_ESTATE, "no population buffers bound");
    if (!c->initialised) return fail(c, LB_ESTATE, "the stored state is not initialised");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    HIP_OR_FAIL(c, launch_reset(c->cfg.lattice, c->cfg.storage, c->geo_aux, c->buf[c->cur], rho, u,
                                c->qs ? phi : nullptr, c->cfg.rho0, c->n, c->stream));
    c->prev_valid = false;
    return LB_OK;
}

int lb_set_force_uniform(lb_ctx* c, double fx, double fy, double fz) {
    if (!c) return LB_EINVAL;
    if (!isfinite(fx) || !isfinite(fy) || !isfinite(fz)) return fail(c, LB_EINVAL, "force must be finite");
    {
        const int rc = check_nearest_kick(
            c, (fabs(fx) + fabs(fy) + (c->dims == 3 ? fabs(fz) : 0.0)) * kick_per_force(c->cfg.lattice), "force");
        if (rc) return rc;
    }
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->force[0] = fx;
    c->force[1] = fy;
    c->force[2] = c->dims == 3 ? fz : 0.0;
    if (c->force_field) (void)hipFree(c->force_field);
    c->force_field = nullptr;
    return LB_OK;
}

// Copies a [comps][N] field into a [comps][plane] device array of the arithmetic type.
static int upload_field(lb_ctx* c, void** slot, const void* src, int comps, int32_t dtype, int32_t mem) {
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    if (!src) {
        if (*slot) (void)hipFree(*slot);
        *slot = nullptr;
        return LB_OK;
    }
    if (dtype != LB_DTYPE_F64 && dtype != LB_DTYPE_F32) return fail(c, LB_EINVAL, "dtype %d unknown", dtype);
    if (mem != LB_MEM_HOST && mem != LB_MEM_DEVICE) return fail(c, LB_EINVAL, "mem %d unknown", mem);
    const bool f64 = c->real_bytes == 8;
    if (mem == LB_MEM_DEVICE && f64 && dtype != LB_DTYPE_F64)
        return fail(c, LB_EINVAL, "device fields must be float64 for this storage");
    if (!*slot) {
        hipError_t e = hipMalloc(slot, (size_t)c->plane * comps * c->real_bytes);
        if (e != hipSuccess) return fail(c, LB_ENOMEM, "field allocation failed: %s", hipGetErrorString(e));
    }
    const size_t es = c->real_bytes;
    if (mem == LB_MEM_DEVICE && (dtype == LB_DTYPE_F64) == f64) {
        HIP_OR_FAIL(c, hipMemcpy2DAsync(*slot, c->plane * es, src, c->n * es, c->n * es, comps,
                                        hipMemcpyDeviceToDevice, c->stream));
    } else if (mem == LB_MEM_DEVICE) {
        // float64 device field for a float32 context: converted plane by plane
        for (int k = 0; k < comps; ++k)
            HIP_OR_FAIL(c, launch_field_from_f64(false, (const double*)src + (size_t)k * c->n,
                                                 (char*)*slot + (size_t)k * c->plane * es, c->n, c->stream));
    } else {
        int rc = ensure_staging(c, (size_t)c->n * sizeof(double));
        if (rc) return rc;
        std::vector<double> tmp;
        std::vector<double> kick_sum(c->n, 0.0);   // per node: sum over the components of |field|
        for (int k = 0; k < comps; ++k) {
            const double* plane_src;
            if (dtype == LB_DTYPE_F64) {
                plane_src = (const double*)src + (size_t)k * c->n;
            } else {
                tmp.resize(c->n);
                const float* fs = (const float*)src + (size_t)k * c->n;
                for (int64_t i = 0; i < c->n; ++i) tmp[i] = fs[i];
                plane_src = tmp.data();
            }
            for (int64_t i = 0; i < c->n; ++i)
                if (!isfinite(plane_src[i])) return fail(c, LB_EINVAL, "field value %lld is not finite", (long long)i);
            for (int64_t i = 0; i < c->n; ++i) kick_sum[i] += fabs(plane_src[i]);
            HIP_OR_FAIL(c, hipMemcpyAsync(c->staging, plane_src, c->n * sizeof(double), hipMemcpyHostToDevice, c->stream));
            HIP_OR_FAIL(c, launch_field_from_f64(f64, c->staging, (char*)*slot + (size_t)k * c->plane * es, c->n, c->stream));
            HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
        }
        const double largest = c->n ? *std::max_element(kick_sum.begin(), kick_sum.end()) : 0.0;
        const bool force = comps == c->dims && slot == &c->force_field;
        rc = check_nearest_kick(c, largest * (force ? kick_per_force(c->cfg.lattice) : 0.2),
                                force ? "force field" : "source field");
        if (rc) {
            (void)hipFree(*slot);
            *slot = nullptr;
            return rc;
        }
    }
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LB_OK;
}

int lb_set_force_field(lb_ctx* c, const void* F, int32_t dtype, int32_t mem) {
    if (!c) return LB_EINVAL;
    return upload_field(c, &c->force_field, F, c->dims, dtype, mem);
}

static int check_time(lb_ctx* c, int32_t mode, double omega) {
    if (mode != LB_TIME_CONSTANT && mode != LB_TIME_COS) return fail(c, LB_EINVAL, "time mode %d unknown", mode);
    if (!isfinite(omega)) return fail(c, LB_EINVAL, "omega must be finite");
    return LB_OK;
}

int lb_set_force_time(lb_ctx* c, int32_t mode, double omega) {
    if (!c) return LB_EINVAL;
    int rc = check_time(c, mode, omega);
    if (rc) return rc;
    c->force_mode = mode;
    c->force_omega = omega;
    return LB_OK;
}

int lb_set_source_uniform(lb_ctx* c, double s) {
    if (!c) return LB_EINVAL;
    if (!c->qs) return fail(c, LB_EINVAL, "the lattice has no scalar field");
    if (!isfinite(s)) return fail(c, LB_EINVAL, "source must be finite");
    {
        const int rc = check_nearest_kick(c, fabs(s) / 5.0, "source");   // eq. 47: S/5 on every population
        if (rc) return rc;
    }
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->source = s;
    if (c->source_field) (void)hipFree(c->source_field);
    c->source_field = nullptr;
    return LB_OK;
}

int lb_set_source_field(lb_ctx* c, const void* S, int32_t dtype, int32_t mem) {
    if (!c) return LB_EINVAL;
    if (!c->qs) return fail(c, LB_EINVAL, "the lattice has no scalar field");
    return upload_field(c, &c->source_field, S, 1, dtype, mem);
}

int lb_set_source_time(lb_ctx* c, int32_t mode, double omega) {
    if (!c) return LB_EINVAL;
    if (!c->qs) return fail(c, LB_EINVAL, "the lattice has no scalar field");
    int rc = check_time(c, mode, omega);
    if (rc) return rc;
    c->source_mode = mode;
    c->source_omega = omega;
    return LB_OK;
}

// Time factors of step n (covering [n, n+1]): trapezoidal averages of tau(t)
// over the pre- and post-collision half steps.
static void time_factors(int mode, double omega, int64_t n, double* pre, double* post) {
    if (mode == LB_TIME_COS) {
        const double a = cos(omega * (double)n), h = cos(omega * ((double)n + 0.5)), b = cos(omega * ((double)n + 1.0));
        *pre = 0.5 * (a + h);
        *post = 0.5 * (h + b);
    } else {
        *pre = *post = 1.0;
    }
}

static StepArgs make_args_p(const lb_ctx* c, const Geometry& g, int64_t n, int parity) {
    StepArgs a;
    memset(&a, 0, sizeof(a));   // padding too: captured arguments are compared bytewise
    a.geo = g;
    a.src = c->buf[parity];
    a.dst = c->buf[parity ^ 1];
    a.rho0 = c->cfg.rho0;
    a.w_shear = 1.0 / (3.0 * c->cfg.nu + 0.5);
    a.w_bulk = c->cfg.omega_bulk;
    a.w_third = c->cfg.omega_third;
    a.w_fourth = c->cfg.omega_fourth;
    a.w_phi = 1.0 / (3.0 * c->cfg.D_phi + 0.5);
    a.w_phi_high = c->cfg.omega_phi_high;
    a.fx = c->force[0];
    a.fy = c->force[1];
    a.fz = c->force[2];
    a.force_field = c->force_field;
    double pre, post;
    time_factors(c->force_mode, c->force_omega, n, &pre, &post);
    a.f_pre = pre;
    a.f_tot = 0.5 * (pre + post);
    a.source = c->source;
    a.source_field = c->source_field;
    time_factors(c->source_mode, c->source_omega, n, &pre, &post);
    a.s_pre = pre;
    a.s_tot = 0.5 * (pre + post);
    a.u_prev = c->u_prev;
    a.partials = c->partials;
    a.walls = c->wall_dev;
    a.heat = c->heat;
    a.ext = (c->walls_used || c->heat != 0.0) ? 1 : 0;
    a.lorentz = c->lorentz;
    a.sr = stochastic_rounding(c) ? 1 : 0;
    a.sr_seed = a.sr ? step_seed(n) : 0u;
    return a;
}

// Upload the wall table on the context's stream (ordered before later steps;
// the host copy lives in the context).
static int upload_walls(lb_ctx* c) {
    bool used = false;
    for (int k = 0; k < 12; ++k) used = used || c->wall_table[k] != 0.0;
    c->walls_used = used;
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    HIP_OR_FAIL(c, hipMemcpyAsync(c->wall_dev, c->wall_table, sizeof(c->wall_table), hipMemcpyHostToDevice,
                                  c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LB_OK;
}

static int wall_side(lb_ctx* c, int32_t axis, int32_t side, int* k) {
    if (c->dims != 2) return fail(c, LB_EINVAL, "wall velocities and scalar walls exist on 2D lattices only");
    if (axis < 0 || axis > 1 || side < 0 || side > 1) return fail(c, LB_EINVAL, "axis must be 0 or 1, side 0 or 1");
    if (c->cfg.bc[axis] != LB_HALFWAY_BB) return fail(c, LB_EINVAL, "axis %d has no walls (periodic)", axis);
    *k = 2 * axis + side;
    return LB_OK;
}

int lb_set_wall_velocity(lb_ctx* c, int32_t axis, int32_t side, double ux, double uy, double uz) {
    if (!c) return LB_EINVAL;
    int k = 0;
    const int rc = wall_side(c, axis, side, &k);
    if (rc) return rc;
    if (!isfinite(ux) || !isfinite(uy) || uz != 0.0) return fail(c, LB_EINVAL, "wall velocity must be finite, uz = 0");
    c->wall_table[2 * k] = ux;
    c->wall_table[2 * k + 1] = uy;
    return upload_walls(c);
}

int lb_set_scalar_wall(lb_ctx* c, int32_t axis, int32_t side, int32_t fixed, double value) {
    if (!c) return LB_EINVAL;
    if (!c->qs) return fail(c, LB_EINVAL, "the lattice has no scalar");
    int k = 0;
    const int rc = wall_side(c, axis, side, &k);
    if (rc) return rc;
    if (!isfinite(value)) return fail(c, LB_EINVAL, "scalar wall value must be finite");
    c->wall_table[8 + k] = fixed ? 1.0 : 0.0;
    c->wall_table[12 + k] = fixed ? value : 0.0;
    return upload_walls(c);
}

int lb_set_lorentz(lb_ctx* c, double s) {
    if (!c) return LB_EINVAL;
    if (c->dims != 2) return fail(c, LB_EINVAL, "the velocity-dependent force exists on 2D lattices only");
    if (!(s >= 0.0) || !isfinite(s)) return fail(c, LB_EINVAL, "s must be finite and >= 0");
    c->lorentz = s;
    return LB_OK;
}

int lb_set_viscous_heating(lb_ctx* c, double coefficient) {
    if (!c) return LB_EINVAL;
    if (!c->qs) return fail(c, LB_EINVAL, "the lattice has no scalar");
    if (!(coefficient >= 0.0) || !isfinite(coefficient)) return fail(c, LB_EINVAL, "heating coefficient must be >= 0");
    c->heat = coefficient;
    return LB_OK;
}

static StepArgs make_args(const lb_ctx* c, const Geometry& g, int64_t n) { return make_args_p(c, g, n, c->cur); }

// Steps launched one by one cost the host-side launch time (several
// microseconds) per step, more than a small lattice's step takes on the GPU.
// Runs of plain steps (no residual check) with arguments that do not change
// from step to step (force and source constant in time) are replayed from
// captured graphs instead: kGraphSteps steps at a time, and the rest of a run
// up to the next residual check (at least kGraphMinSteps) as one graph of its
// own length, so a run between checks costs a few launches.
static constexpr int kGraphSteps = 64;
static constexpr int kGraphMinSteps = 8;

static bool graphs_apply(const lb_ctx* c) {
    // stochastic rounding draws new random bits every step, so its steps never repeat
    return c->force_mode == LB_TIME_CONSTANT && c->source_mode == LB_TIME_CONSTANT &&
           !(c->cfg.flags & LB_FLAG_DEBUG_POISON) && !stochastic_rounding(c);
}

// The graph of n plain steps (alternating buffer parities from p), captured on
// first use or when the step arguments changed.
static int graph_for(lb_ctx* c, int p, int n, hipGraphExec_t* out) {
    const StepArgs a0 = make_args_p(c, c->geo_step, c->step, p);
    const StepArgs a1 = make_args_p(c, c->geo_step, c->step, p ^ 1);
    lb_ctx::StepGraph* slot = nullptr;
    for (auto& g : c->graphs) {
        if (g.exec && g.p == p && g.n == n) {
            if (memcmp(&a0, &g.args[0], sizeof(a0)) == 0 && memcmp(&a1, &g.args[1], sizeof(a1)) == 0) {
                g.used = ++c->graph_clock;
                *out = g.exec;
                return LB_OK;
            }
            slot = &g;   // same run, other arguments: recapture in place
        }
    }
    if (!slot) {
        slot = &c->graphs[0];
        for (auto& g : c->graphs)
            if (!g.exec || g.used < slot->used) slot = &g;
    }
    if (slot->exec) (void)hipGraphExecDestroy(slot->exec);
    if (slot->graph) (void)hipGraphDestroy(slot->graph);
    *slot = lb_ctx::StepGraph{};
    if (!c->cap_stream) HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_OR_FAIL(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int i = 0; i < n && e == hipSuccess; ++i)
        e = launch_step(c->cfg.lattice, c->cfg.storage, (i & 1) ? a1 : a0, c->block, false, c->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(c, LB_EHIP, "step graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    slot->graph = graph;
    HIP_OR_FAIL(c, hipGraphInstantiate(&slot->exec, graph, nullptr, nullptr, 0));
    slot->p = p;
    slot->n = n;
    slot->args[0] = a0;
    slot->args[1] = a1;
    slot->used = ++c->graph_clock;
    *out = slot->exec;
    return LB_OK;
}

int lb_step(lb_ctx* c, int64_t nsteps) {
    if (!c) return LB_EINVAL;
    if (nsteps < 0) return fail(c, LB_EINVAL, "nsteps must be >= 0");
    if (!c->initialised) return fail(c, LB_ESTATE, "state not initialised (lb_init_equilibrium / lb_write_populations)");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    if (c->check_pending && hipEventQuery(c->diag_event) == hipSuccess) c->check_pending = false;
    if (!c->check_pending && c->diag_host[7] > 0.0)
        return fail(c, LB_ENONFINITE, "non-finite values found by the residual check after step %lld",
                    (long long)c->check_step);
    const int K = c->cfg.residual_interval;
    for (int64_t s = 0; s < nsteps; ++s) {
        if (graphs_apply(c)) {
            // plain steps before the next residual check (or the end of the call)
            int64_t plain = nsteps - s;
            if (K > 0) plain = std::min(plain, (int64_t)(K - 1 - c->step % K));
            while (plain >= kGraphMinSteps) {
                const int n = (int)std::min<int64_t>(plain, kGraphSteps);
                hipGraphExec_t ge = nullptr;
                const int rc = graph_for(c, c->cur, n, &ge);
                if (rc) return rc;
                HIP_OR_FAIL(c, hipGraphLaunch(ge, c->stream));
                c->step += n;
                c->cur ^= n & 1;   // each step swaps the buffers
                s += n;
                plain -= n;
            }
            if (s >= nsteps) break;
        }
        const bool check = K > 0 && (c->step + 1) % K == 0;
        StepArgs a = make_args(c, c->geo_step, c->step);
        if (c->cfg.flags & LB_FLAG_DEBUG_POISON)
            HIP_OR_FAIL(c, launch_fill_u16(c->buf[c->cur ^ 1], lb_required_bytes(&c->cfg) / 2, 0xFFFFu, c->stream));
        HIP_OR_FAIL(c, launch_step(c->cfg.lattice, c->cfg.storage, a, c->block, check, c->stream));
        if (check) {
            HIP_OR_FAIL(c, launch_reduce(c->partials, c->geo_step.grid_blocks, c->diag_dev, c->stream));
            HIP_OR_FAIL(c, hipMemcpyAsync(c->diag_host, c->diag_dev, kDiagSlots * sizeof(double),
                                          hipMemcpyDeviceToHost, c->stream));
            HIP_OR_FAIL(c, hipEventRecord(c->diag_event, c->stream));
            c->check_pending = true;
            c->check_valid = c->prev_valid;
            c->prev_valid = true;
            c->check_step = c->step + 1;
        }
        c->cur ^= 1;
        c->step += 1;
    }
    return LB_OK;
}

int lb_synchronize(lb_ctx* c) {
    if (!c) return LB_EINVAL;
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->check_pending = false;
    return LB_OK;
}

int64_t lb_get_step(const lb_ctx* c) { return c ? c->step : -1; }

int lb_set_step(lb_ctx* c, int64_t n) {
    if (!c) return LB_EINVAL;
    if (n < 0) return fail(c, LB_EINVAL, "step must be >= 0");
    c->step = n;
    return LB_OK;
}

int lb_read_moments(lb_ctx* c, int32_t kind, double* rho, double* u, double* phi) {
    if (!c) return LB_EINVAL;
    if (kind != LB_MOMENTS_OUTPUT && kind != LB_MOMENTS_HALF_FORCED) return fail(c, LB_EINVAL, "kind %d unknown", kind);
    if (!c->initialised) return fail(c, LB_ESTATE, "state not initialised");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    if (!c->qs) phi = nullptr;
    const size_t nb = (size_t)c->n * sizeof(double);
    int rc = ensure_staging(c, nb * (2 + c->dims));
    if (rc) return rc;
    double* d_rho = c->staging;
    double* d_u = d_rho + c->n;
    double* d_phi = d_u + c->n * c->dims;
    StepArgs a = make_args(c, c->geo_aux, c->step);
    HIP_OR_FAIL(c, launch_moments(c->cfg.lattice, c->cfg.storage, a, kind, rho ? d_rho : nullptr, u ? d_u : nullptr,
                                  phi ? d_phi : nullptr, c->n, c->stream));
    if (rho) HIP_OR_FAIL(c, hipMemcpyAsync(rho, d_rho, nb, hipMemcpyDeviceToHost, c->stream));
    if (u) HIP_OR_FAIL(c, hipMemcpyAsync(u, d_u, nb * c->dims, hipMemcpyDeviceToHost, c->stream));
    if (phi) HIP_OR_FAIL(c, hipMemcpyAsync(phi, d_phi, nb, hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LB_OK;
}

int lb_read_moments_device(lb_ctx* c, int32_t kind, double* rho, double* u, double* phi) {
    if (!c) return LB_EINVAL;
    if (kind != LB_MOMENTS_OUTPUT && kind != LB_MOMENTS_HALF_FORCED) return fail(c, LB_EINVAL, "kind %d unknown", kind);
    if (!c->initialised) return fail(c, LB_ESTATE, "state not initialised");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    if (!c->qs) phi = nullptr;
    StepArgs a = make_args(c, c->geo_aux, c->step);
    HIP_OR_FAIL(c, launch_moments(c->cfg.lattice, c->cfg.storage, a, kind, rho, u, phi, c->n, c->stream));
    return LB_OK;
}

int lb_read_populations(lb_ctx* c, double* f, double* g) {
    if (!c) return LB_EINVAL;
    if (!f) return fail(c, LB_EINVAL, "f is NULL");
    if (!c->initialised) return fail(c, LB_ESTATE, "state not initialised");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    const size_t nb = (size_t)c->n * sizeof(double);
    int rc = ensure_staging(c, nb);
    if (rc) return rc;
    const char* base = (const char*)c->buf[c->cur];
    const int total = c->q + ((g && c->qs) ? c->qs : 0);
    for (int a = 0; a < total; ++a) {
        const double off = a < c->q ? rest_weight_of(c, a) * c->cfg.rho0 : 0.0;
        double* dst = a < c->q ? f + (size_t)a * c->n : g + (size_t)(a - c->q) * c->n;
        HIP_OR_FAIL(c, launch_plane_to_f64(c->cfg.storage, base + (size_t)a * c->plane * c->elem, c->staging, c->n, off, c->stream));
        HIP_OR_FAIL(c, hipMemcpyAsync(dst, c->staging, nb, hipMemcpyDeviceToHost, c->stream));
        HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    }
    return LB_OK;
}

int lb_write_populations(lb_ctx* c, const double* f, const double* g) {
    if (!c) return LB_EINVAL;
    if (!c->buf[0]) return fail(c, LB_ESTATE, "no population buffers bound");
    if (!f) return fail(c, LB_EINVAL, "f is NULL");
    if (c->qs && !g) return fail(c, LB_EINVAL, "g is required for the scalar lattice");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    const size_t nb = (size_t)c->n * sizeof(double);
    int rc = ensure_staging(c, nb);
    if (rc) return rc;
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    char* base = (char*)c->buf[c->cur];
    for (int a = 0; a < c->q + c->qs; ++a) {
        const double off = a < c->q ? rest_weight_of(c, a) * c->cfg.rho0 : 0.0;
        const double* src = a < c->q ? f + (size_t)a * c->n : g + (size_t)(a - c->q) * c->n;
        HIP_OR_FAIL(c, hipMemcpyAsync(c->staging, src, nb, hipMemcpyHostToDevice, c->stream));
        HIP_OR_FAIL(c, launch_plane_from_f64(c->cfg.storage, c->staging, base + (size_t)a * c->plane * c->elem, c->n, off, c->stream));
        HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    }
    c->initialised = true;
    c->prev_valid = false;
    c->check_pending = false;
    c->diag_host[7] = 0.0;
    return LB_OK;
}

int lb_read_populations_box(lb_ctx* c, const int64_t lo[3], const int64_t ext[3], double* f, double* g) {
    if (!c) return LB_EINVAL;
    if (!lo || !ext || !f) return fail(c, LB_EINVAL, "lo, ext and f are required");
    if (!c->initialised) return fail(c, LB_ESTATE, "state not initialised");
    for (int i = 0; i < 3; ++i)
        if (ext[i] < 1 || ext[i] > (1LL << 20)) return fail(c, LB_EINVAL, "ext[%d] = %lld out of range", i, (long long)ext[i]);
    const int64_t bn = ext[0] * ext[1] * ext[2];
    if (bn > (1LL << 28)) return fail(c, LB_EINVAL, "box too large");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    const size_t nb = (size_t)bn * sizeof(double);
    int rc = ensure_staging(c, nb);
    if (rc) return rc;
    const char* base = (const char*)c->buf[c->cur];
    const int total = c->q + ((g && c->qs) ? c->qs : 0);
    for (int a = 0; a < total; ++a) {
        const double off = a < c->q ? rest_weight_of(c, a) * c->cfg.rho0 : 0.0;
        double* dst = a < c->q ? f + (size_t)a * bn : g + (size_t)(a - c->q) * bn;
        HIP_OR_FAIL(c, launch_box_to_f64(c->cfg.storage, base + (size_t)a * c->plane * c->elem, c->staging, c->geo_aux, lo, ext, off, c->stream));
        HIP_OR_FAIL(c, hipMemcpyAsync(dst, c->staging, nb, hipMemcpyDeviceToHost, c->stream));
        HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    }
    return LB_OK;
}

int lb_totals(lb_ctx* c, double out[5]) {
    if (!c) return LB_EINVAL;
    if (!out) return fail(c, LB_EINVAL, "out is NULL");
    if (!c->initialised) return fail(c, LB_ESTATE, "state not initialised");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    double* d_out = nullptr;
    int rc = ensure_staging(c, kDiagSlots * sizeof(double));
    if (rc) return rc;
    d_out = c->staging;
    HIP_OR_FAIL(c, launch_totals(c->cfg.lattice, c->cfg.storage, c->geo_aux, c->buf[c->cur], c->partials, c->stream));
    HIP_OR_FAIL(c, launch_reduce(c->partials, c->geo_aux.grid_blocks, d_out, c->stream));
    double h[kDiagSlots];
    HIP_OR_FAIL(c, hipMemcpyAsync(h, d_out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    out[0] = (double)c->n * c->cfg.rho0 + h[0];
    out[1] = h[1];
    out[2] = h[2];
    out[3] = h[3];
    out[4] = h[4];
    return LB_OK;
}

int lb_totals_noalloc(lb_ctx* c, double* out_device) {
    if (!c) return LB_EINVAL;
    if (!out_device) return fail(c, LB_EINVAL, "out_device is NULL");
    if (!c->initialised) return fail(c, LB_ESTATE, "state not initialised");
    double* sp = nullptr;
    {
        // resolved by lb_create on this device; a device index beyond the table never got here
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (c->cfg.device >= 0 && c->cfg.device < kMaxDevices) sp = g_scratch_ptr[c->cfg.device];
    }
    if (!sp) return fail(c, LB_ESTATE, "no scratch address for device %d", c->cfg.device);
    const int64_t records = std::min<int64_t>(c->geo_aux.grid_blocks, kScratchRecords);
    if (records < 1 || records > kScratchRecords)
        return fail(c, LB_EINVAL, "%lld partial records exceed the scratch maximum of %lld", (long long)records,
                    (long long)kScratchRecords);
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    HIP_OR_FAIL(c, launch_totals_bounded(c->cfg.lattice, c->cfg.storage, c->geo_aux, c->buf[c->cur], sp, records,
                                         (double)c->n * c->cfg.rho0, out_device, c->stream));
    return LB_OK;
}

int lb_residual(lb_ctx* c, double* r, int64_t* at_step, double totals[5]) {
    if (!c) return LB_EINVAL;
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->check_pending = false;
    if (at_step) *at_step = c->check_step;
    const double* d = c->diag_host;
    if (r) {
        if (c->check_step < 0 || !c->check_valid)
            *r = INFINITY;
        else
            *r = sqrt(d[0]) / ((double)c->cfg.residual_interval * sqrt(d[1]));
    }
    if (totals) {
        totals[0] = (double)c->n * c->cfg.rho0 + d[2];
        totals[1] = d[3];
        totals[2] = d[4];
        totals[3] = d[5];
        totals[4] = d[6];
    }
    if (c->check_step >= 0 && d[7] > 0.0)
        return fail(c, LB_ENONFINITE, "non-finite values at step %lld", (long long)c->check_step);
    return LB_OK;
}

int lb_residual_scalar(lb_ctx* c, double* r_phi) {
    if (!c || !r_phi) return LB_EINVAL;
    if (!c->qs) return fail(c, LB_EINVAL, "the lattice has no scalar");
    HIP_OR_FAIL(c, hipSetDevice(c->cfg.device));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->check_pending = false;
    const double* d = c->diag_host;
    if (c->check_step < 0 || !c->check_valid)
        *r_phi = INFINITY;
    else
        *r_phi = sqrt(d[8]) / ((double)c->cfg.residual_interval * sqrt(d[9]));
    if (c->check_step >= 0 && d[7] > 0.0)
        return fail(c, LB_ENONFINITE, "non-finite values at step %lld", (long long)c->check_step);
    return LB_OK;
}

int lb_get_info(const lb_ctx* c, lb_info* info) {
    if (!c || !info) return LB_EINVAL;
    memset(info, 0, sizeof(*info));
    info->nodes = c->n;
    info->q = c->q;
    info->q_scalar = c->qs;
    info->plane_stride = c->plane;
    info->elem_bytes = c->elem;
    info->block_x = c->block;
    double b = 2.0 * (c->q + c->qs) * c->elem;
    if (c->force_field) b += (double)c->dims * c->real_bytes;
    if (c->source_field) b += (double)c->real_bytes;
    info->bytes_per_update = b;
    info->buf_current = c->buf[c->cur];
    info->buf_other = c->buf[c->cur ^ 1];
    static const char* names[12] = {"casclb_step<D2Q9,f64>", "casclb_step<D2Q9,f32dev>", "casclb_step<D2Q9,f16dev>",
                                   "casclb_step<D2Q9_D2Q5,f64>", "casclb_step<D2Q9_D2Q5,f32dev>", "casclb_step<D2Q9_D2Q5,f16dev>",
                                   "casclb_step<D3Q27,f64>", "casclb_step<D3Q27,f32dev>", "casclb_step<D3Q27,f16dev>",
                                   "casclb_step<D3Q15,f64>", "casclb_step<D3Q15,f32dev>", "casclb_step<D3Q15,f16dev>"};
    static const char* pair_names[4] = {"casclb_step_xpair<D2Q9,f16dev>", "casclb_step_xpair<D2Q9_D2Q5,f16dev>",
                                        "casclb_step_xpair<D3Q27,f16dev>", "casclb_step_xpair<D3Q15,f16dev>"};
    info->step_kernel = c->geo_step.xpair ? pair_names[c->cfg.lattice] : names[c->cfg.lattice * 3 + c->cfg.storage];
    return LB_OK;
}

int lb_stream_bench(void* dst, const void* src, size_t bytes, int32_t mode, int32_t width, int64_t blocks,
                    void* stream) {
    if (mode < 0 || mode > 2 || (width != 8 && width != 16) || bytes % 16 || blocks < 0) return LB_EINVAL;
    if (!dst || (mode != 2 && !src)) return LB_EINVAL;
    const int64_t nblocks = blocks > 0 ? blocks : (int64_t)(bytes / width + 1023) / 1024;
    if (mode == 1 && (size_t)nblocks * width > bytes) return LB_EINVAL;   // one vector per block goes to dst
    hipError_t e = launch_stream(dst, src, bytes, mode, width, blocks, (hipStream_t)stream);
    return e == hipSuccess ? LB_OK : LB_EHIP;
}

int lb_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src || bytes % 16) return LB_EINVAL;
    hipError_t e = launch_copy(dst, src, bytes, (hipStream_t)stream);
    return e == hipSuccess ? LB_OK : LB_EHIP;
}

}  // extern "C"
