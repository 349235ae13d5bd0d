// C ABI of the warm-start surrogate network (include/casclb_unet.h): buffer
// layout, the forward pass, the backward pass in reverse layer order and the
// Adam update, all as launches of the kernels in nn.hip on one stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "casclb_unet.h"
#include "nn.hpp"

using namespace casclb::nn;

namespace {

int up_to(int v, int m) { return (v + m - 1) / m * m; }

struct Layer {
    int co = 0, ci = 0;
    int64_t w_off = 0, b_off = 0;   // offsets in the flat parameter vector
    int ci_pad = 0, kpad = 0, co_pad32 = 0;          // forward weight layout
    int co_pad16 = 0, kpad_t = 0, ci_pad32 = 0;      // input-gradient weight layout
    int level = 0;                                   // resolution level it runs at
    bf16_t* wf = nullptr;
    bf16_t* wb = nullptr;
};

struct Level {
    int h = 0, w = 0;
    int c = 0, cin = 0, cat = 0;  // widths: features, level input, concat (or bottom) buffer
    bf16_t *in = nullptr, *a1 = nullptr, *cat_buf = nullptr, *d = nullptr;
    float *g_in = nullptr, *g_a1 = nullptr, *g_cat = nullptr, *g_d = nullptr;
};

}  // namespace

struct lb_unet {
    lb_unet_config cfg{};
    hipStream_t stream = nullptr;
    int L = 0, out16 = 0;
    int out_cs = 0;   // channel stride of the inference output: out_channels rounded up to 4
    std::vector<Layer> layers;
    std::vector<Level> lv;
    int64_t np = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float *out = nullptr, *g_out = nullptr;
    float* out_inf = nullptr;   // inference output, out_cs floats per pixel
    float* wpart = nullptr;
    int64_t wpart_n = 0;
    float* bpart = nullptr;
    int32_t bpart_blocks = 0;
    double* mse_part = nullptr;
    double* loss_dev = nullptr;
    double* loss_host = nullptr;
    int32_t mse_blocks = 512;
    int64_t t = 0;  // Adam steps taken
    // low-pass loss term: weight * MSE of the (2^lp x 2^lp)-block means
    int32_t lp_levels = 0;
    float lp_weight = 0.0f;
    std::vector<float*> lp_y, lp_t, lp_g;   // per level 1..lp_levels (index l - 1)
    int32_t last_batch = 0;
    // inference: the input is copied into xin, then the whole forward pass
    // (everything between that copy and the output unpacking) is replayed from
    // a graph captured once per batch size on a private stream
    float* xin = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<hipGraph_t> fwd_graph;
    std::vector<hipGraphExec_t> fwd_exec;
    std::vector<void*> allocs;
    std::string err;
};

static thread_local std::string g_unet_create_error;

static int ufail(lb_unet* n, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (n)
        n->err = buf;
    else
        g_unet_create_error = buf;
    return code;
}

#define UHIP(n, call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return ufail((n), LB_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static View view(void* base, int cs, int co) { return View{base, cs, co}; }

static void release(lb_unet* n) {
    for (auto& e : n->fwd_exec)
        if (e) (void)hipGraphExecDestroy(e);
    for (auto& g : n->fwd_graph)
        if (g) (void)hipGraphDestroy(g);
    n->fwd_exec.clear();
    n->fwd_graph.clear();
    if (n->cap_stream) (void)hipStreamDestroy(n->cap_stream);
    n->cap_stream = nullptr;
    for (void* q : n->allocs) (void)hipFree(q);
    n->allocs.clear();
    if (n->loss_host) (void)hipHostFree(n->loss_host);
    n->loss_host = nullptr;
}

template <class T>
static hipError_t dalloc(lb_unet* n, T** ptr, int64_t count) {
    *ptr = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc((void**)ptr, (size_t)count * sizeof(T));
    if (e != hipSuccess) return e;
    n->allocs.push_back((void*)*ptr);
    return hipMemsetAsync(*ptr, 0, (size_t)count * sizeof(T), n->stream);
}

extern "C" {

void lb_unet_config_default(lb_unet_config* c) {
    if (!c) return;
    memset(c, 0, sizeof(*c));
    c->abi_version = LB_UNET_ABI_VERSION;
    c->levels = 4;
    const int ch[4] = {16, 32, 48, 96};
    for (int i = 0; i < 4; ++i) c->channels[i] = ch[i];
    c->in_channels = 5;
    c->out_channels = 3;
    c->height = c->width = 256;
    c->max_batch = 16;
}

const char* lb_unet_last_error(const lb_unet* n) { return n ? n->err.c_str() : g_unet_create_error.c_str(); }

int64_t lb_unet_num_params(const lb_unet* n) { return n ? n->np : 0; }

double lb_unet_macs_per_image(const lb_unet* n) {
    if (!n) return 0.0;
    double s = 0.0;
    for (const Layer& l : n->layers) s += (double)n->lv[l.level].h * n->lv[l.level].w * 9.0 * l.ci * l.co;
    return s;
}

static int pack_all(lb_unet* n) {
    for (const Layer& l : n->layers)
        UHIP(n, launch_pack_weights(n->p + l.w_off, l.co, l.ci, l.wf, l.ci_pad, l.kpad, l.co_pad32, l.wb, l.co_pad16,
                                    l.kpad_t, l.ci_pad32, n->stream));
    return LB_OK;
}

int lb_unet_create(lb_unet** out, const lb_unet_config* cfg) {
    if (!out || !cfg) return ufail(nullptr, LB_EINVAL, "null argument");
    *out = nullptr;
    if (cfg->abi_version != LB_UNET_ABI_VERSION) return ufail(nullptr, LB_EINVAL, "abi_version %d", cfg->abi_version);
    const int L = cfg->levels;
    if (L < 1 || L > LB_UNET_MAX_LEVELS) return ufail(nullptr, LB_EINVAL, "levels must be 1..%d", LB_UNET_MAX_LEVELS);
    for (int l = 0; l < L; ++l)
        if (cfg->channels[l] < 16 || cfg->channels[l] > 256 || cfg->channels[l] % 16)
            return ufail(nullptr, LB_EINVAL, "channels[%d] = %d: need a multiple of 16 in [16, 256]", l, cfg->channels[l]);
    if (cfg->in_channels < 1 || cfg->in_channels > 16 || cfg->out_channels < 1 || cfg->out_channels > 16)
        return ufail(nullptr, LB_EINVAL, "in/out channels must be 1..16");
    const int mult = 4 << (L - 1);
    if (cfg->height < mult || cfg->width < mult || cfg->height % mult || cfg->width % mult)
        return ufail(nullptr, LB_EINVAL, "height and width must be multiples of %d", mult);
    if (cfg->max_batch < 1) return ufail(nullptr, LB_EINVAL, "max_batch must be >= 1");
    if ((int64_t)cfg->max_batch * cfg->height * cfg->width > (1LL << 30))
        return ufail(nullptr, LB_EINVAL, "max_batch * height * width too large");
    hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess) return ufail(nullptr, LB_EHIP, "hipSetDevice: %s", hipGetErrorString(e));

    lb_unet* n = new (std::nothrow) lb_unet();
    if (!n) return ufail(nullptr, LB_ENOMEM, "host allocation failed");
    n->cfg = *cfg;
    n->stream = (hipStream_t)cfg->stream;
    n->L = L;
    n->out16 = 16;
    n->out_cs = (cfg->out_channels + 3) / 4 * 4;
    n->lv.resize(L);
    for (int l = 0; l < L; ++l) {
        Level& q = n->lv[l];
        q.h = cfg->height >> l;
        q.w = cfg->width >> l;
        q.c = cfg->channels[l];
        q.cin = l == 0 ? 16 : cfg->channels[l - 1];
        q.cat = l < L - 1 ? cfg->channels[l] + cfg->channels[l + 1] : cfg->channels[l];
    }
    // layers in parameter order
    auto add = [&](int co, int ci, int level) {
        Layer y;
        y.co = co;
        y.ci = ci;
        y.level = level;
        y.w_off = n->np;
        n->np += (int64_t)co * 9 * ci;
        y.b_off = n->np;
        n->np += co;
        y.ci_pad = up_to(ci, 16);
        y.kpad = up_to(9 * y.ci_pad, 32);
        y.co_pad32 = up_to(co, 32);
        y.co_pad16 = up_to(co, 16);
        y.kpad_t = up_to(9 * y.co_pad16, 32);
        y.ci_pad32 = up_to(ci, 32);
        n->layers.push_back(y);
    };
    for (int l = 0; l < L; ++l) {
        add(cfg->channels[l], l == 0 ? cfg->in_channels : cfg->channels[l - 1], l);
        add(cfg->channels[l], cfg->channels[l], l);
    }
    for (int l = L - 2; l >= 0; --l) add(cfg->channels[l], cfg->channels[l] + cfg->channels[l + 1], l);
    add(cfg->out_channels, cfg->channels[0], 0);

    const int64_t B = cfg->max_batch;
    int rc = LB_OK;
#define UALLOC(ptr, count)                                                                           \
    do {                                                                                             \
        hipError_t ae_ = dalloc(n, &(ptr), (count));                                                 \
        if (ae_ != hipSuccess) {                                                                     \
            rc = ufail(nullptr, LB_ENOMEM, "device allocation: %s", hipGetErrorString(ae_));         \
            goto error;                                                                              \
        }                                                                                            \
    } while (0)
    UALLOC(n->p, n->np);
    UALLOC(n->g, n->np);
    UALLOC(n->m, n->np);
    UALLOC(n->v, n->np);
    for (Layer& y : n->layers) {
        UALLOC(y.wf, (int64_t)y.co_pad32 * y.kpad);
        UALLOC(y.wb, (int64_t)y.ci_pad32 * y.kpad_t);
    }
    for (int l = 0; l < L; ++l) {
        Level& q = n->lv[l];
        const int64_t P = B * q.h * q.w;
        UALLOC(q.in, P * q.cin);
        UALLOC(q.a1, P * q.c);
        UALLOC(q.cat_buf, P * q.cat);
        UALLOC(q.g_a1, P * q.c);
        UALLOC(q.g_cat, P * q.cat);
        if (l > 0) UALLOC(q.g_in, P * q.cin);
        if (l < L - 1) {
            UALLOC(q.d, P * q.c);
            UALLOC(q.g_d, P * q.c);
        }
    }
    {
        const int64_t P0 = B * cfg->height * cfg->width;
        UALLOC(n->out, P0 * n->out16);
        UALLOC(n->g_out, P0 * n->out16);
        UALLOC(n->out_inf, P0 * n->out_cs);
        int64_t wmax = 0;
        int32_t bmax = 0;
        for (const Layer& y : n->layers) {
            const int64_t P = B * n->lv[y.level].h * n->lv[y.level].w;
            int32_t cpw = 0;
            const int32_t splits = wgrad_splits(P, &cpw);
            wmax = std::max(wmax, (int64_t)splits * up_to(y.co, 16) * 9 * up_to(y.ci, 16));
            bmax = std::max(bmax, bias_grad_blocks(P) * (int32_t)y.co);
        }
        n->wpart_n = wmax;
        UALLOC(n->wpart, wmax);
        n->bpart_blocks = 4096;
        UALLOC(n->bpart, bmax);
        UALLOC(n->mse_part, n->mse_blocks);
        UALLOC(n->loss_dev, 2);
        UALLOC(n->xin, P0 * cfg->in_channels);
    }
#undef UALLOC
    e = hipHostMalloc((void**)&n->loss_host, 2 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        rc = ufail(nullptr, LB_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
        goto error;
    }
    rc = pack_all(n);
    if (rc) {
        g_unet_create_error = n->err;
        goto error;
    }
    e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) {
        rc = ufail(nullptr, LB_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
        goto error;
    }
    *out = n;
    return LB_OK;
error:
    release(n);
    delete n;
    return rc;
}

void lb_unet_destroy(lb_unet* n) {
    if (!n) return;
    (void)hipSetDevice(n->cfg.device);
    (void)hipStreamSynchronize(n->stream);
    release(n);
    delete n;
}

int lb_unet_set_params(lb_unet* n, const float* params_host) {
    if (!n || !params_host) return LB_EINVAL;
    UHIP(n, hipSetDevice(n->cfg.device));
    UHIP(n, hipStreamSynchronize(n->stream));
    UHIP(n, hipMemcpy(n->p, params_host, sizeof(float) * n->np, hipMemcpyHostToDevice));
    UHIP(n, hipMemsetAsync(n->m, 0, sizeof(float) * n->np, n->stream));
    UHIP(n, hipMemsetAsync(n->v, 0, sizeof(float) * n->np, n->stream));
    n->t = 0;
    int rc = pack_all(n);
    if (rc) return rc;
    UHIP(n, hipStreamSynchronize(n->stream));
    return LB_OK;
}

int lb_unet_get_params(lb_unet* n, float* params_host) {
    if (!n || !params_host) return LB_EINVAL;
    UHIP(n, hipSetDevice(n->cfg.device));
    UHIP(n, hipStreamSynchronize(n->stream));
    UHIP(n, hipMemcpy(params_host, n->p, sizeof(float) * n->np, hipMemcpyDeviceToHost));
    return LB_OK;
}

// Forward convolution of layer y with the LDS-tiled kernel where the level's
// size allows (fusions: x2 = half-resolution source of the channels from
// c_split on, pool = 2 x 2 means of the output, xin = raw fp32 input with
// cin_raw channels); returns 1 without launching when it does not apply.
static int conv_tiled(lb_unet* n, const Layer& y, View x, View out, bool out_f32, int batch, bool relu, View x2,
                      int c_split, View pool, const float* xin, int cin_raw) {
    const Level& q = n->lv[y.level];
    if (!conv_tiled_fits(q.h, q.w, y.ci_pad)) return 1;
    ConvArgs a{};
    a.x = x;
    a.y = out;
    a.wt = y.wf;
    a.bias = n->p + y.b_off;
    a.n = batch;
    a.h = q.h;
    a.w = q.w;
    a.ci_pad = y.ci_pad;
    a.kpad = y.kpad;
    a.co = y.co;
    a.co_pad32 = y.co_pad32;
    a.relu = relu ? 1 : 0;
    a.accumulate = 0;
    a.x2 = x2;
    a.c_split = x2.base ? c_split : y.ci_pad;
    a.pool = pool;
    a.xin = xin;
    a.cin_raw = cin_raw;
    if (!conv_tiled_offsets_fit(a)) return 1;
    UHIP(n, launch_conv_tiled(a, out_f32, n->stream));
    return LB_OK;
}

static int conv(lb_unet* n, const Layer& y, View x, bool x_f32, View out, bool out_f32, int batch, bool relu) {
    const Level& q = n->lv[y.level];
    ConvArgs a{};
    a.x = x;
    a.y = out;
    a.wt = y.wf;
    a.bias = n->p + y.b_off;
    a.n = batch;
    a.h = q.h;
    a.w = q.w;
    a.ci_pad = y.ci_pad;
    a.kpad = y.kpad;
    a.co = y.co;
    a.co_pad32 = y.co_pad32;
    a.relu = relu ? 1 : 0;
    a.accumulate = 0;
    UHIP(n, launch_conv(a, x_f32, out_f32, n->stream));
    return LB_OK;
}

// input gradient of layer y: dx (fp32 view, y.ci channels) = conv(g, flipped W^T)
static int dgrad(lb_unet* n, const Layer& y, View g, View dx, int batch) {
    const Level& q = n->lv[y.level];
    ConvArgs a{};
    a.x = g;
    a.y = dx;
    a.wt = y.wb;
    a.bias = nullptr;
    a.n = batch;
    a.h = q.h;
    a.w = q.w;
    a.ci_pad = y.co_pad16;
    a.kpad = y.kpad_t;
    a.co = y.ci;
    a.co_pad32 = y.ci_pad32;
    a.relu = 0;
    a.accumulate = 0;
    // on launches that fill the chip (more than 512 tiles) the LDS-tiled kernel reads a
    // dense fp32 gradient (channel offset 0, stride = its padded channel count, up to 48)
    // as its raw input: the same bf16 operands and K order as the plain kernel, so the
    // same sums; on smaller launches its staging rounds cost more than they save
    const bool wide = a.w % 32 == 0 && a.h % 8 == 0;
    const int64_t tiles = (int64_t)batch * (a.h / (wide ? 8 : 16)) * (a.w / (wide ? 32 : 16));
    if (tiles > 512 && g.co == 0 && g.cs == a.ci_pad && g.cs <= 48 && conv_tiled_fits(a.h, a.w, a.ci_pad)) {
        ConvArgs t = a;
        t.x = View{nullptr, 0, 0};
        t.x2 = View{nullptr, 0, 0};
        t.c_split = a.ci_pad;
        t.pool = View{nullptr, 0, 0};
        t.xin = reinterpret_cast<const float*>(g.base);
        t.cin_raw = g.cs;
        if (conv_tiled_offsets_fit(t)) {
            UHIP(n, launch_conv_tiled(t, true, n->stream));
            return LB_OK;
        }
    }
    UHIP(n, launch_conv(a, true, true, n->stream));
    return LB_OK;
}

// weight and bias gradients of layer y from its output gradient g (fp32) and input x (bf16)
static int wgrad(lb_unet* n, const Layer& y, View g, View x, int batch) {
    const Level& q = n->lv[y.level];
    const int64_t P = (int64_t)batch * q.h * q.w;
    WgradArgs a{};
    a.g = g;
    a.x = x;
    a.n = batch;
    a.h = q.h;
    a.w = q.w;
    a.co = y.co;
    a.ci = y.ci;
    a.co_pad16 = up_to(y.co, 16);
    a.ci_pad16 = up_to(y.ci, 16);
    a.splits = wgrad_splits(P, &a.chunks_per_wave);
    if ((int64_t)a.splits * a.co_pad16 * 9 * a.ci_pad16 > n->wpart_n)
        return ufail(n, LB_EINVAL, "internal: weight-gradient scratch too small");
    a.partials = n->wpart;
    a.out = n->g + y.w_off;
    a.accumulate = 0;
    UHIP(n, launch_wgrad(a, n->stream));
    UHIP(n, launch_bias_grad(g, P, y.co, n->bpart, n->bpart_blocks, n->g + y.b_off, 0, n->stream));
    return LB_OK;
}

static int check_batch(lb_unet* n, int32_t batch) {
    if (batch < 1 || batch > n->cfg.max_batch)
        return ufail(n, LB_EINVAL, "batch %d outside 1..%d", batch, n->cfg.max_batch);
    return LB_OK;
}

// forward pass into n->out (fp32, out16 channels; for inference n->out_inf, out_cs
// channels).  Pooling is fused into the
// second convolution of each encoder level wherever the tiled kernel applies.
// For inference (train = false) the first convolution also reads the raw input
// and each decoder convolution reads the coarser level's output at half
// resolution itself; training materialises the packed input and the
// concatenated decoder inputs, which the backward pass reads.
static int forward(lb_unet* n, const float* x, int batch, bool train = true) {
    const int L = n->L;
    const int64_t P0 = (int64_t)batch * n->cfg.height * n->cfg.width;
    const View none{nullptr, 0, 0};
    int rc;
    bool packed = false;
    for (int l = 0; l < L; ++l) {
        Level& q = n->lv[l];
        const View a1 = view(q.a1, q.c, 0), cat = view(q.cat_buf, q.cat, 0);
        if (l == 0 && !train) {
            rc = conv_tiled(n, n->layers[0], none, a1, false, batch, true, none, 0, none, x, n->cfg.in_channels);
            if (rc < 0) return rc;
        } else {
            rc = 1;
        }
        if (rc == 1) {
            if (l == 0 && !packed) {
                UHIP(n, launch_pack_input(x, n->cfg.in_channels, view(n->lv[0].in, 16, 0), 16, P0, n->stream));
                packed = true;
            }
            rc = conv_tiled(n, n->layers[2 * l], view(q.in, q.cin, 0), a1, false, batch, true, none, 0, none, nullptr, 0);
            if (rc < 0) return rc;
            if (rc == 1 && (rc = conv(n, n->layers[2 * l], view(q.in, q.cin, 0), false, a1, false, batch, true)))
                return rc;
        }
        const View pool = l < L - 1 ? view(n->lv[l + 1].in, n->lv[l + 1].cin, 0) : none;
        rc = conv_tiled(n, n->layers[2 * l + 1], a1, cat, false, batch, true, none, 0, pool, nullptr, 0);
        if (rc < 0) return rc;
        if (rc == 1) {
            if ((rc = conv(n, n->layers[2 * l + 1], a1, false, cat, false, batch, true))) return rc;
            if (l < L - 1) UHIP(n, launch_avgpool(cat, pool, batch, q.h, q.w, q.c, n->stream));
        }
    }
    int li = 2 * L;
    for (int l = L - 2; l >= 0; --l, ++li) {
        Level& q = n->lv[l];
        const Level& r = n->lv[l + 1];
        const View src = l + 1 == L - 1 ? view(r.cat_buf, r.cat, 0) : view(r.d, r.c, 0);
        const View cat = view(q.cat_buf, q.cat, 0), d = view(q.d, q.c, 0);
        rc = 1;
        if (!train) {
            rc = conv_tiled(n, n->layers[li], cat, d, false, batch, true, src, q.c, none, nullptr, 0);
            if (rc < 0) return rc;
        }
        if (rc == 1) {
            UHIP(n, launch_upsample(src, view(q.cat_buf, q.cat, q.c), batch, q.h, q.w, r.c, n->stream));
            rc = conv_tiled(n, n->layers[li], cat, d, false, batch, true, none, 0, none, nullptr, 0);
            if (rc < 0) return rc;
            if (rc == 1 && (rc = conv(n, n->layers[li], cat, false, d, false, batch, true))) return rc;
        }
    }
    const Level& q0 = n->lv[0];
    const View top = L == 1 ? view(q0.cat_buf, q0.cat, 0) : view(q0.d, q0.c, 0);
    // training keeps 16 channels per pixel (the gradient kernels read 8 at a time); inference
    // writes out_cs, so that the result leaves as one copy when out_channels is a multiple of 4
    const View outv = train ? view(n->out, n->out16, 0) : view(n->out_inf, n->out_cs, 0);
    rc = conv_tiled(n, n->layers[li], top, outv, true, batch, false, none, 0, none, nullptr, 0);
    if (rc < 0) return rc;
    if (rc == 1) return conv(n, n->layers[li], top, false, outv, true, batch, false);
    return LB_OK;
}

// The captured inference pass for `batch` images (reads xin, writes out).
static int forward_graph(lb_unet* n, int batch, hipGraphExec_t* out) {
    if (n->fwd_exec.empty()) {
        n->fwd_exec.assign(n->cfg.max_batch + 1, nullptr);
        n->fwd_graph.assign(n->cfg.max_batch + 1, nullptr);
    }
    if (n->fwd_exec[batch]) {
        *out = n->fwd_exec[batch];
        return LB_OK;
    }
    if (!n->cap_stream) UHIP(n, hipStreamCreateWithFlags(&n->cap_stream, hipStreamNonBlocking));
    const hipStream_t own = n->stream;
    UHIP(n, hipStreamBeginCapture(n->cap_stream, hipStreamCaptureModeThreadLocal));
    n->stream = n->cap_stream;
    const int rc = forward(n, n->xin, batch, false);
    n->stream = own;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(n->cap_stream, &g);
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : ufail(n, LB_EHIP, "forward graph capture: %s", hipGetErrorString(e));
    }
    n->fwd_graph[batch] = g;
    UHIP(n, hipGraphInstantiate(&n->fwd_exec[batch], g, nullptr, nullptr, 0));
    *out = n->fwd_exec[batch];
    return LB_OK;
}

int lb_unet_forward(lb_unet* n, const float* x_dev, int32_t batch, float* y_dev) {
    if (!n || !x_dev || !y_dev) return LB_EINVAL;
    int rc = check_batch(n, batch);
    if (rc) return rc;
    UHIP(n, hipSetDevice(n->cfg.device));
    const int64_t P0 = (int64_t)batch * n->cfg.height * n->cfg.width;
    hipGraphExec_t ge = nullptr;
    if ((rc = forward_graph(n, batch, &ge))) return rc;
    UHIP(n, hipMemcpyAsync(n->xin, x_dev, sizeof(float) * P0 * n->cfg.in_channels, hipMemcpyDeviceToDevice,
                           n->stream));
    UHIP(n, hipGraphLaunch(ge, n->stream));
    if (n->out_cs == n->cfg.out_channels)
        UHIP(n, hipMemcpyAsync(y_dev, n->out_inf, sizeof(float) * P0 * n->out_cs, hipMemcpyDeviceToDevice,
                               n->stream));
    else
        UHIP(n, launch_unpack_output(view(n->out_inf, n->out_cs, 0), n->cfg.out_channels, y_dev, P0, n->stream));
    return LB_OK;
}

static int backward(lb_unet* n, int batch) {
    const int L = n->L;
    int rc;
    // output layer
    const Layer& last = n->layers[3 * L - 1];
    Level& q0 = n->lv[0];
    const View top = L == 1 ? view(q0.cat_buf, q0.cat, 0) : view(q0.d, q0.c, 0);
    const View gtop = L == 1 ? view(q0.g_cat, q0.cat, 0) : view(q0.g_d, q0.c, 0);
    const View gout = view(n->g_out, n->out16, 0);
    if ((rc = wgrad(n, last, gout, top, batch))) return rc;
    if ((rc = dgrad(n, last, gout, gtop, batch))) return rc;
    // decoder, level 0 upwards (reverse of the forward order)
    for (int l = 0; l <= L - 2; ++l) {
        Level& q = n->lv[l];
        const Level& r = n->lv[l + 1];
        const Layer& y = n->layers[2 * L + (L - 2 - l)];
        const int64_t P = (int64_t)batch * q.h * q.w;
        UHIP(n, launch_relu_mask(view(q.g_d, q.c, 0), view(q.d, q.c, 0), P, q.c, n->stream));
        if ((rc = wgrad(n, y, view(q.g_d, q.c, 0), view(q.cat_buf, q.cat, 0), batch))) return rc;
        if ((rc = dgrad(n, y, view(q.g_d, q.c, 0), view(q.g_cat, q.cat, 0), batch))) return rc;
        const View dst = l + 1 == L - 1 ? view(r.g_cat, r.cat, 0) : view(r.g_d, r.c, 0);
        UHIP(n, launch_upsample_bwd(view(q.g_cat, q.cat, q.c), dst, batch, q.h, q.w, r.c, n->stream));
    }
    // encoder, bottom level first
    for (int l = L - 1; l >= 0; --l) {
        Level& q = n->lv[l];
        const int64_t P = (int64_t)batch * q.h * q.w;
        const View g2 = view(q.g_cat, q.cat, 0);
        UHIP(n, launch_relu_mask(g2, view(q.cat_buf, q.cat, 0), P, q.c, n->stream));
        if ((rc = wgrad(n, n->layers[2 * l + 1], g2, view(q.a1, q.c, 0), batch))) return rc;
        if ((rc = dgrad(n, n->layers[2 * l + 1], g2, view(q.g_a1, q.c, 0), batch))) return rc;
        UHIP(n, launch_relu_mask(view(q.g_a1, q.c, 0), view(q.a1, q.c, 0), P, q.c, n->stream));
        if ((rc = wgrad(n, n->layers[2 * l], view(q.g_a1, q.c, 0), view(q.in, q.cin, 0), batch))) return rc;
        if (l > 0) {
            Level& u = n->lv[l - 1];
            if ((rc = dgrad(n, n->layers[2 * l], view(q.g_a1, q.c, 0), view(q.g_in, q.cin, 0), batch))) return rc;
            UHIP(n, launch_avgpool_bwd(view(q.g_in, q.cin, 0), view(u.g_cat, u.cat, 0), batch, u.h, u.w, u.c,
                                       n->stream));
        }
    }
    return LB_OK;
}

static int loss_grad(lb_unet* n, const float* x, const float* target, int batch) {
    int rc = forward(n, x, batch);
    if (rc) return rc;
    const int64_t P0 = (int64_t)batch * n->cfg.height * n->cfg.width;
    const int oc = n->cfg.out_channels;
    UHIP(n, launch_mse(view(n->out, n->out16, 0), target, oc, P0, view(n->g_out, n->out16, 0), n->mse_part,
                       n->mse_blocks, 1.0f, n->stream));
    UHIP(n, launch_sum(n->mse_part, n->mse_blocks, n->loss_dev, n->stream));
    if (n->lp_levels > 0 && n->lp_weight > 0.0f) {
        // block means of output and target, their weighted MSE, and its gradient
        // carried back to the full grid and added to the output gradient
        View ys = view(n->out, n->out16, 0), ts = view((void*)target, oc, 0);
        for (int l = 1; l <= n->lp_levels; ++l) {
            const int h = n->cfg.height >> (l - 1), w = n->cfg.width >> (l - 1);
            const View yd = view(n->lp_y[l - 1], n->out16, 0), td = view(n->lp_t[l - 1], oc, 0);
            UHIP(n, launch_avgpool_f32(ys, yd, batch, h, w, oc, n->stream));
            UHIP(n, launch_avgpool_f32(ts, td, batch, h, w, oc, n->stream));
            ys = yd;
            ts = td;
        }
        const int L = n->lp_levels;
        const int64_t Pl = (int64_t)batch * (n->cfg.height >> L) * (n->cfg.width >> L);
        UHIP(n, launch_mse(ys, n->lp_t[L - 1], oc, Pl, view(n->lp_g[L - 1], n->out16, 0), n->mse_part,
                           n->mse_blocks, n->lp_weight, n->stream));
        UHIP(n, launch_sum(n->mse_part, n->mse_blocks, n->loss_dev + 1, n->stream));
        for (int l = L; l >= 1; --l) {
            const int h = n->cfg.height >> (l - 1), w = n->cfg.width >> (l - 1);
            const View dst = l == 1 ? view(n->g_out, n->out16, 0) : view(n->lp_g[l - 2], n->out16, 0);
            UHIP(n, launch_unpool_f32(view(n->lp_g[l - 1], n->out16, 0), dst, batch, h, w, oc, l == 1 ? 1 : 0,
                                      n->stream));
        }
    }
    n->last_batch = batch;
    return backward(n, batch);
}

int lb_unet_loss_grad(lb_unet* n, const float* x_dev, const float* target_dev, int32_t batch, double* loss,
                      float* grad_host) {
    if (!n || !x_dev || !target_dev) return LB_EINVAL;
    int rc = check_batch(n, batch);
    if (rc) return rc;
    UHIP(n, hipSetDevice(n->cfg.device));
    if ((rc = loss_grad(n, x_dev, target_dev, batch))) return rc;
    if (loss) {
        UHIP(n, hipMemcpyAsync(n->loss_host, n->loss_dev, 2 * sizeof(double), hipMemcpyDeviceToHost, n->stream));
        UHIP(n, hipStreamSynchronize(n->stream));
        const double oc = n->cfg.out_channels;
        *loss = n->loss_host[0] / ((double)batch * n->cfg.height * n->cfg.width * oc);
        if (n->lp_levels > 0 && n->lp_weight > 0.0f)
            *loss += n->lp_weight * n->loss_host[1] /
                     ((double)batch * (n->cfg.height >> n->lp_levels) * (n->cfg.width >> n->lp_levels) * oc);
    }
    if (grad_host) {
        UHIP(n, hipStreamSynchronize(n->stream));
        UHIP(n, hipMemcpy(grad_host, n->g, sizeof(float) * n->np, hipMemcpyDeviceToHost));
    }
    return LB_OK;
}

int lb_unet_set_lowpass_loss(lb_unet* n, int32_t levels, float weight) {
    if (!n) return LB_EINVAL;
    int maxl = 0;
    while ((n->cfg.height >> (maxl + 1)) >= 1 && (n->cfg.width >> (maxl + 1)) >= 1 &&
           (n->cfg.height % (2 << maxl)) == 0 && (n->cfg.width % (2 << maxl)) == 0)
        ++maxl;
    if (levels < 0 || levels > maxl) return ufail(n, LB_EINVAL, "levels must be 0..%d", maxl);
    if (!(weight >= 0.0f) || !isfinite(weight)) return ufail(n, LB_EINVAL, "weight must be >= 0");
    UHIP(n, hipSetDevice(n->cfg.device));
    for (int l = (int)n->lp_y.size() + 1; l <= levels; ++l) {
        const int64_t P = (int64_t)n->cfg.max_batch * (n->cfg.height >> l) * (n->cfg.width >> l);
        float *y = nullptr, *t = nullptr, *g = nullptr;
        hipError_t e = dalloc(n, &y, P * n->out16);
        if (e == hipSuccess) e = dalloc(n, &t, P * n->cfg.out_channels);
        if (e == hipSuccess) e = dalloc(n, &g, P * n->out16);
        if (e != hipSuccess) return ufail(n, LB_ENOMEM, "device allocation: %s", hipGetErrorString(e));
        n->lp_y.push_back(y);
        n->lp_t.push_back(t);
        n->lp_g.push_back(g);
    }
    UHIP(n, hipStreamSynchronize(n->stream));
    n->lp_levels = levels;
    n->lp_weight = weight;
    return LB_OK;
}

int lb_unet_adam(lb_unet* n, float lr, float beta1, float beta2, float eps) {
    if (!n) return LB_EINVAL;
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return ufail(n, LB_EINVAL, "bad Adam hyper-parameters");
    if (n->last_batch == 0) return ufail(n, LB_ESTATE, "no gradient computed yet");
    UHIP(n, hipSetDevice(n->cfg.device));
    n->t += 1;
    const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)n->t)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)n->t)));
    UHIP(n, launch_adam(n->p, n->g, n->m, n->v, n->np, lr, beta1, beta2, eps, c1, c2, n->stream));
    return pack_all(n);
}

int lb_unet_train_step(lb_unet* n, const float* x_dev, const float* target_dev, int32_t batch, float lr,
                       double* loss) {
    int rc = lb_unet_loss_grad(n, x_dev, target_dev, batch, loss, nullptr);
    if (rc) return rc;
    return lb_unet_adam(n, lr, 0.9f, 0.999f, 1e-8f);
}

}  // extern "C"
