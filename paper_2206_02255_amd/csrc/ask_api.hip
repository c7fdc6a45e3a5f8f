// Host engine and C ABI (include/ask.h): argument checks, mapping constants,
// level count, queue memory, and the launch sequences of the exhaustive image
// and the three subdivision forms.
#include "ask.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "ask_internal.hpp"

using namespace ask;

struct ask_ctx {
    int device = 0;
    int cus = 0;
    int occ_level = 1;       // resident 256-lane blocks per CU, per-level kernel
    int occ_persistent = 1;  // same, persistent kernel
    uint32_t *ctrl = nullptr;
    DevStats *stats = nullptr;
    Region *lvq[2] = {nullptr, nullptr};  // read/write tables of the per-level form
    size_t lvq_cap = 0;                   // entries per table
    Region *queue = nullptr;              // persistent queue
    size_t queue_cap = 0;
    uint32_t epoch = 0;                   // 24-bit launch counter for queue tags
    double wait_limit_s = 10.0;           // persistent kernel: longest wait of one wave
    double clock_hz = 1e8;                // rate of the device's constant clock
    bool timing = false;                  // record events around the dominant kernels
    bool timed = false;                   // the events hold a render
    hipEvent_t ev[2] = {nullptr, nullptr};
    // Batches: image table and level-0 seed offsets on the device, staged
    // through pinned host memory whose last copy `staged` marks.
    void *table = nullptr;
    size_t table_bytes = 0;
    void *staging = nullptr;
    size_t staging_bytes = 0;
    hipEvent_t staged = nullptr;
    char err[512] = {0};
};

namespace {

// Entries per queue buffer never exceed this (1 GiB of 16-byte entries); a
// render whose worst case needs more is checked for overflow after it runs.
constexpr uint64_t kQueueBudget = 64ull << 20;

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
            (void)hipSetDevice(prev);
    }
};

ask_status fail(ask_ctx *ctx, ask_status s, const char *fmt, const char *detail) {
    if (ctx)
        snprintf(ctx->err, sizeof(ctx->err), fmt, detail ? detail : "");
    return s;
}

ask_status hip_fail(ask_ctx *ctx, hipError_t e, const char *where) {
    if (ctx)
        snprintf(ctx->err, sizeof(ctx->err), "%s: %s", where, hipGetErrorString(e));
    return ASK_EDEVICE;
}

ask_status check_window(const ask_window *w) {
    if (!w)
        return ASK_EINVAL;
    if (!std::isfinite(w->x0) || !std::isfinite(w->x1) || !std::isfinite(w->y0) ||
        !std::isfinite(w->y1))
        return ASK_EINVAL;
    if (!(w->x0 < w->x1) || !(w->y0 < w->y1))
        return ASK_EINVAL;
    if (w->W < 1 || w->H < 1 || w->W > 65536 || w->H > 65536)
        return ASK_EINVAL;
    if (w->D < 1 || w->D > 0x7fffffffu || w->reserved != 0)
        return ASK_EINVAL;
    return ASK_OK;
}

ask_status check_params(const ask_window *w, const ask_params *p) {
    if (!p)
        return ASK_EINVAL;
    if (p->g < 1 || p->g > w->W || p->g > w->H)
        return ASK_EINVAL;
    if (p->r < 2 || p->r > 1024 || p->B < 1 || p->B > 65536)
        return ASK_EINVAL;
    if (p->form > ASK_FORM_PERSISTENT)
        return ASK_EINVAL;
    return ASK_OK;
}

// Mapping constants, binary64, in this order (the kernels never divide).
void mapping(const ask_window *w, double m[4]) {
    m[0] = 0.5 * (w->x0 + w->x1);
    m[1] = 0.5 * (w->y0 + w->y1);
    m[2] = (w->x1 - w->x0) / (2.0 * (double)w->W);
    m[3] = (w->y1 - w->y0) / (2.0 * (double)w->H);
}

// Largest side of a level-0 piece, then of an r-fold piece of it: the floor
// partition of a length n into p pieces has pieces of at most ceil(n/p).
uint32_t level_count(uint32_t W, uint32_t H, uint32_t g, uint32_t r, uint32_t B) {
    uint64_t s = std::max((W + g - 1) / g, (H + g - 1) / g);
    uint32_t levels = 1;
    while (s > B) {
        s = (s + r - 1) / r;
        ++levels;
    }
    return levels;
}

// Upper bound on the regions of one level: at most g^2 r^(2 lv), and at most
// one per pixel, since the regions of a level are disjoint and non-empty.
uint64_t level_bound(uint64_t pixels, uint32_t g, uint32_t r, uint32_t lv) {
    double b = (double)g * g * std::pow((double)r * r, (double)lv);
    return b >= (double)pixels ? pixels : (uint64_t)b;
}

Image make_image(const ask_window *w, const ask_params *p, uint32_t *out) {
    double m[4];
    mapping(w, m);
    Image im{};
    im.cxm = m[0];
    im.cym = m[1];
    im.hx = m[2];
    im.hy = m[3];
    im.W = w->W;
    im.H = w->H;
    im.D = w->D;
    im.g = p ? p->g : 1;
    im.r = p ? p->r : 2;
    im.B = p ? p->B : 1;
    im.out = out;
    return im;
}

ask_status grow(ask_ctx *ctx, Region **buf, size_t *cap, size_t need, bool clear) {
    if (*cap >= need)
        return ASK_OK;
    const size_t n = std::max<size_t>(need, std::min<size_t>(*cap * 2, kQueueBudget));
    hipError_t e;
    if (*buf) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess)
            return hip_fail(ctx, e, "hipDeviceSynchronize");
        (void)hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
    }
    e = hipMalloc((void **)buf, n * sizeof(Region));
    if (e != hipSuccess) {
        *buf = nullptr;
        (void)hipGetLastError();
        return fail(ctx, ASK_ENOMEM, "cannot allocate the region queue%s", nullptr);
    }
    if (clear) {
        e = hipMemset(*buf, 0, n * sizeof(Region));
        if (e != hipSuccess)
            return hip_fail(ctx, e, "hipMemset");
    }
    *cap = n;
    return ASK_OK;
}

// Wait for the stream, then take (and clear) the error bits the kernels
// recorded since the last check.
ask_status take_errors(ask_ctx *ctx, hipStream_t s) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "hipStreamSynchronize");
    uint32_t bits = 0;
    e = hipMemcpy(&bits, ctx->ctrl + kSticky, sizeof(bits), hipMemcpyDeviceToHost);
    if (e == hipSuccess && bits) {
        const uint32_t zero = 0;
        e = hipMemcpy(ctx->ctrl + kSticky, &zero, sizeof(zero), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess)
        return hip_fail(ctx, e, "hipMemcpy");
    if (bits & kErrTimeout)
        return fail(ctx, ASK_ETIMEOUT, "a persistent wave waited longer than the wait limit%s",
                    nullptr);
    if (bits & kErrOverflow)
        return fail(ctx, ASK_EOVERFLOW, "region queue overflow%s", nullptr);
    return ASK_OK;
}

ask_status read_stats(ask_ctx *ctx, hipStream_t s, ask_stats *out) {
    ask_status st = take_errors(ctx, s);
    hipError_t e;
    uint32_t ov = 0;
    e = hipMemcpy(&ov, ctx->ctrl + kOverflow, sizeof(ov), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "hipMemcpy");
    if (out) {
        DevStats ds;
        e = hipMemcpy(&ds, ctx->stats, sizeof(ds), hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "hipMemcpy");
        memset(out, 0, sizeof(*out));
        out->levels = ds.levels;
        out->overflow = ov;
        for (int i = 0; i < kMaxLevels; ++i) {
            out->regions[i] = ds.regions[i];
            out->fills[i] = ds.fills[i];
            out->splits[i] = ds.splits[i];
            out->leaves[i] = ds.leaves[i];
        }
        out->iters_ring = ds.iters_ring;
        out->iters_leaf = ds.iters_leaf;
    }
    return st;
}

hipError_t mark(ask_ctx *ctx, int which, hipStream_t s) {
    if (!ctx->timing)
        return hipSuccess;
    if (which == 1)
        ctx->timed = true;
    return hipEventRecord(ctx->ev[which], s);
}

}  // namespace

extern "C" {

const char *ask_status_str(ask_status s) {
    switch (s) {
    case ASK_OK: return "ok";
    case ASK_EINVAL: return "invalid argument";
    case ASK_ENOMEM: return "out of memory";
    case ASK_EDEVICE: return "device error";
    case ASK_EOVERFLOW: return "region queue overflow";
    case ASK_EBUSY: return "busy";
    case ASK_ETIMEOUT: return "timed out";
    }
    return "unknown status";
}

const char *ask_last_error(const ask_ctx *ctx) { return ctx ? ctx->err : ""; }

ask_status ask_validate(const ask_window *win, const ask_params *params) {
    ask_status s = check_window(win);
    if (s != ASK_OK || !params)
        return s;
    return check_params(win, params);
}

ask_status ask_mapping(const ask_window *win, double out[4]) {
    ask_status s = check_window(win);
    if (s != ASK_OK || !out)
        return ASK_EINVAL;
    mapping(win, out);
    return ASK_OK;
}

ask_status ask_level_count(const ask_window *win, const ask_params *params, uint32_t *levels) {
    ask_status s = ask_validate(win, params);
    if (s != ASK_OK || !params || !levels)
        return ASK_EINVAL;
    *levels = level_count(win->W, win->H, params->g, params->r, params->B);
    return ASK_OK;
}

ask_status ask_create(ask_ctx **out, int device) {
    if (!out)
        return ASK_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return ASK_EDEVICE;
    }
    ask_ctx *ctx = new (std::nothrow) ask_ctx();
    if (!ctx)
        return ASK_ENOMEM;
    ctx->device = device;
    DeviceGuard guard(device);
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e == hipSuccess)
        e = hipMalloc((void **)&ctx->ctrl, kCtrlWords * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMalloc((void **)&ctx->stats, sizeof(DevStats));
    if (e == hipSuccess)
        e = hipMemset(ctx->ctrl, 0, kCtrlWords * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipEventCreate(&ctx->ev[0]);
    if (e == hipSuccess)
        e = hipEventCreate(&ctx->ev[1]);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming);
    if (e == hipSuccess)
        e = occupancy_level(&ctx->occ_level);
    if (e == hipSuccess)
        e = occupancy_persistent(&ctx->occ_persistent);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ask_destroy(ctx);
        return ASK_EDEVICE;
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess &&
        khz > 0)
        ctx->clock_hz = 1e3 * khz;
    (void)hipGetLastError();
    ctx->cus = prop.multiProcessorCount;
    ctx->occ_level = std::max(1, ctx->occ_level);
    ctx->occ_persistent = std::max(1, ctx->occ_persistent);
    *out = ctx;
    return ASK_OK;
}

ask_status ask_destroy(ask_ctx *ctx) {
    if (!ctx)
        return ASK_OK;
    {
        DeviceGuard guard(ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->ctrl);
        (void)hipFree(ctx->stats);
        (void)hipFree(ctx->lvq[0]);
        (void)hipFree(ctx->lvq[1]);
        (void)hipFree(ctx->queue);
        if (ctx->ev[0])
            (void)hipEventDestroy(ctx->ev[0]);
        if (ctx->ev[1])
            (void)hipEventDestroy(ctx->ev[1]);
        if (ctx->staged)
            (void)hipEventDestroy(ctx->staged);
        (void)hipFree(ctx->table);
        (void)hipHostFree(ctx->staging);
    }
    delete ctx;
    return ASK_OK;
}

ask_status ask_dwell_exhaustive(ask_ctx *ctx, const ask_window *win, uint32_t *d_out,
                                void *stream) {
    if (!ctx)
        return ASK_EINVAL;
    if (check_window(win) != ASK_OK || !d_out)
        return fail(ctx, ASK_EINVAL, "invalid window or output%s", nullptr);
    DeviceGuard guard(ctx->device);
    const Image im = make_image(win, nullptr, d_out);
    hipError_t e = mark(ctx, 0, (hipStream_t)stream);
    if (e == hipSuccess)
        e = launch_exhaustive(im, (hipStream_t)stream);
    if (e == hipSuccess)
        e = mark(ctx, 1, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "exhaustive kernel launch");
    return ASK_OK;
}

}  // extern "C"

namespace {

// Render n images (n >= 1) that share one form in one sequence of launches:
// counters reset, level-0 seeding of every image, then the level kernels or
// the persistent kernel over one queue. `ims` holds each image's constants.
ask_status render(ask_ctx *ctx, const Image *ims, uint32_t n, uint32_t form, hipStream_t s,
                  ask_stats *stats) {
    uint32_t levels = 0;
    uint64_t nseeds = 0, bands = 0;
    std::vector<uint64_t> bound(kMaxLevels, 0);
    for (uint32_t i = 0; i < n; ++i) {
        const Image &im = ims[i];
        const uint32_t lv_i = level_count(im.W, im.H, im.g, im.r, im.B);
        if (lv_i > (uint32_t)kMaxLevels - 1)
            return fail(ctx, ASK_EINVAL, "too many levels%s", nullptr);
        levels = std::max(levels, lv_i);
        const uint64_t pixels = (uint64_t)im.W * im.H;
        for (uint32_t lv = 0; lv < lv_i; ++lv)
            bound[lv] += level_bound(pixels, im.g, im.r, lv);
        // Leaf bands of the persistent form: every band but a leaf's last
        // holds at least kLeafTask / 2 pixels.
        bands += pixels / (kLeafTask / 2);
        nseeds += (uint64_t)im.g * im.g;
    }
    if (nseeds > 0x7fffffffull)
        return fail(ctx, ASK_EINVAL, "too many level-0 regions%s", nullptr);
    uint64_t widest = 0, total = bands;
    for (uint32_t lv = 0; lv < levels; ++lv) {
        widest = std::max(widest, bound[lv]);
        total += 2 * bound[lv];  // the regions, and at most one last band each
    }
    const uint64_t need = form == ASK_FORM_PERSISTENT ? total : widest;
    const uint64_t want = std::min<uint64_t>(need, kQueueBudget);
    const bool may_overflow = need > want;
    ask_status st;
    if (form == ASK_FORM_PERSISTENT) {
        st = grow(ctx, &ctx->queue, &ctx->queue_cap, want, true);
    } else {
        size_t cap0 = ctx->lvq_cap;
        st = grow(ctx, &ctx->lvq[0], &cap0, want, false);
        if (st == ASK_OK) {
            size_t cap1 = ctx->lvq_cap;
            st = grow(ctx, &ctx->lvq[1], &cap1, want, false);
            ctx->lvq_cap = std::min(cap0, cap1);
        }
    }
    if (st != ASK_OK)
        return st;

    SubdivArgs a{};
    a.nimg = n;
    a.ctrl = ctx->ctrl;
    a.stats = stats ? ctx->stats : nullptr;
    hipError_t e = hipSuccess;
    if (n == 1) {
        a.single = ims[0];
    } else {
        // Image table, then the n + 1 seed offsets, staged through pinned memory.
        const size_t tbytes = (size_t)n * sizeof(Image);
        const size_t bytes = tbytes + (size_t)(n + 1) * sizeof(uint32_t);
        if (ctx->staged) {
            e = hipEventSynchronize(ctx->staged);  // the previous upload has left staging
            if (e != hipSuccess)
                return hip_fail(ctx, e, "hipEventSynchronize");
        }
        if (ctx->staging_bytes < bytes) {
            (void)hipHostFree(ctx->staging);
            ctx->staging = nullptr;
            ctx->staging_bytes = 0;
            if (hipHostMalloc(&ctx->staging, bytes, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return fail(ctx, ASK_ENOMEM, "cannot allocate pinned staging memory%s", nullptr);
            }
            ctx->staging_bytes = bytes;
        }
        if (ctx->table_bytes < bytes) {
            e = hipStreamSynchronize(s);
            if (e == hipSuccess) {
                (void)hipFree(ctx->table);
                ctx->table = nullptr;
                ctx->table_bytes = 0;
                e = hipMalloc(&ctx->table, bytes);
            }
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(ctx, ASK_ENOMEM, "cannot allocate the image table%s", nullptr);
            }
            ctx->table_bytes = bytes;
        }
        memcpy(ctx->staging, ims, tbytes);
        uint32_t *base = reinterpret_cast<uint32_t *>(static_cast<char *>(ctx->staging) + tbytes);
        base[0] = 0;
        for (uint32_t i = 0; i < n; ++i)
            base[i + 1] = base[i] + ims[i].g * ims[i].g;
        e = hipMemcpyAsync(ctx->table, ctx->staging, bytes, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipEventRecord(ctx->staged, s);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "image table upload");
        a.table = static_cast<const Image *>(ctx->table);
        a.seed_base = reinterpret_cast<const uint32_t *>(static_cast<const char *>(ctx->table) + tbytes);
    }
    e = launch_reset(ctx->ctrl, a.stats, s);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "reset kernel launch");

    if (form == ASK_FORM_PERSISTENT) {
        ctx->epoch = (ctx->epoch + 1) & 0xffffffu;
        if (ctx->epoch == 0) {  // tags wrapped: clear the queue once
            e = hipMemsetAsync(ctx->queue, 0, ctx->queue_cap * sizeof(Region), s);
            if (e != hipSuccess)
                return hip_fail(ctx, e, "hipMemsetAsync");
            ctx->epoch = 1;
        }
        a.queue = ctx->queue;
        a.cap = (uint32_t)std::min<size_t>(ctx->queue_cap, 0xffffffffu - 65536u);
        a.epoch = ctx->epoch;
        a.wait_ticks = (uint64_t)(ctx->wait_limit_s * ctx->clock_hz);
        e = launch_seed_queue(a, (uint32_t)nseeds, s);
        if (e == hipSuccess)
            e = mark(ctx, 0, s);
        if (e == hipSuccess)
            e = launch_persistent(a, (uint32_t)(ctx->cus * ctx->occ_persistent), s);
        if (e == hipSuccess)
            e = mark(ctx, 1, s);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "persistent launch");
    } else {
        a.cap = (uint32_t)std::min<size_t>(ctx->lvq_cap, 0xffffffffu - 65536u);
        a.epoch = 0;
        a.out = ctx->lvq[0];
        e = launch_seed_levels(a, (uint32_t)nseeds, s);
        if (e == hipSuccess)
            e = mark(ctx, 0, s);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "seed kernel launch");
        const uint32_t resident = (uint32_t)(ctx->cus * ctx->occ_level);
        for (uint32_t lv = 0; lv < levels; ++lv) {
            a.level = lv;
            a.in = ctx->lvq[lv & 1];
            a.out = ctx->lvq[(lv + 1) & 1];
            if (form == ASK_FORM_LEVELS_READBACK) {
                uint32_t cnt = 0;
                e = hipMemcpyAsync(&cnt, ctx->ctrl + kCount + lv, sizeof(cnt), hipMemcpyDeviceToHost,
                                   s);
                if (e == hipSuccess)
                    e = hipStreamSynchronize(s);
                if (e != hipSuccess)
                    return hip_fail(ctx, e, "level count readback");
                cnt = std::min<uint32_t>(cnt, a.cap);
                if (cnt == 0)
                    break;
                e = launch_level_exact(a, cnt, s);
            } else {
                const uint64_t blocks =
                    std::min<uint64_t>(resident, (bound[lv] + kWavesPerBlock - 1) / kWavesPerBlock);
                e = launch_level(a, (uint32_t)std::max<uint64_t>(1, blocks), s);
            }
            if (e != hipSuccess)
                return hip_fail(ctx, e, "level kernel launch");
        }
        e = mark(ctx, 1, s);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "hipEventRecord");
    }
    if (stats || may_overflow)
        return read_stats(ctx, s, stats);
    return ASK_OK;
}

}  // namespace

extern "C" {

ask_status ask_dwell_subdiv(ask_ctx *ctx, const ask_window *win, const ask_params *params,
                            uint32_t *d_out, void *stream, ask_stats *stats) {
    if (!ctx)
        return ASK_EINVAL;
    if (ask_validate(win, params) != ASK_OK || !params || !d_out)
        return fail(ctx, ASK_EINVAL, "invalid window, parameters or output%s", nullptr);
    DeviceGuard guard(ctx->device);
    const Image im = make_image(win, params, d_out);
    return render(ctx, &im, 1, params->form, (hipStream_t)stream, stats);
}

ask_status ask_dwell_batch(ask_ctx *ctx, uint32_t n, const ask_window *wins,
                           const ask_params *params, uint32_t nparams, uint32_t *const *d_outs,
                           void *stream, ask_stats *stats) {
    if (!ctx)
        return ASK_EINVAL;
    if (n == 0 || !wins || !params || !d_outs || (nparams != 1 && nparams != n))
        return fail(ctx, ASK_EINVAL, "invalid batch arguments%s", nullptr);
    const uint32_t form = params[0].form;
    std::vector<Image> ims(n);
    for (uint32_t i = 0; i < n; ++i) {
        const ask_params *p = &params[nparams == 1 ? 0 : i];
        if (ask_validate(&wins[i], p) != ASK_OK || !d_outs[i] || p->form != form)
            return fail(ctx, ASK_EINVAL, "invalid window, parameters or output in the batch%s",
                        nullptr);
        ims[i] = make_image(&wins[i], p, d_outs[i]);
    }
    DeviceGuard guard(ctx->device);
    return render(ctx, ims.data(), n, form, (hipStream_t)stream, stats);
}

ask_status ask_enable_timing(ask_ctx *ctx, int on) {
    if (!ctx)
        return ASK_EINVAL;
    ctx->timing = on != 0;
    ctx->timed = false;
    return ASK_OK;
}

ask_status ask_last_kernel_ms(ask_ctx *ctx, float *ms) {
    if (!ctx || !ms)
        return ASK_EINVAL;
    if (!ctx->timed)
        return fail(ctx, ASK_EINVAL, "no timed render on this context%s", nullptr);
    DeviceGuard guard(ctx->device);
    hipError_t e = hipEventSynchronize(ctx->ev[1]);
    if (e == hipSuccess)
        e = hipEventElapsedTime(ms, ctx->ev[0], ctx->ev[1]);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "hipEventElapsedTime");
    return ASK_OK;
}

ask_status ask_set_wait_limit(ask_ctx *ctx, double seconds) {
    if (!ctx || !(seconds >= 0.0) || seconds > 3600.0)
        return ASK_EINVAL;
    ctx->wait_limit_s = seconds;
    return ASK_OK;
}

ask_status ask_synchronize(ask_ctx *ctx, void *stream) {
    if (!ctx)
        return ASK_EINVAL;
    DeviceGuard guard(ctx->device);
    return take_errors(ctx, (hipStream_t)stream);
}

}  // extern "C"
