// Host engine and C ABI (include/ask.h): argument checks, mapping constants,
// level count, queue memory, and the launch sequences of the exhaustive image
// and the three subdivision forms.
#include "ask.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ask_internal.hpp"

#include <mutex>

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
    // Start and end events of the last kTimingRing timed renders; render k
    // (counting from the last ask_enable_timing) uses pair k % kTimingRing.
    std::vector<hipEvent_t> ev;
    uint64_t timed_count = 0;
    // Batches: image table and level-0 seed offsets on the device.
    void *table = nullptr;
    size_t table_bytes = 0;
    // Completion of the last render or exhaustive image enqueued on this
    // context (any stream): buffers are reallocated only after it.
    hipEvent_t last = nullptr;
    bool last_set = false;
    // Once a render has been captured into a graph, the graph may replay it
    // at any later time: buffers it names are never freed before the
    // context, only retired.
    bool captured = false;
    std::vector<void *> retired;
    ask_server *server = nullptr;  // the context's server, if one runs
    char err[512] = {0};
};

namespace {

constexpr uint32_t kTimingRing = 256;

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
    if (w->D < 1 || w->D > 0x7fffffffu)
        return ASK_EINVAL;
    if (w->set != ASK_SET_MANDELBROT && w->set != ASK_SET_JULIA)
        return ASK_EINVAL;
    if (w->set == ASK_SET_JULIA && (!std::isfinite(w->cr) || !std::isfinite(w->ci)))
        return ASK_EINVAL;
    return ASK_OK;
}

// The wave tile: both 0 (defaults), or a power-of-two width of 4 to 64
// pixels whose tile holds exactly one wave's 64 lanes.
bool check_tile(const ask_params *p) {
    if (p->tile_w == 0 && p->tile_h == 0)
        return true;
    const uint32_t tw = p->tile_w;
    return tw >= 4 && tw <= 64 && (tw & (tw - 1)) == 0 && p->tile_h * tw == 64;
}

ask_status check_params(const ask_window *w, const ask_params *p) {
    if (!p)
        return ASK_EINVAL;
    if (!check_tile(p))
        return ASK_EINVAL;
    if (p->g < 1 || p->g > w->W || p->g > w->H)
        return ASK_EINVAL;
    if (p->r < 2 || p->r > 1024 || p->B < 1 || p->B > 65536)
        return ASK_EINVAL;
    if (p->band != 0 && p->band != ASK_BAND_NONE && (p->band < 64 || p->band > (1u << 24)))
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

// Worst-case queue memory of a set of images.
struct Bounds {
    std::vector<uint64_t> level = std::vector<uint64_t>(kMaxLevels, 0);  // regions per level
    uint64_t pixels = 0;
    uint32_t band = ASK_BAND_NONE;  // smallest leaf band of the images
    uint64_t regions() const {
        uint64_t t = 0;
        for (uint64_t v : level)
            t += v;
        return t;
    }
    // Queue entries when leaves are queued as bands of `band` pixels: the
    // regions, and the bands, of which every one but a leaf's last has at
    // least band / 2 pixels (none when no leaf is banded).
    uint64_t queue_entries() const {
        return (band == ASK_BAND_NONE ? 0 : pixels / (band / 2)) + 2 * regions();
    }
};

// Add one image's bounds to b; returns its level count.
uint32_t add_bounds(const Image &im, Bounds &b) {
    const uint32_t lv_i = level_count(im.W, im.H, im.g, im.r, im.B);
    const uint64_t pixels = (uint64_t)im.W * im.H;
    for (uint32_t lv = 0; lv < lv_i && lv < (uint32_t)kMaxLevels; ++lv)
        b.level[lv] += level_bound(pixels, im.g, im.r, lv);
    b.pixels += pixels;
    b.band = std::min(b.band, im.band);
    return lv_i;
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
    im.band = p && p->band ? p->band : kLeafTask;
    // Only a 65536 x 65536 leaf has more pixels than one 32-bit stream can
    // index: even without bands it is cut into bands of 2^24 pixels.
    if ((uint64_t)im.W * im.H > im.band && im.band > (1u << 24))
        im.band = 1u << 24;
    im.tile_w = p ? p->tile_w : 0;
    im.tile_h = p ? p->tile_h : 0;
    im.julia = w->set == ASK_SET_JULIA ? 1u : 0u;
    im.jr = im.julia ? w->cr : 0.0;
    im.ji = im.julia ? w->ci : 0.0;
    im.out = out;
    return im;
}

// Wait until the context's last enqueued render has finished.
hipError_t wait_last(ask_ctx *ctx) {
    return ctx->last_set ? hipEventSynchronize(ctx->last) : hipSuccess;
}

hipError_t note_last(ask_ctx *ctx, hipStream_t s) {
    hipError_t e = hipEventRecord(ctx->last, s);
    ctx->last_set = e == hipSuccess;
    return e;
}

template <class T>
ask_status grow(ask_ctx *ctx, T **buf, size_t *cap, size_t need, bool clear) {
    if (*cap >= need)
        return ASK_OK;
    const size_t n = std::max<size_t>(need, std::min<size_t>(*cap * 2, kQueueBudget));
    hipError_t e;
    if (*buf) {
        e = wait_last(ctx);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "hipEventSynchronize");
        if (ctx->captured)
            ctx->retired.push_back(*buf);
        else
            (void)hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
    }
    e = hipMalloc((void **)buf, n * sizeof(T));
    if (e != hipSuccess) {
        *buf = nullptr;
        (void)hipGetLastError();
        return fail(ctx, ASK_ENOMEM, "cannot allocate the region queue or ring records%s", nullptr);
    }
    if (clear) {
        e = hipMemset(*buf, 0, n * sizeof(T));
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
        out->ring_px = ds.ring_px;
        out->leaf_px = ds.leaf_px;
        out->fill_px = ds.fill_px;
    }
    return st;
}

hipError_t mark(ask_ctx *ctx, int which, hipStream_t s) {
    if (!ctx->timing)
        return hipSuccess;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
        return hipSuccess;  // a graph is not timed by the context's events
    (void)hipGetLastError();
    const size_t slot = ctx->timed_count % kTimingRing;
    const hipError_t e = hipEventRecord(ctx->ev[2 * slot + which], s);
    if (which == 1 && e == hipSuccess) {
        ctx->timed = true;
        ++ctx->timed_count;
    }
    return e;
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

ask_status ask_create(ask_ctx **out, int device, size_t queue_bytes) {
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
        e = hipEventCreateWithFlags(&ctx->last, hipEventDisableTiming);
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
    if (queue_bytes) {
        const size_t entries = std::max<size_t>(1, queue_bytes / sizeof(Region));
        size_t cap0 = 0, cap1 = 0;
        ask_status st = grow(ctx, &ctx->queue, &ctx->queue_cap, entries, true);
        if (st == ASK_OK)
            st = grow(ctx, &ctx->lvq[0], &cap0, entries, false);
        if (st == ASK_OK)
            st = grow(ctx, &ctx->lvq[1], &cap1, entries, false);
        ctx->lvq_cap = std::min(cap0, cap1);
        if (st != ASK_OK) {
            ask_destroy(ctx);
            return st;
        }
    }
    *out = ctx;
    return ASK_OK;
}

ask_status ask_destroy(ask_ctx *ctx) {
    if (!ctx)
        return ASK_OK;
    if (ctx->server)
        (void)ask_server_destroy(ctx->server);
    {
        DeviceGuard guard(ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->ctrl);
        (void)hipFree(ctx->stats);
        (void)hipFree(ctx->lvq[0]);
        (void)hipFree(ctx->lvq[1]);
        (void)hipFree(ctx->queue);
        for (hipEvent_t ev : ctx->ev)
            (void)hipEventDestroy(ev);
        if (ctx->last)
            (void)hipEventDestroy(ctx->last);
        for (void *p : ctx->retired)
            (void)hipFree(p);
        (void)hipFree(ctx->table);
    }
    delete ctx;
    return ASK_OK;
}

ask_status ask_dwell_exhaustive(ask_ctx *ctx, const ask_window *win, const ask_params *params,
                                uint32_t *d_out, void *stream) {
    if (!ctx)
        return ASK_EINVAL;
    if (check_window(win) != ASK_OK || !d_out || (params && !check_tile(params)))
        return fail(ctx, ASK_EINVAL, "invalid window, wave tile or output%s", nullptr);
    DeviceGuard guard(ctx->device);
    Image im = make_image(win, nullptr, d_out);
    im.tile_w = params ? params->tile_w : 0;
    im.tile_h = params ? params->tile_h : 0;
    hipError_t e = mark(ctx, 0, (hipStream_t)stream);
    if (e == hipSuccess)
        e = launch_exhaustive(im, (hipStream_t)stream);
    if (e == hipSuccess)
        e = mark(ctx, 1, (hipStream_t)stream);
    if (e == hipSuccess)
        e = note_last(ctx, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "exhaustive kernel launch");
    return ASK_OK;
}

}  // extern "C"

namespace {

// What a render of n images in one form needs, worked out on the host from
// the images alone: level count, level-0 seeds and worst-case queue sizes.
struct Plan {
    uint32_t levels = 0;
    uint64_t nseeds = 0;
    Bounds b;
    bool banded = false;      // some image cuts leaves into bands
    uint64_t band_bound = 0;  // per-level form: bands one level's table may hold
    uint64_t need = 0;        // entries: the persistent queue, or each per-level table
};

ask_status plan_render(ask_ctx *ctx, const Image *ims, uint32_t n, uint32_t form, Plan &p) {
    for (uint32_t i = 0; i < n; ++i) {
        const Image &im = ims[i];
        const uint32_t lv_i = add_bounds(im, p.b);
        if (lv_i > (uint32_t)kMaxLevels - 1)
            return fail(ctx, ASK_EINVAL, "too many levels%s", nullptr);
        p.levels = std::max(p.levels, lv_i);
        p.nseeds += (uint64_t)im.g * im.g;
    }
    if (p.nseeds > 0x7fffffffull)
        return fail(ctx, ASK_EINVAL, "too many level-0 regions%s", nullptr);
    uint64_t widest = 0;
    for (uint32_t lv = 0; lv < p.levels; ++lv)
        widest = std::max(widest, p.b.level[lv]);
    // Per-level form: a level's table holds its regions and the bands of the
    // leaves decided one level up, at most pixels / (band / 2) plus one per
    // leaf; bands of last-level leaves take one more level kernel.
    p.banded = p.b.band != ASK_BAND_NONE;
    p.band_bound = p.banded ? p.b.pixels / (p.b.band / 2) + widest : 0;
    p.need = form == ASK_FORM_PERSISTENT ? p.b.queue_entries() : widest + p.band_bound;
    return ASK_OK;
}

// Device memory a render runs in, and how it is launched.
struct Buffers {
    uint32_t *ctrl = nullptr;
    DevStats *stats = nullptr;            // nullptr: no counters
    Region *lvq[2] = {nullptr, nullptr};  // per-level tables
    Region *queue = nullptr;              // persistent queue
    uint64_t cap = 0;                     // entries of the queue, or of each table
    const Image *table = nullptr;         // device image table (n > 1), or nullptr
    const uint32_t *seed_base = nullptr;  // its n + 1 seed offsets
    uint32_t epoch = 1;                   // tag of this launch's queue entries
    bool clear_queue = false;             // clear the queue's first `cap` entries first
    uint64_t wait_ticks = 0;
    uint32_t grid_persistent = 1;         // workgroups of the persistent kernel
    uint32_t resident_level = 1;          // workgroups the per-level kernels keep resident
};

// Write `words` (n 32-bit words) to device memory at dst with kernels that
// carry the data in their arguments: a stream capture records them as
// kernel nodes, so a graph replays the data itself and depends on no host
// buffer.
hipError_t upload_words(uint32_t *dst, const uint32_t *words, size_t n, hipStream_t s) {
    for (size_t off = 0; off < n; off += kWordsPerWrite) {
        WordsArg w{};
        w.dst = dst + off;
        w.n = (uint32_t)std::min<size_t>(kWordsPerWrite, n - off);
        memcpy(w.words, words + off, w.n * sizeof(uint32_t));
        const hipError_t e = launch_write_words(w, s);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// The longest ring of level lv over the images: regions of the floor
// partition into g r^lv parts per axis are at most ceil(W / (g r^lv)) wide.
uint32_t largest_ring(const Image *ims, uint32_t n, uint32_t lv) {
    uint64_t best = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t parts = ims[i].g;
        for (uint32_t k = 0; k < lv && parts < (1ull << 32); ++k)
            parts *= ims[i].r;
        const uint64_t w = (ims[i].W + parts - 1) / parts, h = (ims[i].H + parts - 1) / parts;
        const uint64_t ring = (w <= 1 || h <= 1) ? w * h : 2 * (w + h) - 4;
        best = std::max(best, ring);
    }
    return (uint32_t)std::min<uint64_t>(best, 0xffffffffu);
}

// The launch sequence of a render: counters reset, level-0 seeding of every
// image, then the persistent kernel over one queue or one kernel per level.
// ctx (may be nullptr) records the timing events and read-back errors.
ask_status launch_render(ask_ctx *ctx, const Plan &p, const Buffers &bf, const Image *ims,
                         uint32_t n, uint32_t form, hipStream_t s) {
    SubdivArgs a{};
    a.nimg = n;
    a.ctrl = bf.ctrl;
    a.stats = bf.stats;
    if (n == 1)
        a.single = ims[0];
    a.table = n == 1 ? nullptr : bf.table;
    a.seed_base = bf.seed_base;
    const uint32_t cap = (uint32_t)std::min<uint64_t>(bf.cap, 0xffffffffu - 65536u);
    hipError_t e = launch_reset(bf.ctrl, bf.stats, s);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "reset kernel launch");
    if (form == ASK_FORM_PERSISTENT) {
        if (bf.clear_queue) {
            e = launch_clear_queue(bf.queue, cap, s);
            if (e != hipSuccess)
                return hip_fail(ctx, e, "queue clear launch");
        }
        a.queue = bf.queue;
        a.cap = cap;
        a.epoch = bf.epoch;
        a.wait_ticks = bf.wait_ticks;
        e = launch_seed_queue(a, (uint32_t)p.nseeds, s);
        if (e == hipSuccess && ctx)
            e = mark(ctx, 0, s);
        if (e == hipSuccess)
            e = launch_persistent(a, bf.grid_persistent, s);
        if (e == hipSuccess && ctx)
            e = mark(ctx, 1, s);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "persistent launch");
        return ASK_OK;
    }
    a.cap = cap;
    a.epoch = 0;
    a.out = bf.lvq[0];
    e = launch_seed_levels(a, (uint32_t)p.nseeds, s);
    if (e == hipSuccess && ctx)
        e = mark(ctx, 0, s);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "seed kernel launch");
    for (uint32_t lv = 0; lv < p.levels + (p.banded ? 1u : 0u); ++lv) {
        a.level = lv;
        a.in = bf.lvq[lv & 1];
        a.out = bf.lvq[(lv + 1) & 1];
        if (form == ASK_FORM_LEVELS_READBACK) {
            uint32_t cnt = 0;
            e = hipMemcpyAsync(&cnt, bf.ctrl + kCount + lv, sizeof(cnt), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipStreamSynchronize(s);
            if (e != hipSuccess)
                return hip_fail(ctx, e, "level count readback");
            cnt = std::min<uint32_t>(cnt, a.cap);
            if (cnt == 0)
                break;
            e = launch_level_exact(a, cnt, s);
        } else {
            const uint64_t entries = p.b.level[lv] + (lv > 0 ? p.band_bound : 0);
            if (largest_ring(ims, n, lv) >= kCoopRingPixels) {
                const uint64_t blocks = std::min<uint64_t>(bf.resident_level, entries);
                e = launch_level_coop(a, (uint32_t)std::max<uint64_t>(1, blocks), s);
            } else {
                const uint64_t blocks = std::min<uint64_t>(
                    bf.resident_level, (entries + kWavesPerBlock - 1) / kWavesPerBlock);
                e = launch_level(a, (uint32_t)std::max<uint64_t>(1, blocks), s);
            }
        }
        if (e != hipSuccess)
            return hip_fail(ctx, e, "level kernel launch");
    }
    if (ctx) {
        e = mark(ctx, 1, s);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "hipEventRecord");
    }
    return ASK_OK;
}

// Render n images (n >= 1) that share one form on a context: plan, make
// room in the context's queues and image table, then launch.
ask_status render(ask_ctx *ctx, const Image *ims, uint32_t n, uint32_t form, hipStream_t s,
                  ask_stats *stats) {
    // Under stream capture the render becomes a graph that may replay many
    // times: nothing may wait, nothing a later call could change may be
    // named, and the persistent queue is cleared by a kernel of the graph
    // (its slots then carry a launch epoch reserved for graphs).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) {
        (void)hipGetLastError();
        cap = hipStreamCaptureStatusNone;
    }
    const bool capturing = cap != hipStreamCaptureStatusNone;
    if (capturing && (stats || form == ASK_FORM_LEVELS_READBACK))
        return fail(ctx, ASK_EINVAL,
                    "a captured render takes no work counters and not the read-back form%s",
                    nullptr);
    Plan p;
    ask_status st = plan_render(ctx, ims, n, form, p);
    if (st != ASK_OK)
        return st;
    const uint64_t want = std::min<uint64_t>(p.need, kQueueBudget);
    const bool may_overflow = p.need > want;
    if (capturing && (may_overflow || (form == ASK_FORM_PERSISTENT ? ctx->queue_cap < want
                                                                   : ctx->lvq_cap < want)))
        return fail(ctx, ASK_EINVAL,
                    "render once outside the capture first (the queues must not grow "
                    "while capturing)%s", nullptr);
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

    Buffers bf;
    bf.ctrl = ctx->ctrl;
    bf.stats = stats ? ctx->stats : nullptr;
    bf.lvq[0] = ctx->lvq[0];
    bf.lvq[1] = ctx->lvq[1];
    bf.queue = ctx->queue;
    bf.cap = form == ASK_FORM_PERSISTENT ? ctx->queue_cap : ctx->lvq_cap;
    bf.wait_ticks = (uint64_t)(ctx->wait_limit_s * ctx->clock_hz);
    bf.grid_persistent = (uint32_t)(ctx->cus * ctx->occ_persistent);
    bf.resident_level = (uint32_t)(ctx->cus * ctx->occ_level);
    hipError_t e = hipSuccess;
    if (n > 1) {
        // The image table and the n + 1 level-0 seed offsets, written by
        // kernels that carry them as arguments. A captured batch gets a
        // table of its own, which no later call writes and the context never
        // frees before it ends; other batches share the context's table.
        std::vector<uint32_t> words((n * sizeof(Image) + (n + 1) * sizeof(uint32_t) + 3) / 4);
        const size_t tbytes = (size_t)n * sizeof(Image);
        memcpy(words.data(), ims, tbytes);
        uint32_t *base = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(words.data()) + tbytes);
        base[0] = 0;
        for (uint32_t i = 0; i < n; ++i)
            base[i + 1] = base[i] + ims[i].g * ims[i].g;
        const size_t bytes = words.size() * sizeof(uint32_t);
        void *table = nullptr;
        if (capturing) {
            // An allocation is not a stream operation: the capture may go on
            // around it, which the thread's relaxed capture mode permits.
            hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
            e = hipThreadExchangeStreamCaptureMode(&mode);
            if (e == hipSuccess) {
                e = hipMalloc(&table, bytes);
                hipStreamCaptureMode back = mode;
                const hipError_t e2 = hipThreadExchangeStreamCaptureMode(&back);
                if (e == hipSuccess)
                    e = e2;
            }
            if (table)
                ctx->retired.push_back(table);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(ctx, ASK_ENOMEM, "cannot allocate the image table%s", nullptr);
            }
        } else {
            if (ctx->table_bytes < bytes) {
                e = wait_last(ctx);
                if (e == hipSuccess) {
                    if (ctx->captured)
                        ctx->retired.push_back(ctx->table);
                    else
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
            table = ctx->table;
        }
        e = upload_words(static_cast<uint32_t *>(table), words.data(), words.size(), s);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "image table upload");
        bf.table = static_cast<const Image *>(table);
        bf.seed_base = reinterpret_cast<const uint32_t *>(static_cast<const char *>(table) + tbytes);
    }
    if (form == ASK_FORM_PERSISTENT) {
        if (capturing) {
            bf.clear_queue = true;
            bf.epoch = kGraphEpoch;
        } else {
            ctx->epoch = (ctx->epoch + 1) & 0xffffffu;
            if (ctx->epoch == 0 || ctx->epoch == kGraphEpoch) {  // wrapped: clear the queue once
                bf.clear_queue = true;
                ctx->epoch = 1;
            }
            bf.epoch = ctx->epoch;
        }
    }
    if (capturing)
        ctx->captured = true;
    st = launch_render(ctx, p, bf, ims, n, form, s);
    if (st != ASK_OK || capturing)
        return st;
    e = note_last(ctx, s);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "hipEventRecord");
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
    if (on && ctx->ev.empty()) {
        DeviceGuard guard(ctx->device);
        ctx->ev.assign(2 * kTimingRing, nullptr);
        for (hipEvent_t &ev : ctx->ev) {
            const hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) {
                for (hipEvent_t &x : ctx->ev)
                    if (x)
                        (void)hipEventDestroy(x);
                ctx->ev.clear();
                return hip_fail(ctx, e, "hipEventCreate");
            }
        }
    }
    if (on && ctx->timing) {  // events of renders still in flight are reused last
        DeviceGuard guard(ctx->device);
        const hipError_t e = wait_last(ctx);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "hipEventSynchronize");
    }
    ctx->timing = on != 0;
    ctx->timed = false;
    ctx->timed_count = 0;
    return ASK_OK;
}

// Device time of timed render k (0 = the first since timing was enabled).
static ask_status kernel_ms(ask_ctx *ctx, uint64_t k, float *ms) {
    const size_t slot = k % kTimingRing;
    hipError_t e = hipEventSynchronize(ctx->ev[2 * slot + 1]);
    if (e == hipSuccess)
        e = hipEventElapsedTime(ms, ctx->ev[2 * slot], ctx->ev[2 * slot + 1]);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "hipEventElapsedTime");
    return ASK_OK;
}

ask_status ask_last_kernel_ms(ask_ctx *ctx, float *ms) {
    if (!ctx || !ms)
        return ASK_EINVAL;
    if (!ctx->timed)
        return fail(ctx, ASK_EINVAL, "no timed render on this context%s", nullptr);
    DeviceGuard guard(ctx->device);
    return kernel_ms(ctx, ctx->timed_count - 1, ms);
}

ask_status ask_kernel_times(ask_ctx *ctx, float *ms, uint32_t cap, uint32_t *n) {
    if (!ctx || !n || (cap && !ms))
        return ASK_EINVAL;
    DeviceGuard guard(ctx->device);
    const uint64_t have = std::min<uint64_t>(ctx->timed_count, kTimingRing);
    const uint64_t take = std::min<uint64_t>(have, cap);
    *n = 0;
    for (uint64_t i = 0; i < take; ++i) {
        const ask_status st = kernel_ms(ctx, ctx->timed_count - take + i, &ms[i]);
        if (st != ASK_OK)
            return st;
        ++*n;
    }
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

// ---------------------------------------------------------------------------
// Serving (include/ask.h): slots, pool memory and the server kernel's life.
// ---------------------------------------------------------------------------
namespace {

// First-fit allocator over [0, size) of a pool, coalescing on release.
class PoolAlloc {
  public:
    void reset(uint64_t size) {
        free_.clear();
        if (size)
            free_[0] = size;
    }
    bool alloc(uint64_t n, uint64_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n)
                continue;
            *off = it->first;
            const uint64_t at = it->first + n, rest = it->second - n;
            free_.erase(it);
            if (rest)
                free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        if (!n)
            return;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<uint64_t, uint64_t> free_;
};

constexpr uint32_t kMaxGen = (1u << 24) - 1;  // request generations are 24-bit tags
constexpr size_t kLatencyKept = 1u << 16;     // latencies of this many recent requests are kept
constexpr uint64_t kDefaultPool = 256ull << 20;

}  // namespace

struct ask_server {
    ask_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    uint32_t nslots = 0;
    uint32_t blocks = 0;
    ServerSlot *slots = nullptr;
    ServerCtl *ctl = nullptr;
    Region *queue = nullptr;
    uint64_t queue_entries = 0;
    ServerMailbox *mb = nullptr;      // host address of the pinned mailbox
    ServerMailbox *mb_dev = nullptr;  // its device address
    PoolAlloc qpool;
    struct Flight {
        bool busy = false;
        bool quarantined = false;  // finished with an error: slot and memory never reused
        uint64_t ticket = 0;
        uint32_t gen = 0;
        uint64_t qoff = 0, qlen = 0;
        std::chrono::steady_clock::time_point submitted;
    } flight[kMaxSlots];
    // Latency (s) of the most recent finished requests, by ticket.
    std::map<uint64_t, double> latency;
    uint32_t next_gen = 1;
    uint64_t next_ticket = 1;
    uint32_t in_flight = 0;
    bool running = false;
    std::deque<std::pair<uint64_t, int32_t>> finished;  // reaped, not yet handed out
    std::unordered_map<uint64_t, int32_t> failed;
};

namespace {

hipError_t server_launch(ask_server *sv) {
    ask_ctx *ctx = sv->ctx;
    // No server kernel runs now: reset the device words and slots, and ring
    // again only the doorbells of requests posted and not finished.
    hipError_t e = hipMemsetAsync(sv->ctl, 0, sizeof(ServerCtl), sv->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(sv->slots, 0, sizeof(ServerSlot) * sv->nslots, sv->stream);
    if (e != hipSuccess)
        return e;
    __atomic_store_n(&sv->mb->stop, 0u, __ATOMIC_RELAXED);
    for (uint32_t k = 0; k < kMaxSlots; ++k)
        if (!sv->flight[k].busy)
            __atomic_store_n(&sv->mb->doorbell[k], 0u, __ATOMIC_RELAXED);
    __atomic_thread_fence(__ATOMIC_SEQ_CST);
    ServerArgs a{};
    a.slots = sv->slots;
    a.ctl = sv->ctl;
    a.nslots = sv->nslots;
    a.queue = sv->queue;
    a.mb = sv->mb_dev;
    a.wait_ticks = (uint64_t)(ctx->wait_limit_s * ctx->clock_hz);
    a.poll_ticks = std::max<uint64_t>(1, (uint64_t)(2e-6 * ctx->clock_hz));
    a.idle_ticks = (uint64_t)(std::max(1.0, ctx->wait_limit_s) * ctx->clock_hz);
    e = launch_server(a, sv->blocks, sv->stream);
    sv->running = e == hipSuccess;
    return e;
}

// Move requests whose completion the device has reported to `finished`,
// returning their pool memory (unless they failed).
void server_reap(ask_server *sv) {
    for (uint32_t k = 0; k < sv->nslots; ++k) {
        ask_server::Flight &f = sv->flight[k];
        if (!f.busy || __atomic_load_n(&sv->mb->done[k].gen, __ATOMIC_ACQUIRE) != f.gen)
            continue;
        const int32_t status = __atomic_load_n(&sv->mb->done[k].status, __ATOMIC_RELAXED);
        sv->latency[f.ticket] =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - f.submitted).count();
        if (sv->latency.size() > kLatencyKept)
            sv->latency.erase(sv->latency.begin());
        f.busy = false;
        --sv->in_flight;
        if (status == ASK_OK) {
            sv->qpool.release(f.qoff, f.qlen);
        } else {
            f.quarantined = true;
            sv->failed[f.ticket] = status;
        }
        sv->finished.emplace_back(f.ticket, status);
    }
}

// Relaunch the server kernel if it has left (it leaves after a long idle
// time); requests posted meanwhile are then admitted by the new launch.
ask_status server_ensure_running(ask_server *sv) {
    if (sv->running) {
        const hipError_t q = hipStreamQuery(sv->stream);
        if (q == hipErrorNotReady)
            return ASK_OK;
        if (q != hipSuccess)
            return hip_fail(sv->ctx, q, "server kernel");
        sv->running = false;
        server_reap(sv);
    }
    const hipError_t e = server_launch(sv);
    return e == hipSuccess ? ASK_OK : hip_fail(sv->ctx, e, "server kernel launch");
}

// Stop the kernel once it has no admitted request and wait for it to leave.
hipError_t server_stop(ask_server *sv) {
    __atomic_store_n(&sv->mb->stop, 1u, __ATOMIC_RELEASE);
    hipError_t e = hipStreamSynchronize(sv->stream);
    sv->running = false;
    return e;
}

}  // namespace

extern "C" {

ask_status ask_server_create(ask_ctx *ctx, const ask_server_cfg *cfg, ask_server **out) {
    if (!out)
        return ASK_EINVAL;
    *out = nullptr;
    if (!ctx || !cfg || cfg->slots < 1 || cfg->slots > kMaxSlots || cfg->waves_per_cu % 4 != 0)
        return fail(ctx, ASK_EINVAL, "invalid server configuration%s", nullptr);
    if (ctx->server)
        return fail(ctx, ASK_EBUSY, "this context already has a server%s", nullptr);
    const uint64_t pool = cfg->pool_bytes ? cfg->pool_bytes : kDefaultPool;
    if (pool < (1ull << 20))
        return fail(ctx, ASK_EINVAL, "server pool below 1 MiB%s", nullptr);
    DeviceGuard guard(ctx->device);
    int occ = 1;
    if (occupancy_server(&occ) != hipSuccess || occ < 1) {
        (void)hipGetLastError();
        occ = 1;
    }
    const uint32_t per_cu = cfg->waves_per_cu ? cfg->waves_per_cu / 4 : (uint32_t)std::max(1, occ - 1);
    if (per_cu > (uint32_t)occ)
        return fail(ctx, ASK_EINVAL, "waves_per_cu above the server kernel's occupancy%s", nullptr);
    ask_server *sv = new (std::nothrow) ask_server();
    if (!sv)
        return ASK_ENOMEM;
    sv->ctx = ctx;
    sv->nslots = cfg->slots;
    sv->blocks = (uint32_t)ctx->cus * per_cu;
    sv->queue_entries = std::min<uint64_t>(pool / sizeof(Region), 0xffffffffull);
    hipError_t e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipMalloc((void **)&sv->slots, sizeof(ServerSlot) * sv->nslots);
    if (e == hipSuccess)
        e = hipMalloc((void **)&sv->ctl, sizeof(ServerCtl));
    if (e == hipSuccess)
        e = hipMalloc((void **)&sv->queue, sizeof(Region) * sv->queue_entries);
    if (e == hipSuccess)
        e = hipMemset(sv->queue, 0, sizeof(Region) * sv->queue_entries);  // no entry carries a generation
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&sv->mb, sizeof(ServerMailbox), hipHostMallocCoherent);
    if (e == hipSuccess)
        e = hipHostGetDevicePointer((void **)&sv->mb_dev, sv->mb, 0);
    if (e == hipSuccess) {
        memset(sv->mb, 0, sizeof(ServerMailbox));
        sv->qpool.reset(sv->queue_entries);
        e = server_launch(sv);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        const ask_status st = hip_fail(ctx, e, "server set-up");
        (void)hipStreamSynchronize(sv->stream);
        (void)hipFree(sv->slots);
        (void)hipFree(sv->ctl);
        (void)hipFree(sv->queue);
            (void)hipHostFree(sv->mb);
        if (sv->stream)
            (void)hipStreamDestroy(sv->stream);
        delete sv;
        return e == hipErrorOutOfMemory ? ASK_ENOMEM : st;
    }
    ctx->server = sv;
    *out = sv;
    return ASK_OK;
}

ask_status ask_server_submit(ask_server *sv, const ask_window *win, const ask_params *params,
                             uint32_t *d_out, uint64_t *ticket) {
    if (!sv || !ticket)
        return ASK_EINVAL;
    ask_ctx *ctx = sv->ctx;
    if (check_window(win) != ASK_OK || check_params(win, params) != ASK_OK || !d_out)
        return fail(ctx, ASK_EINVAL, "invalid window, parameters or output%s", nullptr);
    const Image im = make_image(win, params, d_out);
    Bounds b;
    if (add_bounds(im, b) > (uint32_t)kMaxLevels - 1)
        return fail(ctx, ASK_EINVAL, "too many levels%s", nullptr);
    const uint64_t qlen = b.queue_entries();
    if (qlen > sv->queue_entries)
        return fail(ctx, ASK_ENOMEM, "the request's worst case exceeds the server pool%s", nullptr);
    DeviceGuard guard(ctx->device);
    server_reap(sv);
    if (sv->next_gen > kMaxGen) {
        // Generations would wrap: once idle, stop, clear the queue pool's
        // tags and start again from generation 1.
        if (sv->in_flight)
            return fail(ctx, ASK_EBUSY, "server restarting%s", nullptr);
        hipError_t e = server_stop(sv);
        if (e == hipSuccess)
            e = hipMemset(sv->queue, 0, sizeof(Region) * sv->queue_entries);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "server restart");
        for (uint32_t k = 0; k < kMaxSlots; ++k)
            sv->mb->done[k].gen = 0;
        sv->next_gen = 1;
    }
    ask_status st = server_ensure_running(sv);
    if (st != ASK_OK)
        return st;
    uint32_t k = 0;
    while (k < sv->nslots && (sv->flight[k].busy || sv->flight[k].quarantined))
        ++k;
    if (k == sv->nslots)
        return fail(ctx, ASK_EBUSY, "no free request slot%s", nullptr);
    uint64_t qoff = 0;
    if (!sv->qpool.alloc(qlen, &qoff))
        return fail(ctx, ASK_EBUSY, "not enough free queue memory%s", nullptr);
    const uint32_t gen = sv->next_gen++;
    ServerPost &p = sv->mb->post[k];
    p.im = im;
    p.qoff = (uint32_t)qoff;
    p.qcap = (uint32_t)qlen;
    __atomic_store_n(&sv->mb->doorbell[k], gen, __ATOMIC_RELEASE);
    ask_server::Flight &f = sv->flight[k];
    f.busy = true;
    f.ticket = sv->next_ticket++;
    f.gen = gen;
    f.qoff = qoff;
    f.qlen = qlen;
    f.submitted = std::chrono::steady_clock::now();
    ++sv->in_flight;
    *ticket = f.ticket;
    return ASK_OK;
}

ask_status ask_server_reap(ask_server *sv, uint64_t *tickets, int32_t *status, uint32_t cap,
                           uint32_t *n) {
    if (!sv || !n || (cap && !tickets))
        return ASK_EINVAL;
    DeviceGuard guard(sv->ctx->device);
    server_reap(sv);
    *n = 0;
    while (*n < cap && !sv->finished.empty()) {
        tickets[*n] = sv->finished.front().first;
        if (status)
            status[*n] = sv->finished.front().second;
        sv->finished.pop_front();
        ++*n;
    }
    if (sv->in_flight)
        return server_ensure_running(sv);
    return ASK_OK;
}

ask_status ask_server_poll(ask_server *sv, uint64_t ticket, int *done, double *latency_s) {
    if (!sv || !done || ticket == 0 || ticket >= sv->next_ticket)
        return ASK_EINVAL;
    DeviceGuard guard(sv->ctx->device);
    server_reap(sv);
    if (latency_s)
        *latency_s = -1.0;
    for (uint32_t k = 0; k < sv->nslots; ++k) {
        if (sv->flight[k].busy && sv->flight[k].ticket == ticket) {
            *done = 0;
            return server_ensure_running(sv);
        }
    }
    *done = 1;
    if (latency_s) {
        auto lt = sv->latency.find(ticket);
        if (lt != sv->latency.end())
            *latency_s = lt->second;
    }
    auto it = sv->failed.find(ticket);
    return it == sv->failed.end() ? ASK_OK : (ask_status)it->second;
}

ask_status ask_server_in_flight(const ask_server *sv, uint32_t *n) {
    if (!sv || !n)
        return ASK_EINVAL;
    *n = sv->in_flight;
    return ASK_OK;
}

ask_status ask_server_destroy(ask_server *sv) {
    if (!sv)
        return ASK_OK;
    ask_ctx *ctx = sv->ctx;
    DeviceGuard guard(ctx->device);
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration<double>(ctx->wait_limit_s + 5.0);
    while (sv->in_flight && std::chrono::steady_clock::now() < deadline) {
        server_reap(sv);
        if (sv->in_flight && server_ensure_running(sv) != ASK_OK)
            break;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    const bool late = sv->in_flight != 0;
    (void)server_stop(sv);
    (void)hipFree(sv->slots);
    (void)hipFree(sv->ctl);
    (void)hipFree(sv->queue);
    (void)hipHostFree(sv->mb);
    (void)hipStreamDestroy(sv->stream);
    ctx->server = nullptr;
    delete sv;
    return late ? fail(ctx, ASK_ETIMEOUT, "server requests did not finish in time%s", nullptr)
                : ASK_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free subdivision (include/ask.h, ask_dwell_subdiv_noalloc): the
// render's control words and region queue live in one file-scope device
// array instead of context memory.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = ASK_NOALLOC_SCRATCH_BYTES;
constexpr size_t kScratchQueueOffset = 4096;  // the control words come first
static_assert(kCtrlWords * sizeof(uint32_t) <= kScratchQueueOffset, "control words fit");

// Every device the library runs on holds its own copy of this array, at its
// own address, until the process ends. Host code never uses its name as an
// address: each device's address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;

struct ScratchDevice {
    std::once_flag once;
    hipError_t err = hipSuccess;
    unsigned char *ptr = nullptr;  // this device's address of `scratch`
    uint32_t grid_persistent = 1;
    uint32_t resident_level = 1;
    uint64_t wait_ticks = 0;
};

ScratchDevice g_scratch[kMaxDevices];

// Once per device, with that device current: the device address of the
// scratch array, and the launch sizes of the persistent and level kernels.
void scratch_setup(ScratchDevice &d) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    int dev = 0, cus = 0, occ_p = 1, occ_l = 1, khz = 0;
    if (e == hipSuccess)
        e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = occupancy_persistent(&occ_p);
    if (e == hipSuccess)
        e = occupancy_level(&occ_l);
    if (e == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        khz = 0;
    (void)hipGetLastError();
    d.err = e;
    if (e != hipSuccess || !p)
        return;
    d.ptr = static_cast<unsigned char *>(p);
    d.grid_persistent = (uint32_t)(std::max(1, cus) * std::max(1, occ_p));
    d.resident_level = (uint32_t)(std::max(1, cus) * std::max(1, occ_l));
    d.wait_ticks = (uint64_t)(10.0 * (khz > 0 ? 1e3 * khz : 1e8));  // 10 s
}

}  // namespace

extern "C" {

ask_status ask_dwell_subdiv_noalloc(const ask_window *win, const ask_params *params,
                                    uint32_t *d_out, void *stream) {
    if (ask_validate(win, params) != ASK_OK || !params || !d_out)
        return ASK_EINVAL;
    if (params->form != ASK_FORM_LEVELS && params->form != ASK_FORM_PERSISTENT)
        return ASK_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return ASK_EDEVICE;
    }
    ScratchDevice &d = g_scratch[dev];
    std::call_once(d.once, scratch_setup, std::ref(d));
    if (d.err != hipSuccess || !d.ptr)
        return ASK_EDEVICE;
    const Image im = make_image(win, params, d_out);
    Plan p;
    if (plan_render(nullptr, &im, 1, params->form, p) != ASK_OK)
        return ASK_EINVAL;
    // The worst case must fit: then no queue can overflow.
    const uint64_t room = (kScratchBytes - kScratchQueueOffset) / sizeof(Region);
    const uint64_t per_table = params->form == ASK_FORM_PERSISTENT ? room : room / 2;
    if (p.need > per_table)
        return ASK_EINVAL;
    Buffers bf;
    bf.ctrl = reinterpret_cast<uint32_t *>(d.ptr);
    Region *q = reinterpret_cast<Region *>(d.ptr + kScratchQueueOffset);
    bf.queue = q;
    bf.lvq[0] = q;
    bf.lvq[1] = q + per_table;
    // The persistent queue is cleared (by a kernel) before every render and
    // its entries carry one fixed tag, so no entry of an earlier call is
    // ever taken; only the entries this render can reach are cleared.
    bf.cap = params->form == ASK_FORM_PERSISTENT ? p.need : per_table;
    bf.clear_queue = params->form == ASK_FORM_PERSISTENT;
    bf.epoch = 1;
    bf.wait_ticks = d.wait_ticks;
    bf.grid_persistent = d.grid_persistent;
    bf.resident_level = d.resident_level;
    return launch_render(nullptr, p, bf, &im, 1, params->form, (hipStream_t)stream);
}

}  // extern "C"
