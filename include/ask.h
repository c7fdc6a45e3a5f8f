/*
 * ask.h -- C ABI of the MI355X (gfx950) library for Mandelbrot dwell images
 * by exhaustive evaluation and by Mariani-Silver subdivision, run as
 * Adaptive Serial Kernels (per-level kernels over a compact region queue) or
 * as one persistent kernel over a device-resident region queue.
 *
 * Paper: Quezada, Navarro, Romero, Aguilera, "Modeling GPU Dynamic
 * Parallelism for Self Similar Density Workloads" (arXiv 2206.02255).
 *   - dwell of c: Sec. 6 (z_{i+1} = z_i^2 + c, z_0 = 0, escape radius 2);
 *   - exhaustive image: Sec. 4.1 (W_E = n^2 A, one work unit per pixel);
 *   - subdivision: Sec. 4.2 and 4.2.1 (initial g x g grid, border query Q,
 *     uniform border -> fill T, otherwise split r x r at cost S, until regions
 *     reach the stop size B, then per-pixel work L);
 *   - level-by-level execution with an offset lookup table that is appended
 *     with one atomic add per splitting region and swapped between levels:
 *     Sec. 5.1-5.3.
 *
 * Conventions shared by every call
 *   - Plain C types only; no exception crosses the ABI. Every call returns an
 *     ask_status; ASK_OK is 0, errors are negative.
 *   - Images are W x H uint32 dwell values in device memory, row-major
 *     (index py*W + px), row 0 on the y0 side. The caller owns them; the
 *     library never allocates or frees them.
 *   - Pixel (px, py) maps to c = (cxm + (2px+1-W) hx, cym + (2py+1-H) hy)
 *     with cxm = (x0+x1)/2, cym = (y0+y1)/2, hx = (x1-x0)/(2W),
 *     hy = (y1-y0)/(2H), each operation rounded to binary64 on its own; the
 *     dwell loop is evaluated in binary64 without fused multiply-add, so the
 *     images are bit-for-bit reproducible.
 *   - Calls enqueue work on the given HIP stream (hipStream_t passed as
 *     void*, NULL = the default stream) and return without waiting, except
 *     where stated. Argument errors are reported synchronously.
 *   - A context is bound to one device and is not thread-safe; use one per
 *     host thread. Calls on one context must be ordered on one stream, as
 *     they share the context's queue memory.
 */
#ifndef ASK_H
#define ASK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASK_MAX_LEVELS 64

typedef enum ask_status {
    ASK_OK = 0,
    ASK_EINVAL = -1,    /* bad argument (window, params, pointer) */
    ASK_ENOMEM = -2,    /* device or host allocation failed */
    ASK_EDEVICE = -3,   /* HIP runtime error; see ask_last_error */
    ASK_EOVERFLOW = -4, /* the region queue was too small; the image is invalid */
    ASK_EBUSY = -5,     /* cannot accept the request now */
    ASK_ETIMEOUT = -6   /* a wait ran out of time */
} ask_status;

/* The escape-time set whose dwell image a window samples (the paper's
 * self-similar workload class). In both, z_k = z_{k-1}^2 + c and the dwell
 * of a pixel is the first k >= 1 with |z_k|^2 > 4, or D if there is none.
 *   ASK_SET_MANDELBROT: the pixel's point is c, and z_0 = 0 (Sec. 6).
 *   ASK_SET_JULIA: the filled Julia set of the window's fixed c = (cr, ci);
 *   the pixel's point is z_0. */
enum { ASK_SET_MANDELBROT = 0, ASK_SET_JULIA = 1 };

/* A complex window [x0, x1] x [y0, y1] rendered at W x H pixels with
 * maximum dwell D. Valid: finite bounds, x0 < x1, y0 < y1,
 * 1 <= W, H <= 65536, 1 <= D <= 2^31 - 1, set one of ASK_SET_*, and for
 * ASK_SET_JULIA finite cr, ci. A zeroed set field is the Mandelbrot set. */
typedef struct ask_window {
    double x0, x1, y0, y1;
    uint32_t W, H, D;
    uint32_t set;   /* ASK_SET_MANDELBROT or ASK_SET_JULIA */
    double cr, ci;  /* ASK_SET_JULIA: the fixed c; ignored otherwise */
} ask_window;

/* Execution form of a subdivision render. */
typedef enum ask_form {
    /* Adaptive Serial Kernels (Sec. 5): one kernel per level; every kernel
     * reads the level's region count from device memory, so the host never
     * waits between levels. */
    ASK_FORM_LEVELS = 0,
    /* The same, with the region count read back to the host after every
     * level to size the next grid, as the paper's host loop does (Sec.
     * 5.3.2). Synchronises the stream once per level. */
    ASK_FORM_LEVELS_READBACK = 1,
    /* One persistent kernel whose waves pull regions from a device-resident
     * queue until all work is done. */
    ASK_FORM_PERSISTENT = 2
} ask_form;

/* Leaf work (Sec. 4.3: one block per region, SBR, against several blocks
 * per region, MBR): a leaf of more than `band` pixels is cut into row bands
 * of about `band` pixels that any wave may take (MBR): in the persistent
 * form and in serving they are queued, in the per-level forms put into the
 * next level's table (one more level kernel takes the bands of last-level
 * leaves). Smaller leaves, and every leaf with ASK_BAND_NONE, are computed
 * whole by the wave that decided them (SBR); the one exception is a leaf of
 * 65536 x 65536 pixels, whose 2^32 pixels one 32-bit stream cannot index:
 * it is always cut into bands of 2^24 pixels. 0 selects ASK_BAND_DEFAULT. */
#define ASK_BAND_DEFAULT 1024u
#define ASK_BAND_NONE 0xffffffffu

/* Subdivision parameters (Sec. 4.2.1, 6.2): an initial g x g grid of
 * regions, r x r splits, stop size B (a region with both sides <= B whose
 * border is not uniform is computed per pixel). Valid: 1 <= g <= min(W, H),
 * 2 <= r <= 1024, 1 <= B <= 65536. form: an ask_form. band: 0,
 * ASK_BAND_NONE, or 64 <= band <= 2^24 (see above).
 *
 * tile_w x tile_h: the pixel tile of one 64-lane wave, the block shape of
 * the paper's block-size study (Sec. 6.2, its Table 2). Either both 0 (the
 * defaults) or tile_w in {4, 8, 16, 32, 64} with tile_w * tile_h = 64.
 *   - ask_dwell_exhaustive: each wave computes one tile, a workgroup four
 *     tiles stacked vertically (default 16 x 4, i.e. 16 x 16 workgroups);
 *   - subdivision: the pixels of a leaf (or leaf band) are handed to the
 *     lanes tile by tile, tiles in row-major order over the leaf and pixels
 *     row-major within a tile (default: the leaf's rows, one after another).
 * The tile changes only the order of work, never an image. */
typedef struct ask_params {
    uint32_t g, r, B;
    uint32_t form;
    uint32_t band;
    uint32_t tile_w, tile_h;
} ask_params;

/* Work counters of a render, filled when the caller asks for them. */
typedef struct ask_stats {
    uint32_t levels;                       /* deepest level reached + 1 */
    uint32_t overflow;                     /* nonzero: queue capacity exceeded */
    uint64_t regions[ASK_MAX_LEVELS];      /* regions scanned per level */
    uint64_t fills[ASK_MAX_LEVELS];        /* uniform border -> filled */
    uint64_t splits[ASK_MAX_LEVELS];       /* split into children */
    uint64_t leaves[ASK_MAX_LEVELS];       /* computed per pixel */
    uint64_t iters_ring;                   /* dwell iterations computed on borders (a
                                              border found mixed stops early, so this
                                              can be below the sum of its dwells) */
    uint64_t iters_leaf;                   /* dwell iterations computed for leaf pixels
                                              that are not on the leaf's border (a leaf
                                              keeps its border's dwells), and for every
                                              pixel of leaves cut into bands */
    uint64_t ring_px;                      /* border pixels of scanned regions */
    uint64_t leaf_px;                      /* pixels of leaf regions */
    uint64_t fill_px;                      /* pixels of filled regions */
} ask_stats;

typedef struct ask_ctx ask_ctx;

/* Human-readable name of a status code (static storage). */
const char *ask_status_str(ask_status s);

/* Text of the last error on this context (static per context; never NULL). */
const char *ask_last_error(const ask_ctx *ctx);

/* Create a context on HIP device `device`. *out receives the context, or
 * NULL on error. Returns ASK_EDEVICE when no such device exists.
 * queue_bytes: device memory to set aside now for each region queue of the
 * context (the persistent queue and the two per-level tables), so that
 * renders whose worst case fits allocate nothing; 0 allocates on first use.
 * A render whose worst case exceeds a queue grows it (waiting for earlier
 * renders on the context first). ASK_ENOMEM if it cannot be allocated. */
ask_status ask_create(ask_ctx **out, int device, size_t queue_bytes);

/* Release a context and all device memory it owns (after waiting for its
 * work). NULL is accepted. */
ask_status ask_destroy(ask_ctx *ctx);

/* Host-only helpers (no device needed). */

/* Check a window (and params, when not NULL) for validity. */
ask_status ask_validate(const ask_window *win, const ask_params *params);

/* Mapping constants {cxm, cym, hx, hy} of a window, as the kernels use them. */
ask_status ask_mapping(const ask_window *win, double out[4]);

/* Number of levels a subdivision can reach: 1 + the number of r-fold
 * splits that take the largest level-0 side down to B or below. */
ask_status ask_level_count(const ask_window *win, const ask_params *params,
                           uint32_t *levels);

/* Exhaustive image (Sec. 4.1): d_out[py*W + px] = dwell(c(px, py)) for all
 * pixels. d_out: device memory, W*H uint32, caller-owned. params: NULL, or
 * parameters of which only the wave tile (tile_w, tile_h) is read and
 * checked; the other fields are ignored. */
ask_status ask_dwell_exhaustive(ask_ctx *ctx, const ask_window *win,
                                const ask_params *params, uint32_t *d_out, void *stream);

/* Subdivision image (Sec. 4.2.1, 5): every region of the initial g x g grid
 * has its border dwells computed; a uniform border fills the region with
 * that value, otherwise the region is computed per pixel when both its
 * sides are <= B, or split into its r x r floor partition (pieces
 * [a + j*len/r, a + (j+1)*len/r), empty pieces dropped). d_out as above.
 * stats: NULL, or receives the work counters; a non-NULL stats makes the
 * call wait for the stream and return any error the render recorded (as
 * ask_synchronize does). The call also waits for the stream when the queue
 * could overflow (very large images with tiny B); an overflow then returns
 * ASK_EOVERFLOW. Otherwise device-side errors surface at ask_synchronize.
 *
 * Graphs: the call may be made on a stream that is capturing (HIP stream
 * capture), for the levels and persistent forms, with stats == NULL, after
 * one render of the same size outside the capture (so that no queue grows
 * while capturing; ASK_EINVAL otherwise). The graph then replays the whole
 * render; a captured persistent render clears its own queue at every replay.
 * The context never frees a buffer that a captured render names (it only
 * retires it until ask_destroy), so graphs stay valid while the context
 * lives. */
ask_status ask_dwell_subdiv(ask_ctx *ctx, const ask_window *win,
                            const ask_params *params, uint32_t *d_out,
                            void *stream, ask_stats *stats);

/* Device memory, in bytes, that ask_dwell_subdiv_noalloc works in: one
 * array per device, held from the library's first use on that device until
 * the process ends. */
#define ASK_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid allocation): the subdivision image of
 * ask_dwell_subdiv, bit for bit, without a context and without allocating
 * anything. The render's control words and region queue live in a fixed
 * array of ASK_NOALLOC_SCRATCH_BYTES of device memory on the current HIP
 * device; the call only launches kernels on `stream` and returns.
 * params->form: ASK_FORM_LEVELS or ASK_FORM_PERSISTENT. A window whose worst
 * case does not fit the array (for the persistent form, the queue bound of
 * ask_dwell_subdiv: 16 bytes per region a render can reach and per leaf band;
 * for the per-level form, two tables of the widest level) is refused with
 * ASK_EINVAL, so no queue can overflow. Every call on a device shares that
 * device's array, which keeps the last call's contents (each call clears
 * what it needs): calls that overlap on one device race and give invalid
 * images, so order them on one stream. A wave that waits longer than 10 s
 * leaves (the image is then invalid); this call reports no device-side
 * error. Errors: ASK_EINVAL (arguments, size, form), ASK_EDEVICE (no
 * current device, or a launch failed). */
ask_status ask_dwell_subdiv_noalloc(const ask_window *win, const ask_params *params,
                                    uint32_t *d_out, void *stream);

/* A batch of n >= 1 subdivision images rendered by one sequence of launches
 * over one shared region queue: one seeding pass for all images, then one
 * persistent kernel (or one kernel per level) whose waves take regions of
 * any image. Each image i is the image ask_dwell_subdiv would give for
 * wins[i] and its parameters, bit for bit. params: nparams == 1 (shared by
 * all images) or nparams == n (one per image); every entry must have the
 * same form. d_outs[i]: device memory, wins[i].W * wins[i].H uint32,
 * caller-owned; images must not overlap. stats (optional) sums the counters
 * over the batch and makes the call wait, as for ask_dwell_subdiv. The image
 * table and the level-0 seed offsets go to device memory through kernels
 * that carry them as arguments, so a stream capture records the data: on a
 * capturing stream the batch gets a table of its own, which no later call
 * writes and the context frees only when it is destroyed, and the graph
 * can be replayed as often as wanted; otherwise the batch uses the
 * context's table, which the next batch on the context overwrites (calls
 * on different streams must be ordered by the caller). Errors as for
 * ask_dwell_subdiv, and ASK_ENOMEM when the table cannot be allocated. */
ask_status ask_dwell_batch(ask_ctx *ctx, uint32_t n, const ask_window *wins,
                           const ask_params *params, uint32_t nparams,
                           uint32_t *const *d_outs, void *stream, ask_stats *stats);

/* Wait for `stream`, then report the errors the kernels recorded on this
 * context since the last check: ASK_ETIMEOUT when a persistent wave gave up
 * waiting (see ask_set_wait_limit), else ASK_EOVERFLOW when a queue ran out
 * of room, else ASK_OK. The recorded errors are cleared. A render that
 * reports either error has left an invalid image. */
ask_status ask_synchronize(ask_ctx *ctx, void *stream);

/* Record HIP events, on the render's stream, around the dominant kernels of
 * later renders on this context (on != 0; the count of timed renders starts
 * again from 0), or stop (on == 0). Dominant
 * kernels: the exhaustive kernel; the level kernels, from the first one's
 * start to the last one's end; the persistent kernel. Set-up kernels (counter
 * reset, level-0 seeding) are outside the events. */
ask_status ask_enable_timing(ask_ctx *ctx, int on);

/* Device time, in milliseconds, of the dominant kernels of the last render
 * timed on this context. Waits for that render; ASK_EINVAL if there is none. */
ask_status ask_last_kernel_ms(ask_ctx *ctx, float *ms);

/* Device times, in milliseconds, of the dominant kernels of the last
 * min(timed renders, cap, 256) renders timed since ask_enable_timing(ctx, 1),
 * oldest first, into ms[0 .. *n). Waits for those renders. */
ask_status ask_kernel_times(ask_ctx *ctx, float *ms, uint32_t cap, uint32_t *n);

/* Longest time, in seconds (0 to 3600, default 10), that one wave of the
 * persistent kernel waits for a region before it records ASK_ETIMEOUT and
 * leaves. This bounds every wait of the kernel, so its grid always drains;
 * a render never legitimately idles a wave for seconds. */
ask_status ask_set_wait_limit(ask_ctx *ctx, double seconds);

/* ------------------------------------------------------------------------
 * Serving: continuous batching into one persistent kernel.
 *
 * A server owns one long-running kernel on a stream of its own. Requests
 * (a window, its parameters and a caller-owned output image) are posted
 * while the kernel runs; an idle wave admits a posted request into a free
 * slot, writes its level-0 regions into that request's own region queue in
 * device memory, and from then on every wave of the kernel takes regions of
 * any admitted request, so requests that arrive while others run overlap
 * with them on the device. The wave that finishes a request's last region
 * reports it to the host through pinned host memory. Each image is the one
 * ask_dwell_subdiv gives for the same window and parameters, bit for bit.
 *
 * Admission is by device memory: each request reserves, in the server's
 * pool, the worst-case size of its region queue (the bound
 * ask_dwell_subdiv sizes its queue by); a request that does not fit,
 * or finds every slot taken, is refused with ASK_EBUSY and can be posted
 * again once earlier requests have finished.
 *
 * The kernel keeps waves_per_cu waves resident on every CU until
 * ask_server_destroy; other kernels on the device run beside it in the room
 * it leaves. One server per context; a server is not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct ask_server ask_server;

typedef struct ask_server_cfg {
    uint32_t slots;        /* requests admitted at once, 1..64 */
    uint32_t waves_per_cu; /* resident server waves per CU, a multiple of 4;
                              0: all but one 4-wave workgroup of the
                              kernel's occupancy */
    uint64_t pool_bytes;   /* device memory for the requests' region queues
                              (0: 256 MiB) */
} ask_server_cfg;

/* Start a server on ctx's device. *out receives it, or NULL on error. */
ask_status ask_server_create(ask_ctx *ctx, const ask_server_cfg *cfg, ask_server **out);

/* Post one request. win and params are checked as for ask_dwell_subdiv
 * (params->form is ignored). d_out: device memory, W*H uint32, caller-owned,
 * not to be read or freed until the request has finished. On ASK_OK,
 * *ticket receives the request's ticket (increasing from 1). ASK_EBUSY: no
 * free slot or not enough pool memory right now (finished requests are
 * reaped first, so retrying after a completion can succeed); ASK_ENOMEM:
 * the request's worst case exceeds the whole pool. */
ask_status ask_server_submit(ask_server *sv, const ask_window *win,
                             const ask_params *params, uint32_t *d_out,
                             uint64_t *ticket);

/* Collect finished requests: up to cap of them, in any order, into
 * tickets[] with each one's status (ASK_OK; ASK_ETIMEOUT or ASK_EOVERFLOW
 * for a request whose image is invalid) in status[] (may be NULL); *n gets
 * the count. A finished request's image is complete in device memory and
 * visible to later work on any stream. Does not wait. */
ask_status ask_server_reap(ask_server *sv, uint64_t *tickets, int32_t *status,
                           uint32_t cap, uint32_t *n);

/* *done = 1 when request `ticket` has finished (reaping it if needed), else
 * 0. Returns the request's status once finished; ASK_EINVAL for a ticket
 * never issued. latency_s (may be NULL) receives, once finished, the
 * request's latency in seconds: from its ask_server_submit to the host's
 * first sight of its completion (by a reap or a poll), on the host's
 * monotonic clock; -1 while it runs. Does not wait. */
ask_status ask_server_poll(ask_server *sv, uint64_t ticket, int *done, double *latency_s);

/* Requests posted and not yet reaped. */
ask_status ask_server_in_flight(const ask_server *sv, uint32_t *n);

/* Wait (up to the context's wait limit) for the requests in flight, stop
 * the kernel and release the server. NULL is accepted. ASK_ETIMEOUT if the
 * requests did not finish in time (the kernel is still stopped). */
ask_status ask_server_destroy(ask_server *sv);

#ifdef __cplusplus
}
#endif
#endif
