/*
 * askref.c -- CPU oracle for the Mandelbrot dwell image and its
 * Mariani-Silver subdivision image, and the same images of filled Julia sets.
 *
 * TEST INFRASTRUCTURE: the independent checker of the GPU library. Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * it. Nothing here is shared with the GPU path.
 *
 * Plain and slow on purpose: one pixel at a time, in the order the method
 * states, with threads only over independent rows (exhaustive image) or
 * independent regions (subdivision image). Build with
 *     gcc -O2 -ffp-contract=off -fPIC -shared -pthread
 * and never with -ffast-math / -Ofast: every floating-point operation must be
 * rounded on its own.
 */
#include "askref.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------------ */
/* Pixel -> c and the dwell (Sec. 6: z_{i+1} = z_i^2 + c, z_0 = 0).          */
/* ------------------------------------------------------------------------ */

/* Mapping constants, in binary64, in this order: window centre and half a
 * pixel pitch on each axis. */
void askref_map(double x0, double x1, double y0, double y1,
                uint32_t W, uint32_t H, double m[4])
{
    m[0] = 0.5 * (x0 + x1);
    m[1] = 0.5 * (y0 + y1);
    m[2] = (x1 - x0) / (2.0 * (double)W);
    m[3] = (y1 - y0) / (2.0 * (double)H);
}

/* Pixel centre: c = centre + (2p + 1 - N) * half_pitch, one multiply and one
 * add per axis (not fused). The odd integer 2p + 1 - N is exact in int64 and
 * in binary64. */
void askref_pixel_c(const double m[4], uint32_t W, uint32_t H,
                    uint32_t px, uint32_t py, double *cr, double *ci)
{
    int64_t kx = 2 * (int64_t)px + 1 - (int64_t)W;
    int64_t ky = 2 * (int64_t)py + 1 - (int64_t)H;
    double tx = (double)kx * m[2];
    double ty = (double)ky * m[3];
    *cr = m[0] + tx;
    *ci = m[1] + ty;
}

/* The dwell: iterate z <- z^2 + c from z = 0 and return the first count k at
 * which |z_k|^2 exceeds 4 (escape radius 2), or D when that never happens
 * within D iterations. Each iteration: three products, then the real and the
 * imaginary part, then the squared modulus, each operation rounded. */
uint32_t askref_dwell(double cr, double ci, uint32_t D)
{
    return askref_dwell_julia(0.0, 0.0, cr, ci, D);
}

/* The dwell in the filled Julia set of c (the other escape-time workload of
 * the same class): iterate z <- z^2 + c from z = z0 and return the first
 * count k >= 1 at which |z_k|^2 exceeds 4, or D. Each iteration: three
 * products, then the real and the imaginary part, then the squared modulus,
 * each operation rounded. The Mandelbrot dwell above is this at z0 = 0. */
uint32_t askref_dwell_julia(double zr, double zi, double cr, double ci, uint32_t D)
{
    for (uint32_t k = 1; k <= D; ++k) {
        double zr2 = zr * zr;
        double zi2 = zi * zi;
        double zri = zr * zi;
        zr = (zr2 - zi2) + cr;
        zi = (zri + zri) + ci;
        double mag = zr * zr + zi * zi;
        if (mag > 4.0)
            return k;
    }
    return D;
}

/* The dwell of pixel (px, py): its point is c (Mandelbrot) or z0 (Julia). */
static uint32_t pixel_dwell(const double m[4], uint32_t W, uint32_t H, const askref_set *set,
                            uint32_t px, uint32_t py, uint32_t D)
{
    double pr, pi;
    askref_pixel_c(m, W, H, px, py, &pr, &pi);
    if (set && set->julia)
        return askref_dwell_julia(pr, pi, set->cr, set->ci, D);
    return askref_dwell(pr, pi, D);
}

static int window_ok(double x0, double x1, double y0, double y1,
                     uint32_t W, uint32_t H, uint32_t D)
{
    if (!isfinite(x0) || !isfinite(x1) || !isfinite(y0) || !isfinite(y1))
        return 0;
    if (!(x0 < x1) || !(y0 < y1))
        return 0;
    if (W < 1 || H < 1 || W > 65536 || H > 65536 || D < 1)
        return 0;
    return 1;
}

static int thread_count(int threads)
{
    if (threads > 0)
        return threads;
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int)n : 1;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive image (Sec. 4.1): every pixel, one at a time.                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    const double *m;
    const askref_set *set;
    uint32_t W, H, D;
    uint32_t *out;
    int tid, nthreads;
    uint64_t iters;
} ex_job;

static void *ex_worker(void *arg)
{
    ex_job *j = (ex_job *)arg;
    uint64_t it = 0;
    for (uint32_t py = (uint32_t)j->tid; py < j->H; py += (uint32_t)j->nthreads) {
        for (uint32_t px = 0; px < j->W; ++px) {
            uint32_t d = pixel_dwell(j->m, j->W, j->H, j->set, px, py, j->D);
            j->out[(uint64_t)py * j->W + px] = d;
            it += d;
        }
    }
    j->iters = it;
    return NULL;
}

int askref_exhaustive(double x0, double x1, double y0, double y1,
                      uint32_t W, uint32_t H, uint32_t D,
                      uint32_t *out, uint64_t *iters_out, int threads)
{
    return askref_exhaustive_set(x0, x1, y0, y1, W, H, D, NULL, out, iters_out, threads);
}

int askref_exhaustive_set(double x0, double x1, double y0, double y1,
                          uint32_t W, uint32_t H, uint32_t D, const askref_set *set,
                          uint32_t *out, uint64_t *iters_out, int threads)
{
    if (!window_ok(x0, x1, y0, y1, W, H, D) || !out)
        return -1;
    double m[4];
    askref_map(x0, x1, y0, y1, W, H, m);
    int nt = thread_count(threads);
    if ((uint32_t)nt > H)
        nt = (int)H;
    ex_job *jobs = (ex_job *)calloc((size_t)nt, sizeof(ex_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nt, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return -1;
    }
    for (int t = 0; t < nt; ++t) {
        jobs[t] = (ex_job){m, set, W, H, D, out, t, nt, 0};
        pthread_create(&th[t], NULL, ex_worker, &jobs[t]);
    }
    uint64_t total = 0;
    for (int t = 0; t < nt; ++t) {
        pthread_join(th[t], NULL);
        total += jobs[t].iters;
    }
    free(jobs);
    free(th);
    if (iters_out)
        *iters_out = total;
    return 0;
}

void askref_dwell_pixels(double x0, double x1, double y0, double y1,
                         uint32_t W, uint32_t H, uint32_t D, uint64_t n,
                         const uint32_t *px, const uint32_t *py, uint32_t *out)
{
    askref_dwell_pixels_set(x0, x1, y0, y1, W, H, D, NULL, n, px, py, out);
}

void askref_dwell_pixels_set(double x0, double x1, double y0, double y1,
                             uint32_t W, uint32_t H, uint32_t D, const askref_set *set,
                             uint64_t n, const uint32_t *px, const uint32_t *py, uint32_t *out)
{
    double m[4];
    askref_map(x0, x1, y0, y1, W, H, m);
    for (uint64_t i = 0; i < n; ++i)
        out[i] = pixel_dwell(m, W, H, set, px[i], py[i], D);
}

/* ------------------------------------------------------------------------ */
/* Mariani-Silver subdivision (Sec. 4.2.1 for Q, T and S; Sec. 5 for the     */
/* level-by-level order).                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t x, y, w, h;   /* region [x, x+w) x [y, y+h) */
    uint32_t px, py, pw, ph; /* its parent; pw == 0 at level 0 */
} rect;

/* Floor partition of [a, a+len) into `parts` pieces: piece j is
 * [cut(j), cut(j+1)). Pieces of zero length are never made into regions. */
static uint32_t cut(uint32_t a, uint32_t len, uint32_t parts, uint32_t j)
{
    return a + (uint32_t)(((uint64_t)j * len) / parts);
}

static int on_ring(uint32_t x, uint32_t y, uint32_t w, uint32_t h,
                   uint32_t px, uint32_t py)
{
    return px == x || px == x + w - 1 || py == y || py == y + h - 1;
}

typedef struct {
    const double *m;
    const askref_set *set;
    uint32_t W, H, D, g, r, B;
    uint32_t *out;
    askref_region *recs;
    uint64_t rec_cap;
    uint64_t *rec_count; /* shared, updated atomically */
} sd_ctx;

typedef struct {
    askref_stats st;
    rect *kids;          /* children emitted by the level-by-level order */
    uint64_t nkids, capkids;
} sd_local;

static void record(const sd_ctx *c, const rect *R, uint32_t level,
                   uint32_t kind, uint32_t value)
{
    if (!c->recs)
        return;
    uint64_t i = __atomic_fetch_add(c->rec_count, 1, __ATOMIC_RELAXED);
    if (i < c->rec_cap)
        c->recs[i] = (askref_region){R->x, R->y, R->w, R->h, level, kind, value, 0};
}

static uint32_t dwell_at(const sd_ctx *c, uint32_t px, uint32_t py)
{
    return pixel_dwell(c->m, c->W, c->H, c->set, px, py, c->D);
}

/* Scan the ring of R (every pixel in the first or last column or row of R,
 * each once) and report whether all ring dwells agree; *v gets the dwell of
 * the ring's first pixel. Counts the query work Q of Sec. 4.2.1. */
static void ring_pixel(const sd_ctx *c, sd_local *L, const rect *R,
                       uint32_t px, uint32_t py, int *have, uint32_t *first,
                       int *uniform)
{
    uint32_t d = dwell_at(c, px, py);
    L->st.ring_px += 1;
    L->st.iters_ring += d;
    if (R->pw == 0 || !on_ring(R->px, R->py, R->pw, R->ph, px, py))
        L->st.iters_ring_new += d;
    if (!*have) {
        *first = d;
        *have = 1;
    } else if (d != *first) {
        *uniform = 0;
    }
}

static int scan_ring(const sd_ctx *c, sd_local *L, const rect *R, uint32_t *v)
{
    int uniform = 1;
    int have = 0;
    uint32_t first = 0;
    for (uint32_t py = R->y; py < R->y + R->h; ++py) {
        if (py == R->y || py == R->y + R->h - 1) {
            /* first or last row: all of it */
            for (uint32_t px = R->x; px < R->x + R->w; ++px)
                ring_pixel(c, L, R, px, py, &have, &first, &uniform);
        } else {
            /* a row in between: its first and last pixel */
            ring_pixel(c, L, R, R->x, py, &have, &first, &uniform);
            if (R->w > 1)
                ring_pixel(c, L, R, R->x + R->w - 1, py, &have, &first, &uniform);
        }
    }
    *v = first;
    return uniform;
}

/* Process one region: query, then terminate (fill or per-pixel leaf) or
 * split into r x r children. Children are returned through kids/nk. */
static void process(const sd_ctx *c, sd_local *L, const rect *R, uint32_t level,
                    rect *kids, uint32_t *nk)
{
    uint32_t v;
    *nk = 0;
    L->st.regions[level] += 1;
    if (level + 1 > L->st.levels)
        L->st.levels = level + 1;
    const uint64_t ring_before = L->st.iters_ring;
    int uniform = scan_ring(c, L, R, &v);
    if (uniform) {
        L->st.iters_ring_filled += L->st.iters_ring - ring_before;
        /* T: write the common ring value on every pixel of the region. */
        for (uint32_t py = R->y; py < R->y + R->h; ++py)
            for (uint32_t px = R->x; px < R->x + R->w; ++px)
                c->out[(uint64_t)py * c->W + px] = v;
        L->st.fills[level] += 1;
        L->st.fill_px += (uint64_t)R->w * R->h;
        record(c, R, level, 1, v);
        return;
    }
    if (R->w <= c->B && R->h <= c->B) {
        /* Last-level work L: every pixel of the region, one by one. */
        for (uint32_t py = R->y; py < R->y + R->h; ++py) {
            for (uint32_t px = R->x; px < R->x + R->w; ++px) {
                uint32_t d = dwell_at(c, px, py);
                c->out[(uint64_t)py * c->W + px] = d;
                L->st.iters_leaf += d;
                if (!on_ring(R->x, R->y, R->w, R->h, px, py))
                    L->st.iters_leaf_inner += d;
            }
        }
        L->st.leaves[level] += 1;
        L->st.leaf_px += (uint64_t)R->w * R->h;
        record(c, R, level, 2, 0);
        return;
    }
    /* S: split into the r x r floor partition, skipping empty pieces. */
    for (uint32_t jy = 0; jy < c->r; ++jy) {
        uint32_t y0 = cut(R->y, R->h, c->r, jy), y1 = cut(R->y, R->h, c->r, jy + 1);
        for (uint32_t jx = 0; jx < c->r; ++jx) {
            uint32_t x0 = cut(R->x, R->w, c->r, jx), x1 = cut(R->x, R->w, c->r, jx + 1);
            if (x1 > x0 && y1 > y0)
                kids[(*nk)++] = (rect){x0, y0, x1 - x0, y1 - y0, R->x, R->y, R->w, R->h};
        }
    }
    L->st.splits[level] += 1;
    record(c, R, level, 3, 0);
}

static int push_kids(sd_local *L, const rect *k, uint32_t nk)
{
    if (L->nkids + nk > L->capkids) {
        uint64_t cap = L->capkids ? L->capkids * 2 : 1024;
        while (cap < L->nkids + nk)
            cap *= 2;
        rect *p = (rect *)realloc(L->kids, cap * sizeof(rect));
        if (!p)
            return -1;
        L->kids = p;
        L->capkids = cap;
    }
    memcpy(L->kids + L->nkids, k, nk * sizeof(rect));
    L->nkids += nk;
    return 0;
}

/* Depth-first order: recurse into each child as soon as it is made. */
static int dfs(const sd_ctx *c, sd_local *L, const rect *R, uint32_t level)
{
    if (level >= ASKREF_MAX_LEVELS)
        return -1;
    rect *kids = (rect *)malloc((size_t)c->r * c->r * sizeof(rect));
    if (!kids)
        return -1;
    uint32_t nk;
    process(c, L, R, level, kids, &nk);
    int rc = 0;
    for (uint32_t i = 0; i < nk && rc == 0; ++i)
        rc = dfs(c, L, &kids[i], level + 1);
    free(kids);
    return rc;
}

typedef struct {
    const sd_ctx *c;
    sd_local L;
    const rect *items;
    uint64_t nitems;
    uint64_t *next;     /* shared work index */
    uint32_t level;
    int order;
    int rc;
} sd_job;

static void *sd_worker(void *arg)
{
    sd_job *j = (sd_job *)arg;
    rect *kids = (rect *)malloc((size_t)j->c->r * j->c->r * sizeof(rect));
    if (!kids) {
        j->rc = -1;
        return NULL;
    }
    for (;;) {
        uint64_t i = __atomic_fetch_add(j->next, 1, __ATOMIC_RELAXED);
        if (i >= j->nitems)
            break;
        if (j->order == 1) {
            if (dfs(j->c, &j->L, &j->items[i], j->level) != 0)
                j->rc = -1;
        } else {
            uint32_t nk;
            process(j->c, &j->L, &j->items[i], j->level, kids, &nk);
            if (nk && push_kids(&j->L, kids, nk) != 0)
                j->rc = -1;
        }
    }
    free(kids);
    return NULL;
}

static void add_stats(askref_stats *a, const askref_stats *b)
{
    if (b->levels > a->levels)
        a->levels = b->levels;
    for (int i = 0; i < ASKREF_MAX_LEVELS; ++i) {
        a->regions[i] += b->regions[i];
        a->fills[i] += b->fills[i];
        a->splits[i] += b->splits[i];
        a->leaves[i] += b->leaves[i];
    }
    a->ring_px += b->ring_px;
    a->leaf_px += b->leaf_px;
    a->fill_px += b->fill_px;
    a->iters_ring += b->iters_ring;
    a->iters_leaf += b->iters_leaf;
    a->iters_ring_new += b->iters_ring_new;
    a->iters_leaf_inner += b->iters_leaf_inner;
    a->iters_ring_filled += b->iters_ring_filled;
}

int64_t askref_subdiv(double x0, double x1, double y0, double y1,
                      uint32_t W, uint32_t H, uint32_t D,
                      uint32_t g, uint32_t r, uint32_t B, int order, int threads,
                      uint32_t *out, askref_stats *stats,
                      askref_region *recs, uint64_t rec_cap)
{
    return askref_subdiv_set(x0, x1, y0, y1, W, H, D, NULL, g, r, B, order, threads, out,
                             stats, recs, rec_cap);
}

int64_t askref_subdiv_set(double x0, double x1, double y0, double y1,
                          uint32_t W, uint32_t H, uint32_t D, const askref_set *set,
                          uint32_t g, uint32_t r, uint32_t B, int order, int threads,
                          uint32_t *out, askref_stats *stats,
                          askref_region *recs, uint64_t rec_cap)
{
    if (!window_ok(x0, x1, y0, y1, W, H, D) || !out)
        return -1;
    if (g < 1 || g > W || g > H || r < 2 || B < 1 || (order != 0 && order != 1))
        return -1;
    double m[4];
    askref_map(x0, x1, y0, y1, W, H, m);
    uint64_t rec_count = 0;
    sd_ctx c = {m, set, W, H, D, g, r, B, out, recs, rec_cap, &rec_count};
    askref_stats total;
    memset(&total, 0, sizeof(total));

    /* Level 0: the g x g floor partition of the image (Sec. 4.2, G = g^2). */
    uint64_t n = (uint64_t)g * g;
    rect *cur = (rect *)malloc(n * sizeof(rect));
    if (!cur)
        return -1;
    uint64_t k = 0;
    for (uint32_t jy = 0; jy < g; ++jy)
        for (uint32_t jx = 0; jx < g; ++jx) {
            uint32_t xa = cut(0, W, g, jx), xb = cut(0, W, g, jx + 1);
            uint32_t ya = cut(0, H, g, jy), yb = cut(0, H, g, jy + 1);
            cur[k++] = (rect){xa, ya, xb - xa, yb - ya, 0, 0, 0, 0};
        }

    int nt = thread_count(threads);
    int rc = 0;
    uint32_t level = 0;
    while (n > 0 && rc == 0) {
        if (level >= ASKREF_MAX_LEVELS) {
            rc = -1;
            break;
        }
        int use = nt;
        if ((uint64_t)use > n)
            use = (int)n;
        sd_job *jobs = (sd_job *)calloc((size_t)use, sizeof(sd_job));
        pthread_t *th = (pthread_t *)calloc((size_t)use, sizeof(pthread_t));
        if (!jobs || !th) {
            free(jobs);
            free(th);
            rc = -1;
            break;
        }
        uint64_t next = 0;
        for (int t = 0; t < use; ++t) {
            jobs[t].c = &c;
            jobs[t].items = cur;
            jobs[t].nitems = n;
            jobs[t].next = &next;
            jobs[t].level = level;
            jobs[t].order = order;
            pthread_create(&th[t], NULL, sd_worker, &jobs[t]);
        }
        uint64_t nn = 0;
        for (int t = 0; t < use; ++t) {
            pthread_join(th[t], NULL);
            if (jobs[t].rc)
                rc = -1;
            nn += jobs[t].L.nkids;
        }
        /* The children of this level, concatenated, are the next level. */
        rect *nxt = nn ? (rect *)malloc(nn * sizeof(rect)) : NULL;
        uint64_t o = 0;
        for (int t = 0; t < use; ++t) {
            add_stats(&total, &jobs[t].L.st);
            if (nxt && jobs[t].L.nkids)
                memcpy(nxt + o, jobs[t].L.kids, jobs[t].L.nkids * sizeof(rect));
            o += jobs[t].L.nkids;
            free(jobs[t].L.kids);
        }
        if (nn && !nxt)
            rc = -1;
        free(jobs);
        free(th);
        free(cur);
        cur = nxt;
        n = nn;
        level += 1;
    }
    free(cur);
    if (rc != 0)
        return -1;
    if (stats)
        *stats = total;
    return recs ? (int64_t)rec_count : 0;
}

/* ------------------------------------------------------------------------ */
/* Subdivision values at sampled pixels, by descent through the region tree. */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t x, y, w, h;
    int uniform;
    uint32_t v;
} seen_region;

int askref_subdiv_pixels(double x0, double x1, double y0, double y1,
                         uint32_t W, uint32_t H, uint32_t D,
                         uint32_t g, uint32_t r, uint32_t B,
                         uint64_t n, const uint32_t *px, const uint32_t *py,
                         uint32_t *out)
{
    return askref_subdiv_pixels_set(x0, x1, y0, y1, W, H, D, NULL, g, r, B, n, px, py, out);
}

int askref_subdiv_pixels_set(double x0, double x1, double y0, double y1,
                             uint32_t W, uint32_t H, uint32_t D, const askref_set *set,
                             uint32_t g, uint32_t r, uint32_t B,
                             uint64_t n, const uint32_t *px, const uint32_t *py,
                             uint32_t *out)
{
    if (!window_ok(x0, x1, y0, y1, W, H, D))
        return -1;
    if (g < 1 || g > W || g > H || r < 2 || B < 1)
        return -1;
    double m[4];
    askref_map(x0, x1, y0, y1, W, H, m);
    sd_ctx c = {m, set, W, H, D, g, r, B, NULL, NULL, 0, NULL};
    sd_local L;
    memset(&L, 0, sizeof(L));
    seen_region *seen = NULL;
    uint64_t nseen = 0, capseen = 0;

    for (uint64_t i = 0; i < n; ++i) {
        uint32_t qx = px[i], qy = py[i];
        if (qx >= W || qy >= H) {
            free(seen);
            return -1;
        }
        /* level-0 region holding (qx, qy) */
        uint32_t jx = 0, jy = 0;
        while (!(cut(0, W, g, jx) <= qx && qx < cut(0, W, g, jx + 1)))
            ++jx;
        while (!(cut(0, H, g, jy) <= qy && qy < cut(0, H, g, jy + 1)))
            ++jy;
        rect R = {cut(0, W, g, jx), cut(0, H, g, jy), 0, 0, 0, 0, 0, 0};
        R.w = cut(0, W, g, jx + 1) - R.x;
        R.h = cut(0, H, g, jy + 1) - R.y;
        for (;;) {
            int uniform = 0;
            uint32_t v = 0;
            int found = 0;
            for (uint64_t s = 0; s < nseen; ++s) {
                if (seen[s].x == R.x && seen[s].y == R.y && seen[s].w == R.w && seen[s].h == R.h) {
                    uniform = seen[s].uniform;
                    v = seen[s].v;
                    found = 1;
                    break;
                }
            }
            if (!found) {
                uniform = scan_ring(&c, &L, &R, &v);
                if (nseen == capseen) {
                    capseen = capseen ? capseen * 2 : 256;
                    seen_region *p = (seen_region *)realloc(seen, capseen * sizeof(seen_region));
                    if (!p) {
                        free(seen);
                        return -1;
                    }
                    seen = p;
                }
                seen[nseen++] = (seen_region){R.x, R.y, R.w, R.h, uniform, v};
            }
            if (uniform) {
                out[i] = v;
                break;
            }
            if (R.w <= B && R.h <= B) {
                out[i] = dwell_at(&c, qx, qy);
                break;
            }
            /* child of R holding (qx, qy) */
            uint32_t kx = 0, ky = 0;
            while (!(cut(R.x, R.w, r, kx) <= qx && qx < cut(R.x, R.w, r, kx + 1)))
                ++kx;
            while (!(cut(R.y, R.h, r, ky) <= qy && qy < cut(R.y, R.h, r, ky + 1)))
                ++ky;
            rect C = {cut(R.x, R.w, r, kx), cut(R.y, R.h, r, ky), 0, 0, R.x, R.y, R.w, R.h};
            C.w = cut(R.x, R.w, r, kx + 1) - C.x;
            C.h = cut(R.y, R.h, r, ky + 1) - C.y;
            R = C;
        }
    }
    free(seen);
    return 0;
}
