/*
 * askref3.c -- CPU oracle for the 3-D extension of the subdivision (the
 * paper's section on subdivisions at higher dimensions): a dwell volume and
 * its Mariani-Silver subdivision over boxes (3-orthotopes), with the level
 * tables holding one space-filling-curve scalar per box.
 *
 * TEST INFRASTRUCTURE: the independent checker of the GPU library's 3-D
 * entry points. Only the test suite and the smoke check load it. Nothing here
 * is shared with the GPU path.
 *
 * The volume: voxel (px, py, pz) of a W x H x L grid over the box
 * [x0, x1] x [y0, y1] x [z0, z1] stands for the point (x, y, z) at the voxel
 * centre, mapped per axis as in the 2-D oracle (centre + (2p + 1 - N) * half
 * pitch). Its dwell is the escape time of the quaternion Julia iteration
 * q <- q^2 + c from q0 = x + y i + z j with c = cr + ci i: with q = a + b i + e j
 * (the k part stays 0), q^2 = (a^2 - b^2 - e^2) + 2ab i + 2ae j. The j = 0
 * slice is the filled Julia set of the complex c, and the order of the
 * operations below makes it that image bit for bit.
 *
 * Plain and slow on purpose. Build with gcc -O2 -ffp-contract=off.
 */
#include "askref3.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------------ */
/* Voxel -> point and the dwell.                                            */
/* ------------------------------------------------------------------------ */

void askref3_map(const double box[6], uint32_t W, uint32_t H, uint32_t L, double m[6])
{
    m[0] = 0.5 * (box[0] + box[1]);
    m[1] = 0.5 * (box[2] + box[3]);
    m[2] = 0.5 * (box[4] + box[5]);
    m[3] = (box[1] - box[0]) / (2.0 * (double)W);
    m[4] = (box[3] - box[2]) / (2.0 * (double)H);
    m[5] = (box[5] - box[4]) / (2.0 * (double)L);
}

static double axis_point(double centre, double half, uint32_t p, uint32_t n)
{
    int64_t k = 2 * (int64_t)p + 1 - (int64_t)n;
    double t = (double)k * half;
    return centre + t;
}

/* The first k >= 1 with |q_k|^2 > 4, else D. Per iteration: the products,
 * then the three parts, then the squared modulus, each operation rounded;
 * b^2 + e^2 is summed first so that e = 0 gives the complex iteration's
 * operations exactly. */
uint32_t askref3_dwell(double a, double b, double e, double cr, double ci, uint32_t D)
{
    for (uint32_t k = 1; k <= D; ++k) {
        double a2 = a * a;
        double b2 = b * b;
        double e2 = e * e;
        double ab = a * b;
        double ae = a * e;
        a = (a2 - (b2 + e2)) + cr;
        b = (ab + ab) + ci;
        e = (ae + ae) + 0.0;
        double mag = a * a + (b * b + e * e);
        if (mag > 4.0)
            return k;
    }
    return D;
}

typedef struct vol {
    double m[6];
    double cr, ci;
    uint32_t n[3];
    uint32_t D;
} vol;

static uint32_t voxel_dwell(const vol *v, uint32_t px, uint32_t py, uint32_t pz)
{
    double a = axis_point(v->m[0], v->m[3], px, v->n[0]);
    double b = axis_point(v->m[1], v->m[4], py, v->n[1]);
    double e = axis_point(v->m[2], v->m[5], pz, v->n[2]);
    return askref3_dwell(a, b, e, v->cr, v->ci, v->D);
}

uint32_t askref3_voxel_dwell(const double box[6], uint32_t W, uint32_t H, uint32_t L,
                             double cr, double ci, uint32_t D,
                             uint32_t px, uint32_t py, uint32_t pz)
{
    vol v;
    askref3_map(box, W, H, L, v.m);
    v.cr = cr, v.ci = ci, v.D = D;
    v.n[0] = W, v.n[1] = H, v.n[2] = L;
    return voxel_dwell(&v, px, py, pz);
}

static int threads(void)
{
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n < 1 ? 1 : (n > 64 ? 64 : (int)n);
}

/* ------------------------------------------------------------------------ */
/* Exhaustive volume: every voxel, x fastest, then y, then z.               */
/* ------------------------------------------------------------------------ */

typedef struct ex_job {
    const vol *v;
    uint32_t *out;
    uint32_t next;
    pthread_mutex_t mu;
} ex_job;

static void *ex_worker(void *p)
{
    ex_job *j = (ex_job *)p;
    const vol *v = j->v;
    for (;;) {
        pthread_mutex_lock(&j->mu);
        uint32_t pz = j->next++;
        pthread_mutex_unlock(&j->mu);
        if (pz >= v->n[2])
            return NULL;
        for (uint32_t py = 0; py < v->n[1]; ++py)
            for (uint32_t px = 0; px < v->n[0]; ++px)
                j->out[((uint64_t)pz * v->n[1] + py) * v->n[0] + px] = voxel_dwell(v, px, py, pz);
    }
}

static int vol_ok(uint32_t W, uint32_t H, uint32_t L, uint32_t D)
{
    return W >= 1 && H >= 1 && L >= 1 && D >= 1 && W <= 65536 && H <= 65536 && L <= 65536;
}

int askref3_exhaustive(const double box[6], uint32_t W, uint32_t H, uint32_t L,
                       double cr, double ci, uint32_t D, uint32_t *out)
{
    if (!vol_ok(W, H, L, D))
        return -1;
    vol v;
    askref3_map(box, W, H, L, v.m);
    v.cr = cr, v.ci = ci, v.D = D;
    v.n[0] = W, v.n[1] = H, v.n[2] = L;
    ex_job j = {&v, out, 0, PTHREAD_MUTEX_INITIALIZER};
    int nt = threads();
    pthread_t th[64];
    for (int t = 0; t < nt; ++t)
        pthread_create(&th[t], NULL, ex_worker, &j);
    for (int t = 0; t < nt; ++t)
        pthread_join(th[t], NULL);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Space-filling curves over a level's grid of G x G x G cells.             */
/* ------------------------------------------------------------------------ */

/* Canonical (nested-loop) order: x fastest, then y, then z. */
uint64_t askref3_canonical(uint64_t G, const uint32_t p[3])
{
    return ((uint64_t)p[2] * G + p[1]) * G + p[0];
}

void askref3_canonical_inv(uint64_t G, uint64_t s, uint32_t p[3])
{
    p[0] = (uint32_t)(s % G);
    s /= G;
    p[1] = (uint32_t)(s % G);
    p[2] = (uint32_t)(s / G);
}

/* Morton (Z) order: bit t of p_x, p_y, p_z goes to bit 3t, 3t + 1, 3t + 2. */
uint64_t askref3_morton(const uint32_t p[3])
{
    uint64_t s = 0;
    for (int t = 0; t < 21; ++t)
        for (int d = 0; d < 3; ++d)
            s |= (uint64_t)((p[d] >> t) & 1u) << (3 * t + d);
    return s;
}

void askref3_morton_inv(uint64_t s, uint32_t p[3])
{
    p[0] = p[1] = p[2] = 0;
    for (int t = 0; t < 21; ++t)
        for (int d = 0; d < 3; ++d)
            p[d] |= (uint32_t)((s >> (3 * t + d)) & 1u) << t;
}

static uint64_t encode(int order, uint64_t G, const uint32_t p[3])
{
    return order == ASKREF3_MORTON ? askref3_morton(p) : askref3_canonical(G, p);
}

static void decode(int order, uint64_t G, uint64_t s, uint32_t p[3])
{
    if (order == ASKREF3_MORTON)
        askref3_morton_inv(s, p);
    else
        askref3_canonical_inv(G, s, p);
}

/* Cell j of a floor partition of n voxels into G cells: [lo(j), lo(j + 1)). */
uint32_t askref3_cell_lo(uint64_t j, uint64_t G, uint32_t n)
{
    return (uint32_t)(j * (uint64_t)n / G);
}

/* ------------------------------------------------------------------------ */
/* Subdivision, level by level.                                             */
/* ------------------------------------------------------------------------ */

/* Level i's grid has G_i = g * r^i cells per axis; the r^3 cells
 * (r p + k) of level i + 1 tile cell p of level i exactly, so a box is
 * named by its level and its cell, and the table holds one scalar per box. */
typedef struct box3 {
    uint32_t lo[3], hi[3];
} box3;

static int cell_box(const vol *v, uint64_t G, const uint32_t p[3], box3 *b)
{
    for (int d = 0; d < 3; ++d) {
        b->lo[d] = askref3_cell_lo(p[d], G, v->n[d]);
        b->hi[d] = askref3_cell_lo((uint64_t)p[d] + 1, G, v->n[d]);
        if (b->hi[d] <= b->lo[d])
            return 0;
    }
    return 1;
}

static int on_surface(const box3 *b, uint32_t x, uint32_t y, uint32_t z)
{
    return x == b->lo[0] || x == b->hi[0] - 1 || y == b->lo[1] || y == b->hi[1] - 1 ||
           z == b->lo[2] || z == b->hi[2] - 1;
}

static void put(const vol *v, uint32_t *out, uint32_t x, uint32_t y, uint32_t z, uint32_t d)
{
    out[((uint64_t)z * v->n[1] + y) * v->n[0] + x] = d;
}

/* The sum of the dwells on the box's surface (what a full surface query
 * computes), and of the voxels inside it. */
static void box_work(const vol *v, const box3 *b, uint64_t *surface, uint64_t *inside)
{
    uint64_t s = 0, in = 0;
    for (uint32_t z = b->lo[2]; z < b->hi[2]; ++z)
        for (uint32_t y = b->lo[1]; y < b->hi[1]; ++y)
            for (uint32_t x = b->lo[0]; x < b->hi[0]; ++x) {
                uint32_t d = voxel_dwell(v, x, y, z);
                if (on_surface(b, x, y, z))
                    s += d;
                else
                    in += d;
            }
    *surface = s;
    *inside = in;
}

/* Decide one box: the dwells on its surface all equal -> fill the box with
 * that dwell; otherwise every side <= B -> compute every voxel; otherwise
 * split it into its r^3 child cells (the empty ones dropped). Returns the
 * kind (1 fill, 2 leaf, 3 split). */
static int decide(const vol *v, const box3 *b, uint32_t B, uint32_t *out)
{
    int uniform = 1;
    uint32_t first = voxel_dwell(v, b->lo[0], b->lo[1], b->lo[2]);
    for (uint32_t z = b->lo[2]; z < b->hi[2] && uniform; ++z)
        for (uint32_t y = b->lo[1]; y < b->hi[1] && uniform; ++y)
            for (uint32_t x = b->lo[0]; x < b->hi[0]; ++x)
                if (on_surface(b, x, y, z) && voxel_dwell(v, x, y, z) != first) {
                    uniform = 0;
                    break;
                }
    if (uniform) {
        for (uint32_t z = b->lo[2]; z < b->hi[2]; ++z)
            for (uint32_t y = b->lo[1]; y < b->hi[1]; ++y)
                for (uint32_t x = b->lo[0]; x < b->hi[0]; ++x)
                    put(v, out, x, y, z, first);
        return 1;
    }
    if (b->hi[0] - b->lo[0] <= B && b->hi[1] - b->lo[1] <= B && b->hi[2] - b->lo[2] <= B) {
        for (uint32_t z = b->lo[2]; z < b->hi[2]; ++z)
            for (uint32_t y = b->lo[1]; y < b->hi[1]; ++y)
                for (uint32_t x = b->lo[0]; x < b->hi[0]; ++x)
                    put(v, out, x, y, z, voxel_dwell(v, x, y, z));
        return 2;
    }
    return 3;
}

typedef struct sd_job {
    const vol *v;
    uint32_t *out;
    const uint64_t *olt;
    uint64_t n, next;
    uint64_t G;
    int order;
    uint32_t B;
    uint8_t *kind;
    uint64_t *work;  /* per box: surface iterations, and leaf inside iterations */
    pthread_mutex_t mu;
} sd_job;

static void *sd_worker(void *p)
{
    sd_job *j = (sd_job *)p;
    for (;;) {
        pthread_mutex_lock(&j->mu);
        uint64_t i = j->next++;
        pthread_mutex_unlock(&j->mu);
        if (i >= j->n)
            return NULL;
        uint32_t c[3];
        box3 b;
        decode(j->order, j->G, j->olt[i], c);
        cell_box(j->v, j->G, c, &b);
        j->kind[i] = (uint8_t)decide(j->v, &b, j->B, j->out);
        if (j->work) {
            uint64_t surface, inside;
            box_work(j->v, &b, &surface, &inside);
            j->work[2 * i] = surface;
            j->work[2 * i + 1] = j->kind[i] == 2 ? inside : 0;
        }
    }
}

int64_t askref3_subdiv(const double box[6], uint32_t W, uint32_t H, uint32_t L,
                       double cr, double ci, uint32_t D, uint32_t g, uint32_t r, uint32_t B,
                       int order, uint32_t *out, askref3_stats *st)
{
    if (!vol_ok(W, H, L, D) || g < 1 || r < 2 || B < 1 ||
        (order != ASKREF3_CANONICAL && order != ASKREF3_MORTON))
        return -1;
    vol v;
    askref3_map(box, W, H, L, v.m);
    v.cr = cr, v.ci = ci, v.D = D;
    v.n[0] = W, v.n[1] = H, v.n[2] = L;
    memset(st, 0, sizeof *st);

    /* Level 0: the non-empty cells of the g x g x g grid, in curve order. */
    uint64_t G = g, n = 0, cap = 0;
    uint64_t *olt = NULL;
    for (uint32_t z = 0; z < g; ++z)
        for (uint32_t y = 0; y < g; ++y)
            for (uint32_t x = 0; x < g; ++x) {
                uint32_t p[3] = {x, y, z};
                box3 b;
                if (!cell_box(&v, G, p, &b))
                    continue;
                if (n == cap) {
                    cap = cap ? 2 * cap : 64;
                    olt = realloc(olt, cap * sizeof *olt);
                }
                olt[n++] = encode(order, G, p);
            }
    int nt = threads();
    while (n > 0) {
        if (st->levels >= ASKREF3_MAX_LEVELS || G > (1ull << 21)) {
            free(olt);
            return -2;
        }
        uint32_t lv = st->levels++;
        st->regions[lv] = n;
        uint8_t *kind = calloc(n, 1);
        uint64_t *work = calloc(2 * n, sizeof *work);
        sd_job j = {&v, out, olt, n, 0, G, order, B, kind, work, PTHREAD_MUTEX_INITIALIZER};
        pthread_t th[64];
        for (int t = 0; t < nt; ++t)
            pthread_create(&th[t], NULL, sd_worker, &j);
        for (int t = 0; t < nt; ++t)
            pthread_join(th[t], NULL);
        /* The next level's table: the non-empty children of every split box. */
        uint64_t G1 = G * r, n1 = 0, cap1 = 0;
        uint64_t *olt1 = NULL;
        for (uint64_t i = 0; i < n; ++i) {
            st->iters_surface += work[2 * i];
            st->iters_leaf += work[2 * i + 1];
            if (kind[i] == 1)
                st->fills[lv]++;
            else if (kind[i] == 2)
                st->leaves[lv]++;
            if (kind[i] != 3)
                continue;
            st->splits[lv]++;
            uint32_t c[3];
            decode(order, G, olt[i], c);
            for (uint32_t kz = 0; kz < r; ++kz)
                for (uint32_t ky = 0; ky < r; ++ky)
                    for (uint32_t kx = 0; kx < r; ++kx) {
                        uint32_t p[3] = {c[0] * r + kx, c[1] * r + ky, c[2] * r + kz};
                        box3 b;
                        if (!cell_box(&v, G1, p, &b))
                            continue;
                        if (n1 == cap1) {
                            cap1 = cap1 ? 2 * cap1 : 64;
                            olt1 = realloc(olt1, cap1 * sizeof *olt1);
                        }
                        olt1[n1++] = encode(order, G1, p);
                    }
        }
        free(kind);
        free(work);
        free(olt);
        olt = olt1, n = n1, G = G1;
    }
    free(olt);
    int64_t total = 0;
    for (uint32_t i = 0; i < st->levels; ++i)
        total += (int64_t)st->regions[i];
    return total;
}
