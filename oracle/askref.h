/*
 * askref.h -- CPU oracle for the Mandelbrot dwell image and its
 * Mariani-Silver subdivision image, and the same images of filled Julia sets.
 *
 * TEST INFRASTRUCTURE. This is the independent checker of the GPU library:
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it. It shares no source, header, table or constant with the
 * GPU path, and the GPU path never calls it.
 *
 * Arithmetic is IEEE-754 binary64, round to nearest even, one rounding per
 * operation: the file is compiled with -ffp-contract=off and without any
 * fast-math option, so no multiply-add is ever fused and nothing is
 * reassociated.
 *
 * Paper: Quezada, Navarro, Romero, Aguilera, "Modeling GPU Dynamic
 * Parallelism for Self Similar Density Workloads" (arXiv 2206.02255).
 */
#ifndef ASKREF_H
#define ASKREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASKREF_MAX_LEVELS 64

/* Per-run statistics of a subdivision image (Sec. 4.2 work terms). */
typedef struct askref_stats {
    uint32_t levels;                       /* deepest level reached + 1 */
    uint32_t pad_;
    uint64_t regions[ASKREF_MAX_LEVELS];   /* regions scanned at each level */
    uint64_t fills[ASKREF_MAX_LEVELS];     /* uniform ring -> filled */
    uint64_t splits[ASKREF_MAX_LEVELS];    /* mixed ring, larger than B -> split */
    uint64_t leaves[ASKREF_MAX_LEVELS];    /* mixed ring, within B -> per pixel */
    uint64_t ring_px;                      /* sum of ring sizes over scanned regions */
    uint64_t leaf_px;                      /* pixels of leaf regions */
    uint64_t fill_px;                      /* pixels of filled regions */
    uint64_t iters_ring;                   /* sum of dwell over every scanned ring pixel */
    uint64_t iters_leaf;                   /* sum of dwell over every leaf pixel */
    uint64_t iters_ring_new;               /* ring pixels that are not on the parent's ring */
    uint64_t iters_leaf_inner;             /* leaf pixels that are not on the leaf's own ring */
    uint64_t iters_ring_filled;            /* sum of dwell over the rings of filled regions */
} askref_stats;

/* One scanned region, for invariant checks. kind: 1 fill, 2 leaf, 3 split. */
typedef struct askref_region {
    uint32_t x, y, w, h;
    uint32_t level, kind, value, pad_;
} askref_region;

/* The escape-time set a window's points are iterated in. julia == 0: the
 * Mandelbrot set, the pixel's point is c and z_0 = 0 (cr, ci unused).
 * julia == 1: the filled Julia set of the fixed c = cr + i ci, the pixel's
 * point is z_0. A NULL set means the Mandelbrot set. */
typedef struct askref_set {
    uint32_t julia;
    uint32_t pad_;
    double cr, ci;
} askref_set;

/* Pixel-centre mapping constants {cxm, cym, hx, hy} of a window. */
void askref_map(double x0, double x1, double y0, double y1,
                uint32_t W, uint32_t H, double m[4]);

/* c of pixel (px, py): centre-relative, row 0 on the y0 side. */
void askref_pixel_c(const double m[4], uint32_t W, uint32_t H,
                    uint32_t px, uint32_t py, double *cr, double *ci);

/* Dwell of c: first k >= 1 with |z_k|^2 > 4 for z_0 = 0, z_k = z_{k-1}^2 + c;
 * D if there is none. */
uint32_t askref_dwell(double cr, double ci, uint32_t D);

/* Dwell of z0 in the filled Julia set of c: first k >= 1 with |z_k|^2 > 4
 * for z_k = z_{k-1}^2 + c; D if there is none. askref_dwell(cr, ci, D) is
 * askref_dwell_julia(0, 0, cr, ci, D). */
uint32_t askref_dwell_julia(double zr0, double zi0, double cr, double ci, uint32_t D);

/* Exhaustive image: out[py*W + px] = dwell(c(px, py)). Returns 0, or -1 on a
 * bad argument. iters_out (may be NULL) receives the sum of all dwells.
 * threads <= 0 means one per online CPU. */
int askref_exhaustive(double x0, double x1, double y0, double y1,
                      uint32_t W, uint32_t H, uint32_t D,
                      uint32_t *out, uint64_t *iters_out, int threads);

/* Mariani-Silver subdivision image (level-by-level when order == 0, depth
 * first when order == 1). stats and recs may be NULL. When recs is given, up
 * to rec_cap scanned regions are stored, in no particular order; the return
 * value is then the number of scanned regions (which may exceed rec_cap).
 * Returns -1 on a bad argument. */
int64_t askref_subdiv(double x0, double x1, double y0, double y1,
                      uint32_t W, uint32_t H, uint32_t D,
                      uint32_t g, uint32_t r, uint32_t B, int order, int threads,
                      uint32_t *out, askref_stats *stats,
                      askref_region *recs, uint64_t rec_cap);

/* Subdivision-image values at n sampled pixels, each found by walking down
 * the region tree from the level-0 region that holds it. Returns 0 or -1. */
int askref_subdiv_pixels(double x0, double x1, double y0, double y1,
                         uint32_t W, uint32_t H, uint32_t D,
                         uint32_t g, uint32_t r, uint32_t B,
                         uint64_t n, const uint32_t *px, const uint32_t *py,
                         uint32_t *out);

/* Exhaustive-image values at n sampled pixels. */
void askref_dwell_pixels(double x0, double x1, double y0, double y1,
                         uint32_t W, uint32_t H, uint32_t D, uint64_t n,
                         const uint32_t *px, const uint32_t *py, uint32_t *out);

/* The same four images for a window of the given set (NULL: Mandelbrot). */
int askref_exhaustive_set(double x0, double x1, double y0, double y1,
                          uint32_t W, uint32_t H, uint32_t D, const askref_set *set,
                          uint32_t *out, uint64_t *iters_out, int threads);
int64_t askref_subdiv_set(double x0, double x1, double y0, double y1,
                          uint32_t W, uint32_t H, uint32_t D, const askref_set *set,
                          uint32_t g, uint32_t r, uint32_t B, int order, int threads,
                          uint32_t *out, askref_stats *stats,
                          askref_region *recs, uint64_t rec_cap);
int askref_subdiv_pixels_set(double x0, double x1, double y0, double y1,
                             uint32_t W, uint32_t H, uint32_t D, const askref_set *set,
                             uint32_t g, uint32_t r, uint32_t B,
                             uint64_t n, const uint32_t *px, const uint32_t *py,
                             uint32_t *out);
void askref_dwell_pixels_set(double x0, double x1, double y0, double y1,
                             uint32_t W, uint32_t H, uint32_t D, const askref_set *set,
                             uint64_t n, const uint32_t *px, const uint32_t *py, uint32_t *out);

#ifdef __cplusplus
}
#endif
#endif
