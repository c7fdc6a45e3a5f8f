/* askref3.h -- CPU oracle of the 3-D subdivision (test infrastructure only;
 * see askref3.c). */
#ifndef ASKREF3_H
#define ASKREF3_H

#include <stdint.h>

#define ASKREF3_MAX_LEVELS 32
#define ASKREF3_CANONICAL 0
#define ASKREF3_MORTON 1

typedef struct askref3_stats {
    uint32_t levels, pad_;
    uint64_t regions[ASKREF3_MAX_LEVELS];
    uint64_t fills[ASKREF3_MAX_LEVELS];
    uint64_t splits[ASKREF3_MAX_LEVELS];
    uint64_t leaves[ASKREF3_MAX_LEVELS];
    /* The algorithm's work in dwell iterations: the dwells of every scanned
     * box's whole surface, and of the voxels inside its leaf boxes. */
    uint64_t iters_surface, iters_leaf;
} askref3_stats;

/* box = {x0, x1, y0, y1, z0, z1}; m = {cx, cy, cz, hx, hy, hz}. */
void askref3_map(const double box[6], uint32_t W, uint32_t H, uint32_t L, double m[6]);
uint32_t askref3_dwell(double a, double b, double e, double cr, double ci, uint32_t D);
uint32_t askref3_voxel_dwell(const double box[6], uint32_t W, uint32_t H, uint32_t L,
                             double cr, double ci, uint32_t D,
                             uint32_t px, uint32_t py, uint32_t pz);
/* out: W * H * L voxels, x fastest. 0, or -1 on bad sizes. */
int askref3_exhaustive(const double box[6], uint32_t W, uint32_t H, uint32_t L,
                       double cr, double ci, uint32_t D, uint32_t *out);

uint64_t askref3_canonical(uint64_t G, const uint32_t p[3]);
void askref3_canonical_inv(uint64_t G, uint64_t s, uint32_t p[3]);
uint64_t askref3_morton(const uint32_t p[3]);
void askref3_morton_inv(uint64_t s, uint32_t p[3]);
uint32_t askref3_cell_lo(uint64_t j, uint64_t G, uint32_t n);

/* The subdivision volume; returns the number of boxes processed, -1 on bad
 * arguments, -2 past ASKREF3_MAX_LEVELS levels. */
int64_t askref3_subdiv(const double box[6], uint32_t W, uint32_t H, uint32_t L,
                       double cr, double ci, uint32_t D, uint32_t g, uint32_t r, uint32_t B,
                       int order, uint32_t *out, askref3_stats *st);

#endif
