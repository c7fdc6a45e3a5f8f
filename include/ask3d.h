/* ask3d.h -- the 3-D extension of adaptive subdivision (the paper's section
 * on subdivisions at higher dimensions, k = 3): a dwell volume over a box of
 * points, rendered exhaustively or by Mariani-Silver subdivision over boxes
 * (3-orthotopes), level by level, each level's table holding one
 * space-filling-curve scalar per box (the compact table of that section).
 *
 * The volume: voxel (px, py, pz) of a W x H x L grid over the box
 * [x0, x1] x [y0, y1] x [z0, z1] stands for the point at the voxel centre,
 * per axis centre + (2p + 1 - n) * half pitch, half pitch = extent / (2n).
 * Its dwell is the escape time of the quaternion Julia iteration
 * q <- q^2 + c from q0 = x + y i + z j, c = cr + ci i: the first k >= 1 with
 * |q_k|^2 > 4, else D, every binary64 operation rounded on its own (no fused
 * multiply-add). The z = 0 slice is the filled Julia image of the complex c
 * (ask.h, ASK_SET_JULIA), bit for bit.
 *
 * Subdivision: level i's grid has G_i = g r^i cells per axis; cell j of an
 * axis of n voxels spans [floor(j n / G_i), floor((j + 1) n / G_i)), so the
 * r^3 cells of level i + 1 below a cell of level i tile it exactly and a box
 * is named by its level and the scalar of its cell on the chosen curve. A
 * box whose surface voxels all have one dwell is filled with it; else, when
 * every side is at most B, every voxel is computed; else its r^3 child cells
 * (empty ones dropped) go to the next level's table.
 *
 * Volumes are stored x fastest, then y, then z: voxel (px, py, pz) at
 * (pz * H + py) * W + px. All entry points are asynchronous on `stream`
 * (a hipStream_t, NULL for the null stream) unless stated otherwise, and
 * return ASK_EINVAL, without launching anything, on invalid arguments.
 */
#ifndef ASK3D_H
#define ASK3D_H

#include <stdint.h>

#include "ask.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { ASK_CURVE_CANONICAL = 0, ASK_CURVE_MORTON = 1 };
#define ASK3_MAX_LEVELS 32u

/* The box of points, the voxel counts (each 1..65536, W * H * L <= 2^31), the
 * maximum dwell D >= 1 and the constant c (finite). 80 bytes. */
typedef struct ask_volume {
    double x0, x1, y0, y1, z0, z1;
    uint32_t W, H, L, D;
    double cr, ci;
} ask_volume;

/* g >= 1 level-0 cells per axis, r >= 2 (r^3 <= 4096) children per axis,
 * B >= 1 the largest leaf side, curve: ASK_CURVE_CANONICAL (x fastest, then
 * y, then z) or ASK_CURVE_MORTON (bit t of the cell's x, y, z coordinates
 * at bits 3t, 3t + 1, 3t + 2; needs every level's G_i <= 2^21). The levels
 * the render can reach (the first level whose cells all have sides <= B)
 * must number at most ASK3_MAX_LEVELS. */
typedef struct ask3_params {
    uint32_t g, r, B, curve;
} ask3_params;

/* Per-level counts of boxes taken from the level's table, filled, split and
 * computed voxel by voxel; `levels` counts the levels with boxes; overflow
 * != 0 when a table ran out of room (the volume is then invalid). */
typedef struct ask3_stats {
    uint32_t levels, overflow;
    uint64_t regions[ASK3_MAX_LEVELS];
    uint64_t fills[ASK3_MAX_LEVELS];
    uint64_t splits[ASK3_MAX_LEVELS];
    uint64_t leaves[ASK3_MAX_LEVELS];
} ask3_stats;

/* ASK_OK when the volume (and the parameters, unless NULL) are valid. */
ask_status ask3_validate(const ask_volume *v, const ask3_params *p);

/* Bytes of device workspace ask3_dwell_subdiv needs for this volume and
 * these parameters: a 36 KiB control block and two level tables of
 * min(W H L, max(level-0 cells, r^3 floor(W H L / (B + 1)))) 8-byte entries
 * each (a split box has a side > B, so at least B + 1 voxels). */
ask_status ask3_workspace_bytes(const ask_volume *v, const ask3_params *p, uint64_t *bytes);

/* Device workspace of ask3_dwell_exhaustive: the counters through which its
 * waves claim columns of voxels. */
#define ASK3_EXHAUSTIVE_WORK_BYTES 1024u

/* Exhaustive volume: every voxel's dwell into d_out (device memory,
 * W * H * L uint32, caller-owned). d_work: device memory of at least
 * ASK3_EXHAUSTIVE_WORK_BYTES bytes, 256-byte aligned, caller-owned, not used
 * by another call until this one has finished on `stream` (the call clears
 * it first). No allocation and no host synchronisation. Errors: ASK_EINVAL
 * (volume, buffers), ASK_EDEVICE (no current device, or a launch failed). */
ask_status ask3_dwell_exhaustive(const ask_volume *v, uint32_t *d_out, void *d_work,
                                 uint64_t work_bytes, void *stream);

/* Subdivision volume into d_out (as above). d_work: device memory of at
 * least ask3_workspace_bytes bytes, 256-byte aligned, caller-owned, not
 * used by another call until this render has finished on `stream`. No
 * allocation and no host synchronisation, unless `stats` is non-NULL: then
 * the call waits for the render and fills it (ASK_EOVERFLOW if a table ran
 * out of room). */
ask_status ask3_dwell_subdiv(const ask_volume *v, const ask3_params *p, uint32_t *d_out,
                             void *d_work, uint64_t work_bytes, void *stream,
                             ask3_stats *stats);

#ifdef __cplusplus
}
#endif

#endif
