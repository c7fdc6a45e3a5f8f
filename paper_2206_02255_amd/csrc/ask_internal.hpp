// Internal types shared by the gfx950 kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ask {

constexpr int kWave = 64;
constexpr int kBlock = 256;             // 4 independent waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxLevels = 64;

// Per-image constants, computed on the host (the device never divides).
struct Image {
    double cxm, cym, hx, hy;  // pixel centre = (cxm + (2px+1-W) hx, cym + (2py+1-H) hy)
    uint32_t W, H, D;
    uint32_t g, r, B;         // initial grid, split factor and stop size
    uint32_t *out;            // W*H dwell image, row-major, row 0 on the y0 side
};

// A region of the subdivision, 16 bytes: one entry of the offset lookup
// table / region queue.
struct Region {
    uint32_t img;   // index into the image table
    uint32_t xy;    // x | y << 16
    uint32_t wh;    // (w - 1) | (h - 1) << 16
    uint32_t tag;   // epoch << 8 | kind << 6 | level; in the persistent queue the
                    // tag is stored last, with release order, and marks the entry valid
};

// Entry kinds: a region to scan (border query, then fill, leaf or split), or
// a band of a leaf whose pixels are all computed.
enum Kind : uint32_t { kScan = 0, kLeaf = 1 };

// Pixels per queued leaf task (persistent form).
constexpr uint32_t kLeafTask = 1024;

__host__ __device__ inline uint32_t pack_xy(uint32_t x, uint32_t y) { return x | (y << 16); }
__host__ __device__ inline uint32_t pack_wh(uint32_t w, uint32_t h) { return (w - 1) | ((h - 1) << 16); }

// Device-side work counters (mirrors ask_stats).
struct DevStats {
    unsigned long long regions[kMaxLevels];
    unsigned long long fills[kMaxLevels];
    unsigned long long splits[kMaxLevels];
    unsigned long long leaves[kMaxLevels];
    unsigned long long iters_ring;
    unsigned long long iters_leaf;
    uint32_t levels;
    uint32_t overflow;
};

// Control words in device memory.
enum Ctrl : uint32_t {
    kCount = 0,                   // [kCount + lv]: regions written for level lv
    kClaim = kCount + kMaxLevels, // [kClaim + lv]: next region a wave takes at level lv
    kHead = kClaim + kMaxLevels,  // persistent queue: next slot to take
    kTail,                        // persistent queue: next slot to fill
    kPending,                     // persistent queue: regions taken or queued, not finished
    kOverflow,                    // this render: a queue ran out of room
    kSticky = 255,                // error bits of all renders since the last check
    kCtrlWords = 256
};

enum ErrBits : uint32_t { kErrOverflow = 1, kErrTimeout = 2 };

// Arguments of one subdivision launch.
struct SubdivArgs {
    const Image *table;   // device image table, or nullptr: use `single`
    Image single;
    uint32_t nimg;
    const uint32_t *seed_base;  // batch: prefix sums of g_i^2 (nimg + 1), device
    uint32_t level;             // level kernels: the level being processed
    const Region *in;           // level kernels: regions of this level
    Region *out;                // level kernels: regions of the next level
    Region *queue;              // persistent kernel: the queue
    uint32_t cap;               // capacity (entries) of out / queue
    uint32_t epoch;
    uint64_t wait_ticks;        // persistent kernel: longest wait, constant-clock ticks
    uint32_t *ctrl;
    DevStats *stats;            // nullptr: do not count
};

// Kernel launchers (ask_kernels.hip). All return hipSuccess or the launch error.
hipError_t launch_exhaustive(const Image &im, hipStream_t s);
hipError_t launch_reset(uint32_t *ctrl, DevStats *stats, hipStream_t s);
hipError_t launch_seed_levels(const SubdivArgs &a, uint32_t nseeds, hipStream_t s);
hipError_t launch_seed_queue(const SubdivArgs &a, uint32_t nseeds, hipStream_t s);
hipError_t launch_level(const SubdivArgs &a, uint32_t grid_blocks, hipStream_t s);
hipError_t launch_level_exact(const SubdivArgs &a, uint32_t nregions, hipStream_t s);
hipError_t launch_persistent(const SubdivArgs &a, uint32_t grid_blocks, hipStream_t s);
hipError_t occupancy_level(int *blocks_per_cu);
hipError_t occupancy_persistent(int *blocks_per_cu);

}  // namespace ask
