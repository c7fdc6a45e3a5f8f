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
    double jr, ji;            // julia: the fixed c
    uint32_t W, H, D;
    uint32_t g, r, B;         // initial grid, split factor and stop size
    uint32_t julia;           // 0: the pixel's point is c, z_0 = 0 (Mandelbrot);
                              // 1: the pixel's point is z_0, c = (jr, ji) (filled Julia set)
    uint32_t band;            // queue forms: leaves above band pixels go out as row bands
                              // of about band pixels; others are computed whole
    uint32_t tile_w, tile_h;  // pixel tile of one wave (tile_w * tile_h = 64): the exhaustive
                              // kernel's wave tile; leaf pixels are streamed tile by tile
                              // (tile_w == 0: leaves stream row by row)
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

// Leaf bands of the queue forms, by default: leaves above kLeafTask pixels
// are queued as bands of about kLeafTask pixels, each computed by the wave
// that takes it, so that no wave holds a whole large leaf while others idle.
// An image's band size can be set per render (Image::band).
constexpr uint32_t kLeafTask = ASK_BAND_DEFAULT;

// Launch epoch of persistent renders captured in a graph (whose queue is
// cleared by the graph itself); other renders cycle through 1 .. kGraphEpoch - 1.
constexpr uint32_t kGraphEpoch = 0xffffffu;

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
    unsigned long long ring_px;   // ring sizes summed over scanned regions
    unsigned long long leaf_px;   // pixels of leaf regions
    unsigned long long fill_px;   // pixels of filled regions
    uint32_t levels;
    uint32_t overflow;
};

// Control words in device memory. The counters that every wave updates
// (head, tail, pending) sit on cache lines of their own (128 bytes apart):
// atomics and polls of one line are served one at a time, and sharing a line
// made them the bottleneck of renders with many small regions.
enum Ctrl : uint32_t {
    kCount = 0,                   // [kCount + lv]: regions written for level lv
    kClaim = kCount + kMaxLevels, // [kClaim + lv]: next region a wave takes at level lv
    kHead = 256,                  // persistent queue: next slot to take
    kTail = 288,                  // persistent queue: next slot to fill
    kPending = 320,               // persistent queue: entries queued or taken, not finished
    kOverflow = 352,              // this render: a queue ran out of room
    kRefs = 384,                  // serving: waves holding a reference to the slot
    kSticky = 511,                // error bits of all renders since the last check
    kCtrlWords = 512
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
    Region *queue;              // persistent kernel: the region queue
    uint32_t cap;               // capacity (entries) of out / queue
    uint32_t epoch;
    uint64_t wait_ticks;        // persistent kernel: longest wait, constant-clock ticks
    uint32_t *ctrl;
    DevStats *stats;            // nullptr: do not count
};

// ---------------------------------------------------------------------------
// Serving: one persistent kernel takes regions of any admitted request.
// ---------------------------------------------------------------------------
constexpr uint32_t kMaxSlots = 64;

// Slot state word: gen << 8 | kind. gen (24 bits, never 0 for a request) is
// the request's generation; it tags the request's queue entries, so entries
// left in reused pool memory by earlier requests are never taken for its own.
// A finished request's slot stays kSlotDone until the last wave holding a
// reference to it has left, and only then becomes free for the next request.
enum SlotKind : uint32_t { kSlotFree = 0, kSlotAdmitting = 1, kSlotActive = 2, kSlotDone = 3 };

// What the host posts for a request (pinned host memory).
struct ServerPost {
    Image im;
    uint32_t qoff, qcap;  // the request's region queue: entries [qoff, qoff + qcap) of the pool
};

// What the device reports when a request has finished (pinned host memory);
// gen is written last.
struct ServerDone {
    uint32_t gen;
    int32_t status;
    unsigned long long ticks;  // constant-clock time of completion
};

struct ServerMailbox {
    ServerPost post[kMaxSlots];
    uint32_t doorbell[kMaxSlots];  // generation of the request last posted in each slot
    ServerDone done[kMaxSlots];
    uint32_t stop;                 // nonzero: leave once no request is admitted
};

// A slot's request, in device memory.
struct ServerSlot {
    uint32_t ctrl[kCtrlWords];   // the request's head, tail, pending, error and reference words
    ServerPost post;             // copy of the request's post
};

// Device-wide server words.
struct ServerCtl {
    uint32_t state[kMaxSlots];
    unsigned long long next_poll;  // constant-clock time of the next mailbox poll
    unsigned long long last_busy;  // constant-clock time work was last taken or admitted
    unsigned long long stop_time;  // constant-clock time the stop flag was first seen, or 0
};

struct ServerArgs {
    ServerSlot *slots;
    ServerCtl *ctl;
    uint32_t nslots;
    Region *queue;        // entry pool shared by the requests' queues
    ServerMailbox *mb;    // pinned host memory
    uint64_t wait_ticks;  // longest wait for a claimed entry
    uint64_t poll_ticks;  // mailbox poll interval
    uint64_t idle_ticks;  // the kernel leaves after this long with nothing admitted
};

hipError_t launch_server(const ServerArgs &a, uint32_t grid_blocks, hipStream_t s);
hipError_t occupancy_server(int *blocks_per_cu);

// Up to kWordsPerWrite words of data carried in one kernel's arguments and
// stored at dst (image tables of batches: a captured launch keeps its data).
constexpr uint32_t kWordsPerWrite = 896;
struct WordsArg {
    uint32_t *dst;
    uint32_t n;
    uint32_t words[kWordsPerWrite];
};

// Kernel launchers (ask_kernels.hip). All return hipSuccess or the launch error.
hipError_t launch_write_words(const WordsArg &w, hipStream_t s);
hipError_t launch_exhaustive(const Image &im, hipStream_t s);
hipError_t launch_reset(uint32_t *ctrl, DevStats *stats, hipStream_t s);
hipError_t launch_clear_queue(Region *queue, uint32_t entries, hipStream_t s);
hipError_t launch_seed_levels(const SubdivArgs &a, uint32_t nseeds, hipStream_t s);
hipError_t launch_seed_queue(const SubdivArgs &a, uint32_t nseeds, hipStream_t s);
hipError_t launch_level(const SubdivArgs &a, uint32_t grid_blocks, hipStream_t s);
// Per-level kernel with a workgroup per region, for levels of large regions.
hipError_t launch_level_coop(const SubdivArgs &a, uint32_t grid_blocks, hipStream_t s);
constexpr uint32_t kCoopRingPixels = 512;  // rings of this many pixels or more
hipError_t launch_level_exact(const SubdivArgs &a, uint32_t nregions, hipStream_t s);
hipError_t launch_persistent(const SubdivArgs &a, uint32_t grid_blocks, hipStream_t s);
hipError_t occupancy_level(int *blocks_per_cu);
hipError_t occupancy_persistent(int *blocks_per_cu);

}  // namespace ask
