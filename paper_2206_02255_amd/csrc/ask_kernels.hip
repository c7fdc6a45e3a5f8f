// gfx950 kernels: the dwell core, the exhaustive image, and the subdivision
// (Mariani-Silver) kernels in their per-level and persistent forms.
//
// Every floating-point operation of the dwell is a separate binary64 add or
// multiply: the file is compiled with -ffp-contract=off and also forbids
// contraction below, so no v_fma_f64 can appear and the images equal those of
// the binary64 definition bit for bit.
#pragma clang fp contract(off)

#include "ask.h"
#include "ask_internal.hpp"

namespace ask {

// ---------------------------------------------------------------------------
// Pixel -> c (the host computed cxm, cym, hx, hy; the device never divides).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pixel_c(const Image &im, uint32_t px, uint32_t py,
                                        double &cr, double &ci) {
    const int kx = 2 * (int)px + 1 - (int)im.W;   // odd, |kx| < 2^17: exact
    const int ky = 2 * (int)py + 1 - (int)im.H;
    const double tx = (double)kx * im.hx;
    const double ty = (double)ky * im.hy;
    cr = im.cxm + tx;
    ci = im.cym + ty;
}

// The orbit start of pixel (px, py): z_0 and c. Mandelbrot set: z_0 = 0 and
// c is the pixel's point; filled Julia set: z_0 is the pixel's point and c
// the image's fixed constant.
__device__ __forceinline__ void pixel_orbit(const Image &im, uint32_t px, uint32_t py,
                                            double &zr, double &zi, double &cr, double &ci) {
    double pr, pi;
    pixel_c(im, px, py, pr, pi);
    zr = im.julia ? pr : 0.0;
    zi = im.julia ? pi : 0.0;
    cr = im.julia ? im.jr : pr;
    ci = im.julia ? im.ji : pi;
}

// ---------------------------------------------------------------------------
// Dwell (Sec. 6): first k >= 1 with |z_k|^2 > 4, z_0 = 0, z_k = z_{k-1}^2 + c,
// or D. One iteration is 3 multiplies and 4 adds, and the test reuses the
// squares of the new z, which the next iteration needs anyway.
// ---------------------------------------------------------------------------

// Continue from the state after k iterations, testing after every iteration.
__device__ __forceinline__ uint32_t dwell_from(double cr, double ci, uint32_t D, uint32_t k,
                                               double zr, double zi, double zr2, double zi2) {
    while (k < D) {
        ++k;
        const double zri = zr * zi;
        zr = (zr2 - zi2) + cr;
        zi = (zri + zri) + ci;
        zr2 = zr * zr;
        zi2 = zi * zi;
        if (zr2 + zi2 > 4.0)
            return k;
    }
    return D;
}

// Iterations between escape tests in the fast loop.
constexpr uint32_t kStride = 16;
// Steps tested one by one when a lane takes a Julia-set pixel.
constexpr uint32_t kRefillSteps = 3;

// The fast loop runs kStride iterations without testing and then tests
// !(|z|^2 <= 4), which also catches inf and NaN. When |c|^2 <= 3.99, once
// |z_k|^2 > 4 has been seen the orbit grows strictly at every later step
// (|z'| >= |z|^2 - |c| minus rounding, with 2 - |c| far above the rounding),
// so a passing test at the end of a stretch proves that no escape happened
// inside it. A failing test restarts the stretch from its saved start with a
// test after every iteration, which finds the same first k as the plain loop.
// Other c (|c| near or above 2, NaN) take the plain loop from the start.
// The orbit starts at z_0 = (zr, zi): 0 for the Mandelbrot set, the pixel's
// point for a filled Julia set; the growth argument does not depend on z_0.
__device__ __forceinline__ uint32_t dwell(double zr, double zi, double cr, double ci, uint32_t D) {
    double zr2 = zr * zr, zi2 = zi * zi;
    uint32_t k = 0;
    if (cr * cr + ci * ci <= 3.99) {
        while (k + kStride <= D) {
            const double szr = zr, szi = zi, szr2 = zr2, szi2 = zi2;
#pragma unroll
            for (uint32_t u = 0; u < kStride; ++u) {
                const double zri = zr * zi;
                zr = (zr2 - zi2) + cr;
                zi = (zri + zri) + ci;
                zr2 = zr * zr;
                zi2 = zi * zi;
            }
            if (!(zr2 + zi2 <= 4.0)) {
                zr = szr;
                zi = szi;
                zr2 = szr2;
                zi2 = szi2;
                break;
            }
            k += kStride;
        }
    }
    return dwell_from(cr, ci, D, k, zr, zi, zr2, zi2);
}

// ---------------------------------------------------------------------------
// Wave helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = min(v, (uint32_t)__shfl_xor((unsigned int)v, o));
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, (uint32_t)__shfl_xor((unsigned int)v, o));
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ uint32_t lane_rank(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Wave-wide values are made uniform with readfirstlane (the value of the
// first active lane), never by branching on the lane index: a branch such as
// `if (lane == 0)` ahead of a broadcast lets the optimiser route the other
// lanes around it, and the broadcast then runs with the source lane missing.
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ bool first_lane() {
    const uint32_t lane = __lane_id();
    return lane == uniform(lane);
}

// The constant-rate clock (100 MHz on gfx950), one value for the wave.
__device__ __forceinline__ unsigned long long clock_now() {
    const unsigned long long t = __builtin_amdgcn_s_memrealtime();
    return ((unsigned long long)uniform((uint32_t)(t >> 32)) << 32) | uniform((uint32_t)t);
}

// One atomic per wave, issued by the first active lane alone; every lane
// gets the old value through readfirstlane (which reads that same lane, also
// if the optimiser moves it into the branch).
__device__ __forceinline__ uint32_t wave_add(uint32_t *p, uint32_t v) {
    uint32_t old = 0;
    if (first_lane())
        old = atomicAdd(p, v);
    return uniform(old);
}

__device__ __forceinline__ void wave_add64(unsigned long long *p, unsigned long long v) {
    if (first_lane())
        atomicAdd(p, v);
}

__device__ __forceinline__ void wave_or(uint32_t *p, uint32_t v) {
    if (first_lane())
        atomicOr(p, v);
}

__device__ __forceinline__ void wave_max(uint32_t *p, uint32_t v) {
    if (first_lane())
        atomicMax(p, v);
}

// A dwell written to the image in device memory with a global store. Through
// a generic pointer the store would be a flat one, which also counts on the
// counter of scalar and LDS operations: every later wait on those (a scalar
// load, a lane permute) would then also wait for the store to complete.
__device__ __forceinline__ void put_pixel(uint32_t *out, size_t i, uint32_t d) {
    ((__attribute__((address_space(1))) uint32_t *)out)[i] = d;
}

// The subdivision kernels write the image through to memory (a relaxed
// device-scope store, which leaves no dirty line in the XCD's L2). A wave
// that publishes queue entries makes its earlier writes visible device-wide
// first, and on MI355X that writes back every dirty line of its XCD's L2;
// with the image written through, that write-back has almost nothing to do
// (the 16384^2 render went from 4.33 to 3.98 ms).
__device__ __forceinline__ void put_dwell(uint32_t *out, size_t i, uint32_t d) {
    __hip_atomic_store(out + i, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Exhaustive image (Sec. 4.1): one lane per pixel. Each wave owns a tile of
// kTileW x (64 / kTileW) pixels, and a 256-lane workgroup four such tiles
// stacked vertically (the default 16 x 4 wave tile makes 16 x 16 workgroup
// tiles, the paper's best block for this kernel).
// ---------------------------------------------------------------------------
template <uint32_t kTileW>
__global__ __launch_bounds__(kBlock) void exhaustive_kernel(Image im) {
    constexpr uint32_t kTileH = kWave / kTileW;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    const uint32_t px = blockIdx.x * kTileW + (lane % kTileW);
    const uint32_t py = (blockIdx.y * kWavesPerBlock + wave) * kTileH + lane / kTileW;
    if (px >= im.W || py >= im.H)
        return;
    double zr, zi, cr, ci;
    pixel_orbit(im, px, py, zr, zi, cr, ci);
    put_pixel(im.out, (size_t)py * im.W + px, dwell(zr, zi, cr, ci, im.D));
}


// ---------------------------------------------------------------------------
// Dwell of a stream of pixels with lane refill (border and leaf work).
//
// Border and leaf pixels lie on the set boundary, where neighbouring dwells
// differ by orders of magnitude, so a wave that gives each lane one pixel
// waits for its slowest pixel with most lanes idle. Here every lane iterates
// its own pixel, and at each round boundary (kRoundBlocks stretches of
// kStride iterations) every lane whose pixel has finished takes the next
// pixel of the stream.
//
// Each stretch is the fast loop of dwell(): kStride iterations without a
// test, then !(|z|^2 <= 4); a failing test restarts the stretch from its
// saved start with a test after every iteration. Lanes with |c|^2 > 3.99 (or
// NaN) test after every iteration throughout. Iterations past D are
// harmless: an escape after D, or none by D, both give D, so D is checked
// once per round.
//
// pixel_of(i, px, py) names pixel i of the stream (false: no pixel there);
// done(px, py, dwell, ring) is called by the lane that finished a pixel,
// ring telling whether it was one of the first n_ring stream positions.
//
// A leaf stream (kRing false) computes positions [0, n_all). A ring stream
// (kRing true) takes the border first, positions [0, n_ring), and decides
// uniformity as it goes, so that it can stop as soon as the border is known
// to be mixed: once some pixel has finished with dwell v (the least dwell of
// the first round in which any pixel finished), the border is mixed if
// another pixel finishes with a different dwell, or if a pixel still running
// has already done v iterations (its dwell is larger than v). The decision
// is the one the whole border would give.
//   - n_all == n_ring: the stream stops there; `partial` receives, per lane,
//     the iterations of a pixel left unfinished (work done, for counters).
//   - n_all > n_ring (a leaf-size region whose wave computes the leaf): the
//     stream goes on after a mixed decision with the border's remaining
//     positions and then positions [n_ring, n_all), the leaf's inside, so no
//     finished border dwell is recomputed and no lane's work is dropped.
// Returns kUniform for a border whose every pixel finished with v, kMixed
// for a mixed border that stopped, kLeafDone for a mixed border whose leaf
// the stream then completed (and kLeafDone for leaf streams).
// ---------------------------------------------------------------------------
constexpr uint32_t kRoundBlocks = 4;

enum StreamEnd : uint32_t { kUniform = 0, kMixed = 1, kLeafDone = 2 };

// The ring decision of one wave alone: v is the wave's own.
struct SoloDecision {
    __device__ uint32_t propose(uint32_t x) const { return x; }
    __device__ bool known(uint32_t &) const { return false; }
    __device__ bool mixed() const { return false; }
    __device__ void set_mixed() const {}
};

template <bool kRing, class PixelOf, class Done, class Decision = SoloDecision>
__device__ __forceinline__ uint32_t dwell_stream(const Image &im, uint32_t n_ring, uint32_t n_all,
                                                 PixelOf pixel_of, Done done, uint32_t &v,
                                                 uint32_t &partial, Decision dec = Decision{}) {
    const uint32_t D = im.D;
    uint32_t next = 0;  // first stream index no lane has taken yet (uniform)
    uint32_t n = kRing ? n_ring : n_all;  // end of the stream as far as it is known to run
    bool scanning = kRing;                // the border's uniformity is still undecided
    bool have = false, special = false, vset = false, ring = false;
    uint32_t px = 0, py = 0, kbase = 0;
    double cr = 0.0, ci = 0.0, zr = 0.0, zi = 0.0, zr2 = 0.0, zi2 = 0.0;
    partial = 0;
    for (;;) {
        // Idle lanes take the next stream positions; a position that names no
        // pixel is passed over, so this repeats until no lane is idle or the
        // stream is exhausted.
        unsigned long long idle = __ballot(!have);
        uint32_t rlo = 0xffffffffu, rhi = 0u;  // dwells of the pixels this lane finished here
        while (idle && next < n) {
            if (!have) {
                const uint32_t j = next + lane_rank(idle);
                if (j < n && pixel_of(j, px, py)) {
                    have = true;
                    ring = kRing && j < n_ring;
                    pixel_orbit(im, px, py, zr, zi, cr, ci);
                    special = !(cr * cr + ci * ci <= 3.99);
                    zr2 = zr * zr;
                    zi2 = zi * zi;
                    kbase = 0;
                    if (im.julia) {
                        // A Julia set's pixels start on the orbit, and many
                        // escape within a few steps: those steps are tested
                        // here, and such a lane takes its next pixel at once.
                        bool out = false;
#pragma unroll 1
                        for (uint32_t t = 0; t < kRefillSteps && !out && kbase < D; ++t) {
                            const double zri = zr * zi;
                            zr = (zr2 - zi2) + cr;
                            zi = (zri + zri) + ci;
                            zr2 = zr * zr;
                            zi2 = zi * zi;
                            ++kbase;
                            out = zr2 + zi2 > 4.0;
                        }
                        if (out || kbase >= D) {
                            done(px, py, kbase, ring);
                            have = false;
                            rlo = min(rlo, kbase);
                            rhi = max(rhi, kbase);
                        }
                    }
                }
            }
            next = min(n, next + (uint32_t)__popcll(idle));
            idle = __ballot(!have);
        }
        // A ring pixel finished here has a dwell of at most kRefillSteps (or
        // D, and then every pixel finishes here), below that of any pixel
        // still running: the least of them sets v when none is set yet, and
        // then a pixel still running, or one finished here with another
        // dwell, shows a mixed ring.
        if (kRing && scanning && __ballot(rhi != 0)) {
            const uint32_t lo = uniform(wave_min(rlo));
            const uint32_t hi = uniform(wave_max(rhi));
            if (!vset) {
                v = dec.propose(lo);
                vset = true;
            }
            if (lo != v || hi != v || __ballot(have) || dec.mixed()) {
                dec.set_mixed();
                if (n_all == n_ring) {
                    partial = have ? kbase : 0u;
                    return kMixed;
                }
                scanning = false;  // mixed: go on as the leaf
                n = n_all;
                continue;
            }
        }
        if (__ballot(have) == 0)
            break;
        uint32_t dw = 0;
        bool fin = false;
        if (have) {
            // A lane whose pixel escapes inside a stretch goes back to the
            // stretch's start and leaves the loop; the replay that finds the
            // first k follows the loop, once per round for all such lanes
            // rather than once in every stretch in which some lane escaped.
            bool replay = false;
            for (uint32_t bi = 0; bi < kRoundBlocks && !fin && !replay; ++bi) {
                if (__builtin_expect(!special, 1)) {
                    const double szr = zr, szi = zi, szr2 = zr2, szi2 = zi2;
#pragma unroll
                    for (uint32_t u = 0; u < kStride; ++u) {
                        const double zri = zr * zi;
                        zr = (zr2 - zi2) + cr;
                        zi = (zri + zri) + ci;
                        zr2 = zr * zr;
                        zi2 = zi * zi;
                    }
                    if (!(zr2 + zi2 <= 4.0)) {
                        // Escapes are rare: an empty asm keeps the restore
                        // on a branch, so the common stretch does not pay
                        // a select per register of the state.
                        asm volatile("");
                        zr = szr;
                        zi = szi;
                        zr2 = szr2;
                        zi2 = szi2;
                        replay = true;
                    } else {
                        kbase += kStride;
                    }
                } else {
                    // Kept rolled: unrolled, its sixteen exits hold enough
                    // scalar registers to spill in the common path too.
#pragma unroll 1
                    for (uint32_t u = 0; u < kStride; ++u) {
                        const double zri = zr * zi;
                        zr = (zr2 - zi2) + cr;
                        zi = (zri + zri) + ci;
                        zr2 = zr * zr;
                        zi2 = zi * zi;
                        if (zr2 + zi2 > 4.0) {
                            dw = kbase + u + 1;
                            fin = true;
                            break;
                        }
                    }
                    if (!fin)
                        kbase += kStride;
                }
            }
            if (replay) {
                dw = dwell_from(cr, ci, D, kbase, zr, zi, zr2, zi2);
                fin = true;
            }
            if (!fin && kbase >= D) {
                dw = D;
                fin = true;
            }
            if (fin) {
                dw = dw > D ? D : dw;
                done(px, py, dw, ring);
                have = false;
            }
        }
        if (kRing && scanning) {
            if (!vset && dec.known(v))
                vset = true;
            if (!vset && __ballot(fin)) {
                v = dec.propose(uniform(wave_min(fin ? dw : 0xffffffffu)));
                vset = true;
            }
            if ((vset && __ballot((fin && dw != v) || (have && kbase >= v))) || dec.mixed()) {
                dec.set_mixed();
                if (n_all == n_ring) {
                    partial = have ? kbase : 0u;
                    return kMixed;
                }
                scanning = false;  // mixed: go on as the leaf
                n = n_all;
            }
        }
    }
    return (kRing && scanning) ? kUniform : kLeafDone;
}

// ---------------------------------------------------------------------------
// Subdivision: one wave owns one region (the single-block-per-region scheme
// of Sec. 4.3.1 with a wave64 as the block).
// ---------------------------------------------------------------------------

// The i-th pixel of the ring of [x, x+w) x [y, y+h): first row, last row,
// then the first and last column between them.
__device__ __forceinline__ void ring_pixel(uint32_t x, uint32_t y, uint32_t w, uint32_t h,
                                           uint32_t i, uint32_t &px, uint32_t &py) {
    if (h == 1) {
        px = x + i;
        py = y;
    } else if (w == 1) {
        px = x;
        py = y + i;
    } else if (i < w) {
        px = x + i;
        py = y;
    } else if (i < 2 * w) {
        px = x + (i - w);
        py = y + h - 1;
    } else {
        const uint32_t j = i - 2 * w;
        const uint32_t side = h - 2;
        if (j < side) {
            px = x;
            py = y + 1 + j;
        } else {
            px = x + w - 1;
            py = y + 1 + (j - side);
        }
    }
}

__device__ __forceinline__ uint32_t ring_size(uint32_t w, uint32_t h) {
    return (w == 1 || h == 1) ? w * h : 2 * (w + h) - 4;
}

// Terminal work T: write v on every pixel of the region. Rows of 64 or more
// pixels are written row by row, narrower regions several rows per pass.
__device__ void fill_region(uint32_t *out, uint32_t W, uint32_t x, uint32_t y, uint32_t w,
                            uint32_t h, uint32_t v, uint32_t lane, uint32_t part = 0,
                            uint32_t parts = 1) {
    if (w >= kWave) {
        for (uint32_t row = part; row < h; row += parts) {
            uint32_t *p = out + (size_t)(y + row) * W + x;
            for (uint32_t c = lane; c < w; c += kWave)
                put_dwell(p, c, v);
        }
    } else {
        const uint32_t per = kWave / w;
        const uint32_t lr = lane / w, lc = lane - lr * w;
        if (lr < per)
            for (uint32_t row = lr + part * per; row < h; row += per * parts)
                put_dwell(out, (size_t)(y + row) * W + x + lc, v);
    }
}

// Pixel order of a rectangle [x, x+w) x [y, y+h) as a stream: row-major, or
// tile by tile when the image sets a wave tile (tiles of tile_w x tile_h
// pixels in row-major order over the rectangle, pixels row-major within a
// tile, positions beyond the rectangle's right or bottom edge passed over).
struct RectOrder {
    uint32_t x, y, w, h, tw, sh, th, ntx;
    __device__ RectOrder(const Image &im, uint32_t x_, uint32_t y_, uint32_t w_, uint32_t h_)
        : x(x_), y(y_), w(w_), h(h_), tw(im.tile_w),
          sh(im.tile_w ? (uint32_t)__builtin_ctz(im.tile_w) : 0u),
          th(im.tile_w ? (kWave >> sh) : 1u), ntx(im.tile_w ? (w_ + im.tile_w - 1) >> sh : 1u) {}
    // Stream positions (pixels, and passed-over positions of partial tiles).
    __device__ uint32_t positions() const {
        return tw ? ntx * ((h + th - 1) / th) * kWave : w * h;
    }
    __device__ bool pixel(uint32_t i, uint32_t &px, uint32_t &py) const {
        if (tw == 0) {
            const uint32_t row = i / w;
            px = x + (i - row * w);
            py = y + row;
            return true;
        }
        const uint32_t t = i / kWave, p = i % kWave;
        const uint32_t ty = t / ntx, tx = t - ty * ntx;
        const uint32_t cx = (tx << sh) + (p & (tw - 1)), cy = ty * th + (p >> sh);
        px = x + cx;
        py = y + cy;
        return cx < w && cy < h;
    }
};

// Last-level work L for a band of a leaf: the dwell of every pixel of the
// rectangle as one refilled stream.
__device__ unsigned long long leaf_region(const Image &im, uint32_t x, uint32_t y, uint32_t w,
                                          uint32_t h) {
    unsigned long long it = 0;
    uint32_t v, partial;
    const RectOrder order(im, x, y, w, h);
    dwell_stream<false>(
        im, 0u, order.positions(),
        [&](uint32_t i, uint32_t &px, uint32_t &py) { return order.pixel(i, px, py); },
        [&](uint32_t px, uint32_t py, uint32_t d, bool) {
            put_dwell(im.out, (size_t)py * im.W + px, d);
            it += d;
        },
        v, partial);
    return it;
}

// The image table is written before a launch and never by a kernel, so it is
// read with scalar loads (constant address space): the image's fields live in
// scalar registers, and no wait inside the pixel loops has to cover them.
__device__ __forceinline__ Image image_of(const SubdivArgs &a, uint32_t img) {
    if (a.table) {
        const __attribute__((address_space(4))) Image &t =
            ((const __attribute__((address_space(4))) Image *)a.table)[img];
        Image im;
        im.cxm = t.cxm;
        im.cym = t.cym;
        im.hx = t.hx;
        im.hy = t.hy;
        im.W = t.W;
        im.H = t.H;
        im.D = t.D;
        im.g = t.g;
        im.r = t.r;
        im.B = t.B;
        im.jr = t.jr;
        im.ji = t.ji;
        im.julia = t.julia;
        im.band = t.band;
        im.tile_w = t.tile_w;
        im.tile_h = t.tile_h;
        im.out = t.out;
        return im;
    }
    return a.single;
}

// Append `count` entries (entry_of(j, e) fills e's img, xy and wh, or
// returns false for an empty one) to table q, whose next free slot is *tail
// and whose capacity is cap: the next level's table (per-level form) or a
// queue (persistent forms), with the given kind and level, using one atomic
// add per wave and per 64 entries: a ballot of the non-empty entries and
// their rank give every entry its slot (Sec. 5.3.1, compact insertion).
// Queue entries are counted as pending and published by their tag.
template <bool kQueue, class EntryOf>
__device__ void emit_entries(const SubdivArgs &a, Region *q, uint32_t *tail, uint32_t cap,
                             uint32_t count, uint32_t kind, uint32_t level, uint32_t lane,
                             EntryOf entry_of) {
    const uint32_t tag = (a.epoch << 8) | (kind << 6) | level;
    for (uint32_t base = 0; base < count; base += kWave) {
        const uint32_t j = base + lane;
        Region e{0, 0, 0, tag};
        const bool ok = j < count && entry_of(j, e);
        const unsigned long long mask = __ballot(ok);
        const uint32_t n = (uint32_t)__popcll(mask);
        if (n == 0)
            continue;
        const uint32_t slot0 = wave_add(tail, n);
        const bool fits = (uint64_t)slot0 + n <= cap;
        if (fits) {
            if (kQueue)
                wave_add(&a.ctrl[kPending], n);
        } else {
            wave_or(&a.ctrl[kOverflow], 1u);
            wave_or(&a.ctrl[kSticky], kErrOverflow);
        }
        if (ok && fits) {
            Region *d = q + slot0 + lane_rank(mask);
            if (kQueue) {
                d->img = e.img;
                d->xy = e.xy;
                d->wh = e.wh;
                __hip_atomic_store(&d->tag, tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                *d = e;
            }
        }
    }
}

// S: the non-empty pieces of the r x r floor partition of the region become
// regions of the next level.
template <bool kQueue>
__device__ void split_region(const SubdivArgs &a, uint32_t img, uint32_t x, uint32_t y,
                             uint32_t w, uint32_t h, uint32_t r, uint32_t level, uint32_t lane) {
    Region *q = kQueue ? a.queue : a.out;
    uint32_t *tail = kQueue ? &a.ctrl[kTail] : &a.ctrl[kCount + level + 1];
    emit_entries<kQueue>(a, q, tail, a.cap, r * r, kScan, level + 1, lane, [&](uint32_t j, Region &e) {
        const uint32_t jx = j % r, jy = j / r;
        const uint32_t x0 = x + (uint32_t)(((uint64_t)jx * w) / r);
        const uint32_t x1 = x + (uint32_t)(((uint64_t)(jx + 1) * w) / r);
        const uint32_t y0 = y + (uint32_t)(((uint64_t)jy * h) / r);
        const uint32_t y1 = y + (uint32_t)(((uint64_t)(jy + 1) * h) / r);
        e.img = img;
        e.xy = pack_xy(x0, y0);
        e.wh = pack_wh(x1 - x0, y1 - y0);
        return x1 > x0 && y1 > y0;
    });
}

// The per-pixel work of a leaf as row bands of about `band` pixels, leaf
// entries that any wave can take (several blocks per region, MBR, Sec.
// 4.3.2): in the queue forms appended to the queue, in the per-level form to
// the next level's table, whose kernel computes them beside that level's
// regions.
template <bool kQueue>
__device__ void queue_leaf_bands(const SubdivArgs &a, uint32_t img, uint32_t x, uint32_t y,
                                 uint32_t w, uint32_t h, uint32_t band, uint32_t level,
                                 uint32_t lane) {
    const uint32_t hb = max(1u, band / w);
    const uint32_t nb = (h + hb - 1) / hb;
    Region *q = kQueue ? a.queue : a.out;
    uint32_t *tail = kQueue ? &a.ctrl[kTail] : &a.ctrl[kCount + level + 1];
    emit_entries<kQueue>(a, q, tail, a.cap, nb, kLeaf, level, lane,
                       [&](uint32_t j, Region &e) {
                           const uint32_t y0 = y + j * hb;
                           e.img = img;
                           e.xy = pack_xy(x, y0);
                           e.wh = pack_wh(w, min(y + h, y0 + hb) - y0);
                           return true;
                       });
}

// What follows the border query of a region (Sec. 4.2.1): fill T when the
// ring is uniform, else leaf L at size B, else split S.
template <bool kQueue>
__device__ void decide_region(const SubdivArgs &a, uint32_t img, const Image &im, uint32_t x,
                              uint32_t y, uint32_t w, uint32_t h, uint32_t level,
                              uint32_t outcome, uint32_t v, uint32_t lane) {
    DevStats *st = a.stats;
    const unsigned long long area = (unsigned long long)w * h;
    if (st) {
        wave_add64(&st->regions[level], 1ull);
        wave_add64(&st->ring_px, ring_size(w, h));
        wave_max(&st->levels, level + 1);
    }
    if (outcome == kUniform) {
        fill_region(im.out, im.W, x, y, w, h, v, lane);
        if (st) {
            wave_add64(&st->fills[level], 1ull);
            wave_add64(&st->fill_px, area);
        }
        return;
    }
    if (w <= im.B && h <= im.B) {
        if (st) {
            wave_add64(&st->leaves[level], 1ull);
            wave_add64(&st->leaf_px, area);
        }
        // The ring stream has computed a leaf the wave keeps; a larger one
        // (64-bit area: a 65536 x 65536 leaf has 2^32 pixels) goes out as bands.
        if (outcome != kLeafDone)
            queue_leaf_bands<kQueue>(a, img, x, y, w, h, im.band, level, lane);
        return;
    }
    if (level + 1 >= kMaxLevels) {  // unreachable for valid sizes; never write past the tables
        wave_or(&a.ctrl[kOverflow], 2u);
        wave_or(&a.ctrl[kSticky], kErrOverflow);
        return;
    }
    split_region<kQueue>(a, img, x, y, w, h, im.r, level, lane);
    if (st)
        wave_add64(&st->splits[level], 1ull);
}

// The positions of a ring scan: the ring in its spread order (n_ring
// positions), then, for a leaf, its inside (RectOrder).
struct RingLeafOrder {
    uint32_t x, y, w, h, nring, q, bits, n_ring, n_all;
    RectOrder order;
    __device__ RingLeafOrder(const Image &im, uint32_t x_, uint32_t y_, uint32_t w_, uint32_t h_,
                             bool leaf)
        : x(x_), y(y_), w(w_), h(h_), nring(ring_size(w_, h_)), q((nring + kWave - 1) / kWave),
          bits(q > 1 ? 32u - (uint32_t)__builtin_clz(q - 1) : 0u),  // 2^bits >= q
          n_ring(kWave << bits), n_all(0),
          order(im, x_ + 1, y_ + 1, leaf && w_ > 2 && h_ > 2 ? w_ - 2 : 1u,
                leaf && w_ > 2 && h_ > 2 ? h_ - 2 : 1u) {
        n_all = n_ring + (leaf && w_ > 2 && h_ > 2 ? order.positions() : 0u);
    }
    // The stream's end: a leaf's stream runs past the ring even with no inside.
    __device__ uint32_t end(bool leaf) const { return leaf ? max(n_all, n_ring + 1u) : n_ring; }
    __device__ __forceinline__ bool pixel(uint32_t j, uint32_t &px, uint32_t &py) const {
        if (j >= n_ring)
            return j < n_all && order.pixel(j - n_ring, px, py);
        const uint32_t round = j / kWave;
        const uint32_t off = bits ? __brev(round) >> (32u - bits) : 0u;
        const uint32_t t = (j % kWave) * q + off;
        if (off >= q || t >= nring)
            return false;
        ring_pixel(x, y, w, h, t, px, py);
        return true;
    }
};

// Q over the whole ring, taken in a spread order. The ring is cut into 64
// arcs of q pixels, one per lane of the first round, so the first 64 pixels
// are spaced evenly around it; later rounds take, in every arc, the offsets
// 0, q/2, q/4, 3q/4, q/8, ... (bit-reversed round numbers), so that after
// 2^k rounds the pixels taken are spaced q/2^k apart. A mixed ring is found
// mixed as soon as one of its pixels has a dwell other than the rest; on a
// ring whose pixels mostly run to D this finds a short arc of other dwells
// in a few rounds rather than after up to q rounds of D iterations each, and
// those rings are the ones a split must wait for.
//
// Every finished ring dwell is written to the image: a pixel on a scanned
// ring ends up with its own dwell whatever follows (a fill of that ring
// writes the same value; a split puts the pixel on a child's ring), so the
// write is never wrong and a leaf need not compute it again. When `leaf` is
// set (a leaf-size region the wave computes itself), a mixed ring goes on
// into the leaf's inside in the same stream. Returns the stream's outcome
// (kUniform with v, kMixed, kLeafDone) and adds the iterations done to the
// counters: ring pixels to the ring's, inside pixels to the leaves'.
__device__ uint32_t scan_ring(const SubdivArgs &a, const Image &im, uint32_t x, uint32_t y,
                              uint32_t w, uint32_t h, bool leaf, uint32_t &v) {
    const RingLeafOrder ro(im, x, y, w, h, leaf);
    unsigned long long it_ring = 0, it_leaf = 0;
    uint32_t partial = 0;
    const uint32_t outcome = dwell_stream<true>(
        im, ro.n_ring, ro.end(leaf),
        [&](uint32_t j, uint32_t &px, uint32_t &py) { return ro.pixel(j, px, py); },
        [&](uint32_t px, uint32_t py, uint32_t d, bool ring) {
            put_dwell(im.out, (size_t)py * im.W + px, d);
            if (ring)
                it_ring += d;
            else
                it_leaf += d;
        },
        v, partial);
    if (a.stats) {
        wave_add64(&a.stats->iters_ring, wave_sum(it_ring + partial));
        if (leaf)
            wave_add64(&a.stats->iters_leaf, wave_sum(it_leaf));
    }
    return outcome;
}

// One region, by one wave: border query Q, then fill T, leaf L or split S
// (Sec. 4.2.1).
template <bool kQueue>
__device__ void process_region(const SubdivArgs &a, const Region &R, uint32_t lane) {
    const uint32_t img = uniform(R.img), xy = uniform(R.xy), wh = uniform(R.wh);
    const uint32_t tag = uniform(R.tag);
    const uint32_t level = tag & 0x3fu, kind = (tag >> 6) & 0x3u;
    const Image im = image_of(a, img);
    const uint32_t x = xy & 0xffffu, y = xy >> 16;
    const uint32_t w = (wh & 0xffffu) + 1, h = (wh >> 16) + 1;
    if (kind == kLeaf) {  // a band of a leaf decided earlier: every pixel
        unsigned long long li = leaf_region(im, x, y, w, h);
        if (a.stats)
            wave_add64(&a.stats->iters_leaf, wave_sum(li));
        return;
    }
    // A leaf-size region whose leaf this wave computes: its ring stream goes
    // on into the leaf when the ring is mixed.
    const bool leaf = w <= im.B && h <= im.B && (unsigned long long)w * h <= im.band;
    uint32_t v = 0;
    const uint32_t outcome = scan_ring(a, im, x, y, w, h, leaf, v);
    decide_region<kQueue>(a, img, im, x, y, w, h, level, outcome, v, lane);
}

// Per-level kernel: waves take the level's regions through an atomic counter;
// the region count was written by the previous level. One counter address
// serves one atomic at a time (about 11 ns apart on MI355X), so on levels with
// many regions per wave a wave takes a few consecutive regions per atomic
// (one while the level has few regions per wave, which balances best).
__global__ __launch_bounds__(kBlock) void level_kernel(SubdivArgs a) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t n = min(a.ctrl[kCount + a.level], a.cap);
    const uint32_t waves = gridDim.x * kWavesPerBlock;
    const uint32_t chunk = max(1u, min(8u, n / (waves * 8u)));
    for (;;) {
        const uint32_t idx0 = wave_add(&a.ctrl[kClaim + a.level], chunk);
        if (idx0 >= n)
            break;
        const uint32_t idx1 = min(n, idx0 + chunk);
        for (uint32_t idx = idx0; idx < idx1; ++idx)
            process_region<false>(a, a.in[idx], lane);
    }
}

// Per-level kernel with the grid sized on the host to the level's region
// count: wave i takes region i.
__global__ __launch_bounds__(kBlock) void level_exact_kernel(SubdivArgs a, uint32_t n) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t idx = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (idx >= n)
        return;
    process_region<false>(a, a.in[idx], lane);
}

// The ring decision of a workgroup's waves sharing one region, in LDS: the
// first dwell proposed becomes v for all, and a wave that sees the ring
// mixed says so to the others.
constexpr uint32_t kNoVal = 0xffffffffu;

struct SharedDecision {
    uint32_t *val, *flag;
    __device__ uint32_t propose(uint32_t x) const {
        uint32_t old = kNoVal;
        if (first_lane())
            old = atomicCAS(val, kNoVal, x);
        old = uniform(old);
        return old == kNoVal ? x : old;
    }
    __device__ bool known(uint32_t &x) const {
        const uint32_t y = uniform(*(volatile uint32_t *)val);
        if (y == kNoVal)
            return false;
        x = y;
        return true;
    }
    __device__ bool mixed() const { return uniform(*(volatile uint32_t *)flag) != 0; }
    __device__ void set_mixed() const {
        if (first_lane())
            *(volatile uint32_t *)flag = 1u;
    }
};

// Per-level kernel for levels of large regions (rings of kCoopRingPixels
// pixels or more): the four waves of a workgroup share one region. Each scans every
// fourth position of the ring order and they decide the ring together
// through LDS (a mixed ring stops every wave at its next round); after a
// barrier they fill the region together, or stream a leaf's inside together
// (a leaf's ring is always scanned whole), or one wave queues its bands or
// appends its children. A long ring is then a quarter of a wave's work
// instead of all of it.
__global__ __launch_bounds__(kBlock) void level_coop_kernel(SubdivArgs a) {
    __shared__ uint32_t sh_idx, sh_val, sh_mixed;
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint32_t n = min(a.ctrl[kCount + a.level], a.cap);
    const SharedDecision dec{&sh_val, &sh_mixed};
    DevStats *st = a.stats;
    for (;;) {
        if (threadIdx.x == 0) {
            sh_idx = atomicAdd(&a.ctrl[kClaim + a.level], 1u);
            sh_val = kNoVal;
            sh_mixed = 0;
        }
        __syncthreads();
        const uint32_t idx = uniform(*(volatile uint32_t *)&sh_idx);
        if (idx >= n)
            break;
        const Region R = a.in[idx];
        const uint32_t img = uniform(R.img), xy = uniform(R.xy), wh = uniform(R.wh);
        const uint32_t tag = uniform(R.tag);
        const uint32_t level = tag & 0x3fu, kind = (tag >> 6) & 0x3u;
        const Image im = image_of(a, img);
        const uint32_t x = xy & 0xffffu, y = xy >> 16;
        const uint32_t w = (wh & 0xffffu) + 1, h = (wh >> 16) + 1;
        const unsigned long long area = (unsigned long long)w * h;
        const bool leaf_size = w <= im.B && h <= im.B;
        const bool leaf = leaf_size && area <= im.band;
        const RingLeafOrder ro(im, x, y, w, h, leaf);
        if (kind == kLeaf) {  // a leaf band: every fourth position on each wave
            const RectOrder band(im, x, y, w, h);
            const uint32_t np = band.positions();
            const uint32_t part = np > wave ? (np - wave + kWavesPerBlock - 1) / kWavesPerBlock : 0u;
            unsigned long long it_leaf = 0;
            uint32_t vloc = 0, partial = 0;
            dwell_stream<false>(
                im, 0u, part,
                [&](uint32_t i, uint32_t &px, uint32_t &py) {
                    return band.pixel(wave + i * kWavesPerBlock, px, py);
                },
                [&](uint32_t px, uint32_t py, uint32_t d, bool) {
                    put_dwell(im.out, (size_t)py * im.W + px, d);
                    it_leaf += d;
                },
                vloc, partial);
            if (st)
                wave_add64(&st->iters_leaf, wave_sum(it_leaf));
        } else {
            const uint32_t part = ro.n_ring > wave ? (ro.n_ring - wave + kWavesPerBlock - 1) / kWavesPerBlock : 0u;
            unsigned long long it_ring = 0;
            uint32_t vloc = 0, partial = 0;
            dwell_stream<true>(
                im, part, leaf ? part + 1u : part,
                [&](uint32_t i, uint32_t &px, uint32_t &py) {
                    return i < part && ro.pixel(wave + i * kWavesPerBlock, px, py);
                },
                [&](uint32_t px, uint32_t py, uint32_t d, bool) {
                    put_dwell(im.out, (size_t)py * im.W + px, d);
                    it_ring += d;
                },
                vloc, partial, dec);
            if (st)
                wave_add64(&st->iters_ring, wave_sum(it_ring + partial));
        }
        __syncthreads();
        if (kind != kLeaf) {
            const bool mixed = dec.mixed();
            uint32_t val = 0;
            dec.known(val);
            if (st && wave == 0) {
                wave_add64(&st->regions[level], 1ull);
                wave_add64(&st->ring_px, ring_size(w, h));
                wave_max(&st->levels, level + 1);
            }
            if (!mixed) {
                fill_region(im.out, im.W, x, y, w, h, val, lane, wave, kWavesPerBlock);
                if (st && wave == 0) {
                    wave_add64(&st->fills[level], 1ull);
                    wave_add64(&st->fill_px, area);
                }
            } else if (leaf_size) {
                if (st && wave == 0) {
                    wave_add64(&st->leaves[level], 1ull);
                    wave_add64(&st->leaf_px, area);
                }
                if (leaf) {
                    const uint32_t np = w > 2 && h > 2 ? ro.order.positions() : 0u;
                    const uint32_t part = np > wave ? (np - wave + kWavesPerBlock - 1) / kWavesPerBlock : 0u;
                    unsigned long long it_leaf = 0;
                    uint32_t vloc = 0, partial = 0;
                    dwell_stream<false>(
                        im, 0u, part,
                        [&](uint32_t i, uint32_t &px, uint32_t &py) {
                            return ro.order.pixel(wave + i * kWavesPerBlock, px, py);
                        },
                        [&](uint32_t px, uint32_t py, uint32_t d, bool) {
                            put_dwell(im.out, (size_t)py * im.W + px, d);
                            it_leaf += d;
                        },
                        vloc, partial);
                    if (st)
                        wave_add64(&st->iters_leaf, wave_sum(it_leaf));
                } else if (wave == 0) {
                    queue_leaf_bands<false>(a, img, x, y, w, h, im.band, level, lane);
                }
            } else if (wave == 0) {
                if (level + 1 >= kMaxLevels) {
                    wave_or(&a.ctrl[kOverflow], 2u);
                    wave_or(&a.ctrl[kSticky], kErrOverflow);
                } else {
                    split_region<false>(a, img, x, y, w, h, im.r, level, lane);
                    if (st)
                        wave_add64(&st->splits[level], 1ull);
                }
            }
        }
        __syncthreads();  // the LDS words are the next region's
    }
}

// Persistent kernel: every wave takes the next queue slot (one atomic add, a
// ticket), waits until the slot is published (its tag carries this launch's
// epoch), processes the region and appends its children to the queue.
// `pending` counts entries queued or in progress; a producer adds its
// children to it before it removes itself, so pending reaches 0 only when no
// entry is left or can still be published, and then every waiting wave
// leaves.
//
// Waiting is cheap on purpose: the slot's tag and `pending` are read with
// relaxed loads (no cache invalidation), with a growing pause between reads,
// and once the tag is seen the entry's fields are read with device-scope
// loads, past the XCD's L2, instead of an acquire fence. Every wait is also
// bounded in wall-clock time: a wave that waits longer than a.wait_ticks of
// the constant-rate clock records a timeout and leaves, so the grid always
// drains.
__device__ __forceinline__ void pause(uint32_t n) {
    for (uint32_t i = 0; i < n; ++i)
        __builtin_amdgcn_s_sleep(2);
}

__global__ __launch_bounds__(kBlock) void persistent_kernel(SubdivArgs a) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    uint32_t *ctrl = a.ctrl;
    for (;;) {
        // Every lane runs the wait; the values it reads are made uniform.
        const uint32_t idx = wave_add(&ctrl[kHead], 1u);
        const unsigned long long t0 = clock_now();
        uint32_t nap = 1, polls = 0;
        bool ready = false;
        for (;;) {
            if (idx < a.cap) {
                const uint32_t t = uniform(__hip_atomic_load(&a.queue[idx].tag, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT));
                if ((t >> 8) == a.epoch) {
                    ready = true;
                    break;
                }
            }
            if ((++polls & 7) == 0 || idx >= a.cap) {
                if (uniform(__hip_atomic_load(&ctrl[kPending], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT)) == 0)
                    break;
                if (clock_now() - t0 > a.wait_ticks) {
                    wave_or(&ctrl[kSticky], kErrTimeout);
                    break;
                }
            }
            pause(nap);
            nap = min(nap * 2, 32u);
        }
        if (!ready)
            return;
        // The entry's fields are read past the XCD's L2, with device-scope
        // loads, after its tag: the producer wrote them back before it
        // published the tag, so they are the entry's. (An acquire fence
        // would invalidate the whole L2 instead: 4 % slower.)
        Region R;
        R.img = __hip_atomic_load(&a.queue[idx].img, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        R.xy = __hip_atomic_load(&a.queue[idx].xy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        R.wh = __hip_atomic_load(&a.queue[idx].wh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        R.tag = __hip_atomic_load(&a.queue[idx].tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        process_region<true>(a, R, lane);
        wave_add(&ctrl[kPending], (uint32_t)-1);
    }
}

// ---------------------------------------------------------------------------
// Serving kernel: continuous batching into one persistent kernel.
//
// Every wave loops: pick the oldest admitted request with a queue entry not
// yet taken, take a reference to its slot (so that the slot cannot be handed
// to another request while the wave may still touch it), take a ticket (one
// atomic add on the request's head), process the entry exactly as the
// persistent kernel does, with the request's own queue and counters, and
// drop the reference. Between entries, one wave at a time (at most every
// poll_ticks) reads the host's mailbox and admits posted requests into free
// slots. The wave that counts a request's last entry done reports the
// request to the host; the last wave to drop a reference to the finished
// request frees its slot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long uniform64(unsigned long long v) {
    return ((unsigned long long)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

__device__ __forceinline__ uint32_t slot_gen(uint32_t st) { return st >> 8; }
__device__ __forceinline__ uint32_t slot_kind(uint32_t st) { return st & 0xffu; }

// A struct that the host or other waves write while the kernel runs, read
// whole by one wave: one 32-bit word per lane with a relaxed atomic load (a
// vector load, never through the scalar cache), then each word made uniform.
// Every lane of the wave must be active.
template <class T, int kScope>
__device__ __forceinline__ T load_words(const T *p) {
    constexpr uint32_t nw = sizeof(T) / 4;
    static_assert(sizeof(T) % 4 == 0 && nw <= (uint32_t)kWave, "one word per lane");
    const uint32_t lane = __lane_id();
    const uint32_t *w = reinterpret_cast<const uint32_t *>(p);
    const uint32_t v = lane < nw ? __hip_atomic_load(w + lane, __ATOMIC_RELAXED, kScope) : 0u;
    T out;
    uint32_t *o = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (uint32_t i = 0; i < nw; ++i)
        o[i] = __builtin_amdgcn_readlane(v, i);
    return out;
}

template <class T>
__device__ __forceinline__ void store_words(T *p, const T &v) {
    constexpr uint32_t nw = sizeof(T) / 4;
    static_assert(sizeof(T) % 4 == 0 && nw <= (uint32_t)kWave, "one word per lane");
    const uint32_t lane = __lane_id();
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&v);
    uint32_t word = 0;
#pragma unroll
    for (uint32_t i = 0; i < nw; ++i)
        word = lane == i ? src[i] : word;
    if (lane < nw)
        reinterpret_cast<uint32_t *>(p)[lane] = word;
}

// The request in a slot as subdivision arguments.
__device__ __forceinline__ SubdivArgs slot_args(const ServerArgs &sa, ServerSlot *sl,
                                                const ServerPost &post, uint32_t gen) {
    SubdivArgs a{};
    a.single = post.im;
    a.nimg = 1;
    a.queue = sa.queue + post.qoff;
    a.cap = post.qcap;
    a.epoch = gen;
    a.wait_ticks = sa.wait_ticks;
    a.ctrl = sl->ctrl;
    return a;
}

// Admit the request posted in slot k (this wave holds the slot in
// kSlotAdmitting): copy its post, set its counters, write its level-0
// regions (the g x g floor partition) into its queue, then publish the slot.
__device__ void admit(const ServerArgs &sa, uint32_t k, uint32_t gen, uint32_t lane) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // the post was written before its doorbell
    const ServerPost post = load_words<ServerPost, __HIP_MEMORY_SCOPE_SYSTEM>(&sa.mb->post[k]);
    ServerSlot *sl = sa.slots + k;
    store_words(&sl->post, post);
    const Image &im = post.im;
    const uint32_t g = im.g, nseed = g * g;
    // The reference word is left alone: a wave that read the slot before it
    // was freed may still add and drop a reference.
    for (uint32_t i = lane; i < kCtrlWords; i += kWave)
        if (i != kRefs)
            sl->ctrl[i] = (i == kTail || i == kPending) ? nseed : 0u;
    Region *q = sa.queue + post.qoff;
    for (uint32_t j = lane; j < nseed; j += kWave) {
        const uint32_t jx = j % g, jy = j / g;
        const uint32_t x0 = (uint32_t)(((uint64_t)jx * im.W) / g);
        const uint32_t x1 = (uint32_t)(((uint64_t)(jx + 1) * im.W) / g);
        const uint32_t y0 = (uint32_t)(((uint64_t)jy * im.H) / g);
        const uint32_t y1 = (uint32_t)(((uint64_t)(jy + 1) * im.H) / g);
        q[j] = Region{0, pack_xy(x0, y0), pack_wh(x1 - x0, y1 - y0), gen << 8};
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&sa.ctl->state[k], (gen << 8) | kSlotActive, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Read the doorbells and admit every request posted in a free slot. Returns
// whether one was admitted. Also turns the host's stop flag into a device
// word that every wave can read cheaply.
__device__ bool poll_mailbox(const ServerArgs &sa, uint32_t lane) {
    if (uniform(__hip_atomic_load(&sa.mb->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))) {
        const unsigned long long t = clock_now() | 1ull;
        if (first_lane())
            atomicCAS(&sa.ctl->stop_time, 0ull, t);
        return false;
    }
    uint32_t posted = 0, st = 0;
    if (lane < sa.nslots) {
        posted = __hip_atomic_load(&sa.mb->doorbell[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        st = __hip_atomic_load(&sa.ctl->state[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned long long mask =
        __ballot(posted != 0 && slot_kind(st) == kSlotFree && posted != slot_gen(st));
    bool any = false;
    while (mask) {
        const uint32_t k = uniform((uint32_t)__builtin_ctzll(mask));
        mask &= mask - 1;
        const uint32_t gen = __builtin_amdgcn_readlane(posted, k);
        const uint32_t stk = __builtin_amdgcn_readlane(st, k);
        uint32_t old = ~stk;
        if (first_lane())
            old = atomicCAS(&sa.ctl->state[k], stk, (gen << 8) | kSlotAdmitting);
        if (uniform(old) != stk)
            continue;
        admit(sa, k, gen, lane);
        any = true;
    }
    return any;
}

// Report request k as finished: mark its slot done, then make its image
// visible beyond the device and tell the host. The slot is freed by the last
// wave that drops its reference.
__device__ void finish_request(const ServerArgs &sa, ServerSlot *sl, uint32_t k, uint32_t gen) {
    const uint32_t err = uniform(__hip_atomic_load(&sl->ctrl[kSticky], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT));
    const int32_t status = (err & kErrTimeout)    ? (int32_t)ASK_ETIMEOUT
                           : (err & kErrOverflow) ? (int32_t)ASK_EOVERFLOW
                                                  : (int32_t)ASK_OK;
    __hip_atomic_store(&sa.ctl->state[k], (gen << 8) | kSlotDone, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long t = clock_now();
    if (first_lane()) {
        ServerDone *d = &sa.mb->done[k];
        __hip_atomic_store(&d->status, status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&d->ticks, t,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        __hip_atomic_store(&d->gen, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Take a reference to slot k while it holds request gen; false (and no
// reference) if it no longer does.
__device__ bool take_ref(const ServerArgs &sa, uint32_t k, uint32_t gen) {
    ServerSlot *sl = sa.slots + k;
    if (first_lane())
        __hip_atomic_fetch_add(&sl->ctrl[kRefs], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t st = uniform(__hip_atomic_load(&sa.ctl->state[k], __ATOMIC_ACQUIRE,
                                                  __HIP_MEMORY_SCOPE_AGENT));
    return st == ((gen << 8) | kSlotActive);
}

// Drop a reference to slot k. The wave that drops the last reference frees
// the slot if it holds a finished request (whichever: a wave whose reference
// was taken for an older request may be the last). A request is marked done
// before its finishing wave drops its own reference, so when the count
// reaches 0 after that, the dropping wave sees the mark.
__device__ void drop_ref(const ServerArgs &sa, uint32_t k) {
    ServerSlot *sl = sa.slots + k;
    uint32_t old = 0;
    if (first_lane())
        old = __hip_atomic_fetch_add(&sl->ctrl[kRefs], (uint32_t)-1, __ATOMIC_ACQ_REL,
                                     __HIP_MEMORY_SCOPE_AGENT);
    if (uniform(old) != 1u)
        return;
    const uint32_t st = uniform(__hip_atomic_load(&sa.ctl->state[k], __ATOMIC_ACQUIRE,
                                                  __HIP_MEMORY_SCOPE_AGENT));
    if (slot_kind(st) == kSlotDone && first_lane())
        atomicCAS(&sa.ctl->state[k], st, (st & ~0xffu) | kSlotFree);
}

// Serve ticket idx of request k (generation gen), holding a reference to
// the slot: wait until the entry is published (or the request has finished,
// when the ticket lies beyond its last entry), process it and count it done.
__device__ void serve_ticket(const ServerArgs &sa, uint32_t k, uint32_t gen, uint32_t idx,
                             uint32_t lane) {
    ServerSlot *sl = sa.slots + k;
    const ServerPost post = load_words<ServerPost, __HIP_MEMORY_SCOPE_AGENT>(&sl->post);
    const SubdivArgs a = slot_args(sa, sl, post, gen);
    const unsigned long long t0 = clock_now();
    uint32_t nap = 1, polls = 0;
    bool ready = false;
    for (;;) {
        if (idx < a.cap) {
            const uint32_t t = uniform(__hip_atomic_load(&a.queue[idx].tag, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT));
            if ((t >> 8) == gen) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                ready = true;
                break;
            }
        }
        if ((++polls & 7) == 0 || idx >= a.cap) {
            if (uniform(__hip_atomic_load(&sl->ctrl[kPending], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT)) == 0)
                return;  // the request has finished: no entry will come
            if (clock_now() - t0 > a.wait_ticks) {
                // Never expected: the request cannot finish without this entry.
                wave_or(&sl->ctrl[kSticky], kErrTimeout);
                break;
            }
        }
        pause(nap);
        nap = min(nap * 2, 32u);
    }
    if (ready)
        process_region<true>(a, a.queue[idx], lane);
    // Count the entry done, releasing this wave's writes; the last one also
    // acquires everyone else's.
    uint32_t left = 0;
    if (first_lane())
        left = __hip_atomic_fetch_add(&sl->ctrl[kPending], (uint32_t)-1, __ATOMIC_ACQ_REL,
                                      __HIP_MEMORY_SCOPE_AGENT);
    if (uniform(left) == 1u)
        finish_request(sa, sl, k, gen);
}

__global__ __launch_bounds__(kBlock) void server_kernel(ServerArgs sa) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    uint32_t nap = 1;
    const unsigned long long t0 = clock_now();
    if (first_lane())  // the idle clock starts with the first wave
        atomicCAS(&sa.ctl->last_busy, 0ull, t0);
    for (;;) {
        // Mailbox, at most every poll_ticks over the whole grid.
        const unsigned long long now = clock_now();
        const unsigned long long due = uniform64(
            __hip_atomic_load(&sa.ctl->next_poll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (now >= due) {
            unsigned long long old = ~due;
            if (first_lane())
                old = atomicCAS(&sa.ctl->next_poll, due, now + sa.poll_ticks);
            if (uniform64(old) == due && poll_mailbox(sa, lane)) {
                __hip_atomic_store(&sa.ctl->last_busy, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                nap = 1;
            }
        }
        // Lane k looks at slot k: an active request with an entry reserved
        // below its tail (and inside its queue) not yet taken.
        uint32_t st = 0;
        bool avail = false;
        if (lane < sa.nslots) {
            st = __hip_atomic_load(&sa.ctl->state[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (slot_kind(st) == kSlotActive) {
                ServerSlot *sl = sa.slots + lane;
                const uint32_t head = __hip_atomic_load(&sl->ctrl[kHead], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t lim = min(__hip_atomic_load(&sl->ctrl[kTail], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT),
                                         __hip_atomic_load(&sl->post.qcap, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT));
                avail = head < lim;
            }
        }
        if (__ballot(avail)) {
            // The oldest request first: the least generation (the host hands
            // them out in order and restarts the server before they wrap).
            const uint32_t oldest = uniform(wave_min(avail ? slot_gen(st) : 0xffffffffu));
            const uint32_t k = uniform((uint32_t)__builtin_ctzll(__ballot(avail && slot_gen(st) == oldest)));
            if (take_ref(sa, k, oldest)) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the slot's post and counters
                const uint32_t idx = wave_add(&sa.slots[k].ctrl[kHead], 1u);
                serve_ticket(sa, k, oldest, idx, lane);
                __hip_atomic_store(&sa.ctl->last_busy, clock_now(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            drop_ref(sa, k);
            nap = 1;
            continue;
        }
        // Nothing to take. Leave when stopped, or idle for idle_ticks, with no
        // request admitted or being admitted, or stopped for wait_ticks in
        // any case (a request that cannot finish never holds the grid);
        // otherwise rest a little longer each time.
        const unsigned long long t = clock_now();
        const unsigned long long stop_time = uniform64(
            __hip_atomic_load(&sa.ctl->stop_time, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        const unsigned long long busy = uniform64(
            __hip_atomic_load(&sa.ctl->last_busy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        const bool none = __ballot(slot_kind(st) == kSlotActive || slot_kind(st) == kSlotAdmitting) == 0;
        // (The times were taken by other waves and may be a little later
        // than t.)
        const unsigned long long since_stop = t > stop_time ? t - stop_time : 0;
        const unsigned long long since_busy = t > busy ? t - busy : 0;
        if ((stop_time && (none || since_stop > sa.wait_ticks)) || (none && since_busy > sa.idle_ticks))
            return;
        pause(nap);
        nap = min(nap * 2, 256u);
    }
}

// ---------------------------------------------------------------------------
// Set-up kernels.
// ---------------------------------------------------------------------------
// Clears the per-render control words (not the sticky error word) and the
// counters.
__global__ void reset_kernel(uint32_t *ctrl, DevStats *stats) {
    for (uint32_t i = threadIdx.x; i < kSticky; i += blockDim.x)
        ctrl[i] = 0;
    if (stats) {
        uint32_t *s = reinterpret_cast<uint32_t *>(stats);
        for (uint32_t i = threadIdx.x; i < sizeof(DevStats) / 4; i += blockDim.x)
            s[i] = 0;
    }
}

// Every entry of a queue zeroed (no slot then carries a launch epoch): the
// persistent queue of a render captured in a graph, cleared by the graph.
__global__ void clear_queue_kernel(uint4 *q, uint32_t entries) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < entries)
        q[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Data carried in the launch's arguments, stored to device memory.
__global__ void write_words_kernel(WordsArg w) {
    for (uint32_t i = threadIdx.x; i < w.n; i += blockDim.x)
        w.dst[i] = w.words[i];
}

// Level 0 (Sec. 4.2: G = g x g initial regions): the floor partition of each
// image. Seed i belongs to the image whose seed range holds it.
template <bool kQueue>
__global__ void seed_kernel(SubdivArgs a, uint32_t nseeds) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (kQueue) {
            a.ctrl[kTail] = nseeds;
            a.ctrl[kPending] = nseeds;
        } else {
            a.ctrl[kCount] = nseeds;
        }
    }
    if (i >= nseeds)
        return;
    uint32_t img = 0, local = i;
    if (a.table) {
        uint32_t lo = 0, hi = a.nimg;  // find seed_base[lo] <= i < seed_base[lo+1]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (a.seed_base[mid] <= i)
                lo = mid;
            else
                hi = mid;
        }
        img = lo;
        local = i - a.seed_base[img];
    }
    const Image im = image_of(a, img);
    const uint32_t g = im.g;
    const uint32_t jx = local % g, jy = local / g;
    const uint32_t x0 = (uint32_t)(((uint64_t)jx * im.W) / g);
    const uint32_t x1 = (uint32_t)(((uint64_t)(jx + 1) * im.W) / g);
    const uint32_t y0 = (uint32_t)(((uint64_t)jy * im.H) / g);
    const uint32_t y1 = (uint32_t)(((uint64_t)(jy + 1) * im.H) / g);
    const Region e{img, pack_xy(x0, y0), pack_wh(x1 - x0, y1 - y0), a.epoch << 8};
    if (kQueue)
        a.queue[i] = e;
    else
        a.out[i] = e;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <uint32_t kTileW>
static hipError_t launch_exhaustive_tile(const Image &im, hipStream_t s) {
    constexpr uint32_t rows = kWavesPerBlock * (kWave / kTileW);  // pixel rows per workgroup
    dim3 grid((im.W + kTileW - 1) / kTileW, (im.H + rows - 1) / rows);
    hipLaunchKernelGGL(exhaustive_kernel<kTileW>, grid, dim3(kBlock), 0, s, im);
    return hipGetLastError();
}

hipError_t launch_exhaustive(const Image &im, hipStream_t s) {
    switch (im.tile_w) {
    case 4: return launch_exhaustive_tile<4>(im, s);
    case 8: return launch_exhaustive_tile<8>(im, s);
    case 32: return launch_exhaustive_tile<32>(im, s);
    case 64: return launch_exhaustive_tile<64>(im, s);
    default: return launch_exhaustive_tile<16>(im, s);
    }
}

hipError_t launch_write_words(const WordsArg &w, hipStream_t s) {
    hipLaunchKernelGGL(write_words_kernel, dim3(1), dim3(kBlock), 0, s, w);
    return hipGetLastError();
}

hipError_t launch_reset(uint32_t *ctrl, DevStats *stats, hipStream_t s) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(kBlock), 0, s, ctrl, stats);
    return hipGetLastError();
}

hipError_t launch_clear_queue(Region *queue, uint32_t entries, hipStream_t s) {
    const uint32_t blocks = (entries + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(clear_queue_kernel, dim3(blocks ? blocks : 1), dim3(kBlock), 0, s,
                       reinterpret_cast<uint4 *>(queue), entries);
    return hipGetLastError();
}

hipError_t launch_seed_levels(const SubdivArgs &a, uint32_t nseeds, hipStream_t s) {
    const uint32_t blocks = (nseeds + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(seed_kernel<false>, dim3(blocks ? blocks : 1), dim3(kBlock), 0, s, a, nseeds);
    return hipGetLastError();
}

hipError_t launch_seed_queue(const SubdivArgs &a, uint32_t nseeds, hipStream_t s) {
    const uint32_t blocks = (nseeds + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(seed_kernel<true>, dim3(blocks ? blocks : 1), dim3(kBlock), 0, s, a, nseeds);
    return hipGetLastError();
}

hipError_t launch_level(const SubdivArgs &a, uint32_t grid_blocks, hipStream_t s) {
    hipLaunchKernelGGL(level_kernel, dim3(grid_blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_level_coop(const SubdivArgs &a, uint32_t grid_blocks, hipStream_t s) {
    hipLaunchKernelGGL(level_coop_kernel, dim3(grid_blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_level_exact(const SubdivArgs &a, uint32_t nregions, hipStream_t s) {
    const uint32_t blocks = (nregions + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(level_exact_kernel, dim3(blocks), dim3(kBlock), 0, s, a, nregions);
    return hipGetLastError();
}

hipError_t launch_persistent(const SubdivArgs &a, uint32_t grid_blocks, hipStream_t s) {
    hipLaunchKernelGGL(persistent_kernel, dim3(grid_blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t occupancy_level(int *blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, level_kernel, kBlock, 0);
}

hipError_t launch_server(const ServerArgs &a, uint32_t grid_blocks, hipStream_t s) {
    hipLaunchKernelGGL(server_kernel, dim3(grid_blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t occupancy_server(int *blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, server_kernel, kBlock, 0);
}

hipError_t occupancy_persistent(int *blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, persistent_kernel, kBlock, 0);
}

}  // namespace ask
