// ask3d.hip -- the 3-D extension of the subdivision (the paper's section on
// subdivisions at higher dimensions): exhaustive and level-by-level
// subdivision volumes of the quaternion Julia set, the level tables holding
// one space-filling-curve scalar per box (canonical or Morton order).
//
// One wave per box: the waves the device holds at once claim the entries
// of their level's table from eight counters, one per XCD (a box or a chunk
// of boxes per atomic), so a level launch needs no count from the host and
// waves that drew cheap boxes take more. The host knows in advance the last
// level any box can reach (the first whose cells all have sides <= B) and
// launches that many level kernels back to back, with no read-back. The
// exhaustive volume is claimed the same way, in columns of voxels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "ask3d.h"

namespace {

constexpr uint32_t kLanes = 64;
constexpr uint32_t kThreads = 256;  // 4 waves per workgroup
constexpr uint32_t kWavesPer = kThreads / kLanes;

// Control block, in 64-bit words: entries per level table (one more word
// than levels: the last level's children slot), then per-level fills,
// splits and leaves and the overflow flag (the words read back for stats),
// then per level eight claim counters, one per XCD, each on a 128-byte line
// of its own.
constexpr uint32_t kCountW = 0;
constexpr uint32_t kFillW = 40;
constexpr uint32_t kSplitW = kFillW + ASK3_MAX_LEVELS;
constexpr uint32_t kLeafW = kSplitW + ASK3_MAX_LEVELS;
constexpr uint32_t kOverW = kLeafW + ASK3_MAX_LEVELS;
constexpr uint32_t kStatWords = kOverW + 8;
constexpr uint32_t kXcds = 8;         // claim counters per level: one per XCD of MI355X
constexpr uint32_t kLineWords = 16;   // 128 bytes
constexpr uint32_t kClaimW = 256;
constexpr uint32_t kCtrlWords = kClaimW + ASK3_MAX_LEVELS * kXcds * kLineWords;
constexpr uint64_t kTableOffset = kCtrlWords * 8 + 2048;  // 36864: 256-byte aligned
static_assert(kStatWords <= kClaimW && kTableOffset % 256 == 0, "control block layout");
constexpr uint32_t kMaxCoordBits = 21;  // per axis, so that a Morton scalar fits 63 bits

struct Vol3 {
    double cx, cy, cz, hx, hy, hz, cr, ci;
    uint32_t n[3];
    uint32_t D;
    uint32_t *out;
};

struct Level3 {
    const uint64_t *in;
    uint64_t *next;
    unsigned long long *ctrl;
    uint64_t G, cap;
    uint32_t r, B, curve, level;
};

__device__ __forceinline__ double axis_point(double centre, double half, uint32_t p, uint32_t n) {
    const int k = 2 * (int)p + 1 - (int)n;  // odd, |k| < 2^17: exact as int and as double
    const double t = (double)k * half;
    return centre + t;
}

__device__ __forceinline__ void put_voxel(const Vol3 &v, uint32_t x, uint32_t y, uint32_t z,
                                          uint32_t d) {
    v.out[((uint64_t)z * v.n[1] + y) * v.n[0] + x] = d;
}

// ---------------------------------------------------------------------------
// Voxel streams with lane refill. Voxels near the set's boundary have dwells
// that differ by orders of magnitude from their neighbours', so a wave that
// gives each lane one voxel waits for its slowest voxel with most lanes
// idle. Here every lane iterates its own voxel, and after every stretch of
// kStride3 iterations the lanes whose voxel has finished take the next
// voxels of the stream. A lane takes a voxel with its first two steps done
// and tested, and takes another at once when that voxel escaped there.
//
// The dwell: q <- q^2 + c with q = a + b i + e j, c = cr + ci i, the first k
// with |q_k|^2 > 4, else D; per step a' = (a^2 - (b^2 + e^2)) + cr,
// b' = (ab + ab) + ci, e' = (ae + ae) + 0, |q'|^2 = a'^2 + (b'^2 + e'^2),
// every operation rounded on its own. b^2 + e^2 is summed first, so e = 0
// performs the complex iteration's operations exactly, and it is kept for
// the next step. The "+ 0" of e's update is left out: it can only turn a -0
// into a +0, and e enters a, b and |q|^2 only through e^2 (and, as a
// factor, e's own update), so no dwell changes.
//
// A stretch runs without testing and then tests !(|q|^2 <= 4), which also
// catches inf and NaN. The quaternion norm is multiplicative, so
// |q'| >= |q|^2 - |c|: when |c|^2 <= 3.99, an orbit that once has
// |q|^2 > 4 grows at every later step (2 - |c| is far above the rounding),
// and a passing test proves that no escape happened inside the stretch. A
// failing test replays the stretch from its saved start, testing every
// step, which finds the same first k as a test after every iteration.
// Volumes with |c|^2 > 3.99 test after every iteration throughout.
// Iterations past D are harmless: an escape after D, or none by D, both
// give D.
//
// voxel_of(i, x, y, z) names voxel i of the stream (false: none there);
// done(x, y, z, dwell, surface) is called by the lane that finished a voxel,
// surface telling whether it was one of the first n_surf stream positions.
// A surface stream (kSurface) takes positions [0, n_surf) first and decides
// whether their dwells are all equal as it goes: once some voxel has
// finished with dwell v (the least of the first refill or stretch in which
// any finished), another finishing with a
// different dwell, or one still running after v iterations, shows the
// surface is mixed. It then stops (n_all ==
// n_surf), or (n_all > n_surf: a leaf box) goes on with the surface's other
// positions and then positions [n_surf, n_all), the box's inside. Returns
// 0 for a uniform surface (dwell v), 1 for a mixed one that stopped, 2 for a
// mixed one whose leaf was completed (and 2 for plain streams).
// ---------------------------------------------------------------------------
constexpr uint32_t kStride3 = 16;

// One step of the orbit; s2 = b^2 + e^2 of the new q.
__device__ __forceinline__ void quat_step(double &a, double &b, double &e, double &a2, double &s2,
                                          double cr, double ci) {
    const double ab = a * b, ae = a * e;
    a = (a2 - s2) + cr;
    b = (ab + ab) + ci;
    e = ae + ae;
    a2 = a * a;
    s2 = b * b + e * e;
}

// The surface decision of one wave alone: v is the wave's own.
struct SoloDecision {
    __device__ uint32_t propose(uint32_t v) const { return v; }
    __device__ bool known(uint32_t &) const { return false; }
    __device__ bool mixed() const { return false; }
    __device__ void set_mixed() const {}
};

template <bool kSurface, class VoxelOf, class Done, class Decision = SoloDecision>
__device__ __forceinline__ uint32_t quat_stream(const Vol3 &v, uint32_t n_surf, uint32_t n_all,
                                                VoxelOf voxel_of, Done done, uint32_t &val,
                                                Decision dec = Decision{}) {
    const uint32_t D = v.D;
    const double cr = v.cr, ci = v.ci;
    const bool special = !(cr * cr + ci * ci <= 3.99);  // the same for every voxel
    uint32_t next = 0;
    uint32_t n = kSurface ? n_surf : n_all;
    bool scanning = kSurface;
    bool have = false, vset = false, surf = false;
    uint32_t x = 0, y = 0, z = 0, k = 0;
    double a = 0.0, b = 0.0, e = 0.0, a2 = 0.0, s2 = 0.0;
    for (;;) {
        unsigned long long idle = __ballot(!have);
        // least and greatest dwell of the voxels this lane finished here
        uint32_t rlo = 0xffffffffu, rhi = 0u;
        while (idle && next < n) {
            if (!have) {
                const uint32_t j = next + (uint32_t)__builtin_amdgcn_mbcnt_hi(
                                              (uint32_t)(idle >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                if (j < n && voxel_of(j, x, y, z)) {
                    have = true;
                    surf = kSurface && j < n_surf;
                    a = axis_point(v.cx, v.hx, x, v.n[0]);
                    b = axis_point(v.cy, v.hy, y, v.n[1]);
                    e = axis_point(v.cz, v.hz, z, v.n[2]);
                    a2 = a * a;
                    s2 = b * b + e * e;
                    // The first two steps, tested here: most voxels of a
                    // volume lie outside the set and escape at once or at
                    // the next step, and such a lane takes its next voxel
                    // in the same refill instead of holding a whole stretch.
                    quat_step(a, b, e, a2, s2, cr, ci);
                    k = 1;
                    bool out = a2 + s2 > 4.0;
                    if (!out && D > 1) {
                        quat_step(a, b, e, a2, s2, cr, ci);
                        k = 2;
                        out = a2 + s2 > 4.0;
                    }
                    if (out || k >= D) {
                        done(x, y, z, k, surf);
                        have = false;
                        rlo = min(rlo, k);
                        rhi = max(rhi, k);
                    }
                }
            }
            next = min(n, next + (uint32_t)__popcll(idle));
            idle = __ballot(!have);
        }
        // A surface voxel finished here has dwell 1 or 2 (D, when D <= 2,
        // and then every voxel finishes here), below that of any voxel still
        // running: the least of them sets v when none is set yet, and then a
        // voxel still running, or one finished here with another dwell,
        // shows a mixed surface.
        if (kSurface && scanning && __ballot(rhi != 0)) {
            uint32_t lo = rlo, hi = rhi;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                lo = min(lo, (uint32_t)__shfl_xor((unsigned int)lo, o));
                hi = max(hi, (uint32_t)__shfl_xor((unsigned int)hi, o));
            }
            lo = __builtin_amdgcn_readfirstlane(lo);
            hi = __builtin_amdgcn_readfirstlane(hi);
            if (!vset) {
                val = dec.propose(lo);
                vset = true;
            }
            if (lo != val || hi != val || __ballot(have)) {
                dec.set_mixed();
                if (n_all == n_surf)
                    return 1;
                scanning = false;
                n = n_all;
                continue;
            }
        }
        if (__ballot(have) == 0)
            break;
        uint32_t dw = 0;
        bool fin = false;
        if (have) {
            bool replay = false;
            if (__builtin_expect(!special, 1)) {
                const double sa = a, sb = b, se = e, sa2 = a2, ss2 = s2;
#pragma unroll
                for (uint32_t u = 0; u < kStride3; ++u)
                    quat_step(a, b, e, a2, s2, cr, ci);
                if (!(a2 + s2 <= 4.0)) {
                    // Escapes are rare: an empty asm keeps the restore on a
                    // branch, so the common stretch pays no select per
                    // register of the state.
                    asm volatile("");
                    a = sa, b = sb, e = se, a2 = sa2, s2 = ss2;
                    replay = true;
                } else {
                    k += kStride3;
                }
            } else {
                // Kept rolled: unrolled, its sixteen exits hold enough scalar
                // registers to spill, and the spills lower the occupancy.
#pragma unroll 1
                for (uint32_t u = 0; u < kStride3; ++u) {
                    quat_step(a, b, e, a2, s2, cr, ci);
                    if (a2 + s2 > 4.0) {
                        dw = k + u + 1;
                        fin = true;
                        break;
                    }
                }
                if (!fin)
                    k += kStride3;
            }
            if (replay) {
                // the stretch again with a test after every step
                while (k < D) {
                    ++k;
                    quat_step(a, b, e, a2, s2, cr, ci);
                    if (a2 + s2 > 4.0)
                        break;
                }
                dw = k;
                fin = true;
            }
            if (!fin && k >= D) {
                dw = D;
                fin = true;
            }
            if (fin) {
                dw = dw > D ? D : dw;
                done(x, y, z, dw, surf);
                have = false;
            }
        }
        if (kSurface && scanning) {
            if (!vset && dec.known(val))
                vset = true;
            if (!vset && __ballot(fin)) {
                uint32_t m = fin ? dw : 0xffffffffu;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1)
                    m = min(m, (uint32_t)__shfl_xor((unsigned int)m, o));
                val = dec.propose(__builtin_amdgcn_readfirstlane(m));
                vset = true;
            }
            if ((vset && __ballot((fin && dw != val) || (have && k >= val))) || dec.mixed()) {
                dec.set_mixed();
                if (n_all == n_surf)
                    return 1;
                scanning = false;
                n = n_all;
            }
        }
    }
    return (kSurface && scanning) ? 0u : 2u;
}

// ---------------------------------------------------------------------------
// Space-filling curves over a level's G x G x G cells.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t spread3(uint32_t c) {
    uint64_t x = c & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

__host__ __device__ __forceinline__ uint32_t gather3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

__device__ __forceinline__ uint64_t cell_scalar(const uint32_t p[3], uint64_t G, uint32_t curve) {
    if (curve == ASK_CURVE_MORTON)
        return spread3(p[0]) | spread3(p[1]) << 1 | spread3(p[2]) << 2;
    return ((uint64_t)p[2] * G + p[1]) * G + p[0];
}

__device__ __forceinline__ void scalar_cell(uint64_t s, uint64_t G, uint32_t curve, uint32_t p[3]) {
    if (curve == ASK_CURVE_MORTON) {
        p[0] = gather3(s);
        p[1] = gather3(s >> 1);
        p[2] = gather3(s >> 2);
        return;
    }
    p[0] = (uint32_t)(s % G);
    s /= G;
    p[1] = (uint32_t)(s % G);
    p[2] = (uint32_t)(s / G);
}

__device__ __forceinline__ uint32_t cell_lo(uint64_t j, uint64_t G, uint32_t n) {
    return (uint32_t)(j * (uint64_t)n / G);
}

// Cell p of a G-grid as a box; false when it is empty or outside the grid.
__device__ __forceinline__ bool cell_box(const Vol3 &v, uint64_t G, const uint32_t p[3],
                                         uint32_t lo[3], uint32_t hi[3]) {
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ok = ok && (uint64_t)p[d] < G;
        lo[d] = cell_lo(p[d], G, v.n[d]);
        hi[d] = cell_lo((uint64_t)p[d] + 1, G, v.n[d]);
        ok = ok && lo[d] < hi[d] && hi[d] <= v.n[d];
    }
    return ok;
}

// Wave-wide values come from the first active lane through readfirstlane,
// which reads that lane whatever branch the optimiser puts the atomic in.
__device__ __forceinline__ bool first_lane3() {
    const uint32_t lane = __lane_id();
    return lane == __builtin_amdgcn_readfirstlane(lane);
}

__device__ __forceinline__ uint64_t uniform64_3(uint64_t x) {
    return (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32)) << 32 |
           __builtin_amdgcn_readfirstlane((uint32_t)x);
}

// One atomic add of the wave's count of set mask bits; every lane gets the
// counter's old value.
__device__ __forceinline__ uint64_t wave_base(unsigned long long *counter, uint64_t mask,
                                              uint32_t) {
    uint64_t base = 0;
    if (mask && first_lane3())
        base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    return uniform64_3(base);
}

// The XCD this wave runs on (HW_REG_XCC_ID). Only the claim order depends
// on it: every counter is drained by somebody whatever it reads.
__device__ __forceinline__ uint32_t xcd_id() {
    return __builtin_amdgcn_s_getreg((3 << 11) | 20) & (kXcds - 1);
}

// Items [0, n) claimed by the waves of a persistent grid: item i belongs to
// counter i mod kXcds (at counters[x * stride]), a wave drains its own
// XCD's counter `chunk` items per atomic add, then the others' in turn, and
// calls item(i) for every item it claimed. One counter address serves one
// atomic at a time (about 11 ns apart on MI355X), eight serve six times as
// many, and no wave starts past the last item.
template <class Item>
__device__ __forceinline__ void claim_items(unsigned long long *counters, uint32_t stride,
                                            uint64_t n, uint64_t chunk, Item item);

// One atomic add of n; every lane gets the counter's old value.
__device__ __forceinline__ uint64_t wave_claim(unsigned long long *counter, uint64_t n,
                                               uint32_t) {
    uint64_t base = 0;
    if (first_lane3())
        base = atomicAdd(counter, (unsigned long long)n);
    return uniform64_3(base);
}

template <class Item>
__device__ __forceinline__ void claim_items(unsigned long long *counters, uint32_t stride,
                                            uint64_t n, uint64_t chunk, Item item) {
    const uint32_t home = xcd_id();
    for (uint32_t q = 0; q < kXcds; ++q) {
        const uint32_t x = (home + q) & (kXcds - 1);
        const uint64_t mine = n > x ? (n - x + kXcds - 1) / kXcds : 0;  // items x, x + 8, ...
        for (;;) {
            const uint64_t k0 = wave_claim(&counters[x * stride], chunk, 0);
            if (k0 >= mine)
                break;
            const uint64_t k1 = std::min(k0 + chunk, mine);
            for (uint64_t k = k0; k < k1; ++k)
                item(x + k * kXcds);
        }
    }
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask, uint32_t lane) {
    return (uint32_t)__popcll(mask & ((1ull << lane) - 1));
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Every voxel: the volume is cut into columns of kTile3 x kTile3 x kCol3
// voxels, and the waves of a grid that the device holds at once claim them
// (per-XCD counters in the caller's workspace) and stream each column's
// voxels, slice by slice and row by row, lane refilled. Most voxels of a
// volume escape within a step or two, so a wave per column lives only a few
// microseconds, and the hardware then starts new waves far more slowly than
// they end (a wave trace showed 1 300 to 2 800 of the 8 192 wave slots in
// use); waves that stay and claim work keep every slot busy.
constexpr uint32_t kTile3 = 16;
constexpr uint32_t kCol3 = 2;
constexpr uint32_t kEx3Waves = 4;

__global__ __launch_bounds__(kEx3Waves * kLanes) void exhaustive3_kernel(Vol3 v, uint32_t tiles_x,
                                                                uint32_t tiles_y, uint32_t cols,
                                                                unsigned long long *counters) {
    claim_items(counters, kLineWords, cols, 1, [&](uint64_t c) {
        const uint32_t t = (uint32_t)c;
        const uint32_t rest = t / tiles_x;
        const uint32_t x0 = (t % tiles_x) * kTile3, y0 = (rest % tiles_y) * kTile3;
        const uint32_t z0 = (rest / tiles_y) * kCol3;
        uint32_t val = 0;
        quat_stream<false>(
            v, 0u, kTile3 * kTile3 * kCol3,
            [&](uint32_t i, uint32_t &x, uint32_t &y, uint32_t &zz) {
                x = x0 + i % kTile3;
                y = y0 + (i / kTile3) % kTile3;
                zz = z0 + i / (kTile3 * kTile3);
                return x < v.n[0] && y < v.n[1] && zz < v.n[2];
            },
            [&](uint32_t x, uint32_t y, uint32_t zz, uint32_t d, bool) { put_voxel(v, x, y, zz, d); },
            val);
    });
}

__global__ __launch_bounds__(kThreads) void clear3_kernel(unsigned long long *w, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += kThreads)
        w[i] = 0;
}

__global__ __launch_bounds__(kThreads) void reset3_kernel(unsigned long long *ctrl) {
    for (uint32_t i = threadIdx.x; i < kCtrlWords; i += kThreads)
        ctrl[i] = 0;
}

// Level 0: the non-empty cells of the g x g x g grid.
__global__ __launch_bounds__(kThreads) void seed3_kernel(Vol3 v, uint64_t *table,
                                                         unsigned long long *ctrl, uint32_t g,
                                                         uint32_t curve, uint64_t cap) {
    const uint32_t lane = threadIdx.x & (kLanes - 1);
    const uint64_t cells = (uint64_t)g * g * g;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t i0 = (uint64_t)blockIdx.x * kThreads + (threadIdx.x & ~(kLanes - 1));
         i0 < cells; i0 += stride) {
        const uint64_t i = i0 + lane;
        uint32_t p[3] = {0, 0, 0}, lo[3], hi[3];
        bool ok = false;
        if (i < cells) {
            p[0] = (uint32_t)(i % g);
            p[1] = (uint32_t)((i / g) % g);
            p[2] = (uint32_t)(i / ((uint64_t)g * g));
            ok = cell_box(v, g, p, lo, hi);
        }
        const uint64_t mask = __ballot(ok);
        const uint64_t base = wave_base(&ctrl[kCountW], mask, lane);
        if (ok) {
            const uint64_t at = base + lanes_below(mask, lane);
            if (at < cap)
                table[at] = cell_scalar(p, g, curve);
            else
                atomicOr(&ctrl[kOverW], 1ull);
        }
    }
}

// Division by a divisor fixed for a whole box (a side, a face, a ring):
// its binary64 reciprocal is taken once, and n * r, within a relative
// 2^-52 of n / d, truncates to the quotient or one off it, which the
// remainder corrects. Exact for n < 2^31 and 1 <= d < 2^31, in a few
// instructions instead of an integer division sequence per voxel.
struct Div {
    uint32_t d;
    double r;
    __device__ explicit Div(uint32_t d_) : d(d_), r(1.0 / (double)d_) {}
    __device__ __forceinline__ uint32_t div(uint32_t n) const {
        uint32_t q = (uint32_t)((double)n * r);
        const int32_t rem = (int32_t)(n - q * d);
        q = rem < 0 ? q - 1 : (rem >= (int32_t)d ? q + 1 : q);
        return q;
    }
};

// Voxel t of the surface of a w x h x l box: the two z faces, then the
// rectangular ring of each inner slice. A box with a side of 1 or 2 is all
// surface and is walked in storage order.
__host__ __device__ __forceinline__ uint32_t surface_count(uint32_t w, uint32_t h, uint32_t l) {
    if (w <= 2 || h <= 2 || l <= 2)
        return w * h * l;
    return 2 * w * h + (l - 2) * (2 * w + 2 * (h - 2));
}

struct Surface {
    uint32_t w, h, l, face;
    bool thin;
    Div dw, dh, dring;
    __device__ Surface(uint32_t w_, uint32_t h_, uint32_t l_)
        : w(w_), h(h_), l(l_), face(w_ * h_), thin(w_ <= 2 || h_ <= 2 || l_ <= 2), dw(w_),
          dh(h_), dring(thin ? 1u : 2 * w_ + 2 * (h_ - 2)) {}

    __device__ __forceinline__ void voxel(uint32_t t, uint32_t &x, uint32_t &y, uint32_t &z) const {
        if (thin) {
            const uint32_t row = dw.div(t);
            x = t - row * w;
            z = dh.div(row);
            y = row - z * h;
            return;
        }
        if (t < 2 * face) {
            z = t < face ? 0 : l - 1;
            t = t < face ? t : t - face;
            y = dw.div(t);
            x = t - y * w;
            return;
        }
        const uint32_t u = t - 2 * face;
        const uint32_t zi = dring.div(u);
        z = 1 + zi;
        const uint32_t q = u - zi * dring.d;
        if (q < w) {
            x = q, y = 0;
        } else if (q < 2 * w) {
            x = q - w, y = h - 1;
        } else {
            const uint32_t q2 = q - 2 * w;
            x = (q2 & 1) ? w - 1 : 0;
            y = 1 + q2 / 2;
        }
    }
};

// T: every voxel of the box (lo, w x h x l) takes dwell d, written by part
// `part` of `parts` waves. With w <= 64 the lanes hold a column x each and
// walk rows (y fastest, then z) 64 / w rows apart per wave, so no voxel
// needs a division.
__device__ void fill_box(const Vol3 &v, const uint32_t lo[3], uint32_t w, uint32_t h,
                         uint32_t l, uint32_t d, uint32_t lane, uint32_t part = 0,
                         uint32_t parts = 1) {
    if (w > kLanes) {
        for (uint32_t r = part; r < h * l; r += parts)
            for (uint32_t x = lane; x < w; x += kLanes)
                put_voxel(v, lo[0] + x, lo[1] + r % h, lo[2] + r / h, d);
        return;
    }
    const uint32_t rows = kLanes / w;
    const uint32_t x = lane % w;
    uint32_t y = lane / w, z = 0;
    if (y >= rows)
        return;
    y += part * rows;
    while (y >= h) {
        y -= h;
        ++z;
    }
    while (z < l) {
        put_voxel(v, lo[0] + x, lo[1] + y, lo[2] + z, d);
        y += rows * parts;
        while (y >= h) {
            y -= h;
            ++z;
        }
    }
}

// A box of a level table, decoded, with its surface order: the surface in a
// spread order, so that a mixed surface shows it early: A arcs of 2^bits
// voxels (A between 64 and 128 once the surface has 64 voxels or more), one
// voxel of every arc per round, at offsets taken in bit-reversed round order
// (0, 1/2, 1/4, 3/4, ... of an arc), so that only the last arc's tail names
// no voxel. Inside voxels are numbered in storage order.
struct Box {
    uint32_t p[3], lo[3];
    uint32_t w, h, l, S, bits, arcs, n_surf, iw, ih, inside;
    bool ok, leaf_size;
    Surface surf;
    Div darcs, diw, dih;

    __device__ static Box decode(const Vol3 &v, const Level3 &L, uint64_t scalar) {
        uint32_t p[3], lo[3], hi[3];
        scalar_cell(scalar, L.G, L.curve, p);
        const bool ok = cell_box(v, L.G, p, lo, hi);
        return Box(p, lo, ok ? hi[0] - lo[0] : 1u, ok ? hi[1] - lo[1] : 1u,
                   ok ? hi[2] - lo[2] : 1u, ok, L.B);
    }

    __device__ Box(const uint32_t p_[3], const uint32_t lo_[3], uint32_t w_, uint32_t h_,
                   uint32_t l_, bool ok_, uint32_t B)
        : w(w_), h(h_), l(l_), S(surface_count(w_, h_, l_)),
          bits(S >= 2 * kLanes ? 31u - (uint32_t)__builtin_clz(S / kLanes) : 0u),
          arcs((S + (1u << bits) - 1) >> bits), n_surf(arcs << bits),
          iw(w_ <= 2 || h_ <= 2 || l_ <= 2 ? 1u : w_ - 2),
          ih(w_ <= 2 || h_ <= 2 || l_ <= 2 ? 1u : h_ - 2),
          inside(w_ <= 2 || h_ <= 2 || l_ <= 2 ? 0u : (w_ - 2) * (h_ - 2) * (l_ - 2)), ok(ok_),
          leaf_size(w_ <= B && h_ <= B && l_ <= B), surf(w_, h_, l_), darcs(arcs), diw(iw),
          dih(ih) {
        for (int d = 0; d < 3; ++d) {
            p[d] = p_[d];
            lo[d] = lo_[d];
        }
    }

    // Surface position j of the spread order; false when it names no voxel.
    __device__ __forceinline__ bool surface_at(uint32_t j, uint32_t &x, uint32_t &y,
                                               uint32_t &z) const {
        const uint32_t round = darcs.div(j);
        const uint32_t off = bits ? __brev(round) >> (32u - bits) : 0u;
        const uint32_t t = ((j - round * arcs) << bits) + off;
        if (t >= S)
            return false;
        surf.voxel(t, x, y, z);
        x += lo[0];
        y += lo[1];
        z += lo[2];
        return true;
    }

    // Inside voxel t (t < inside).
    __device__ __forceinline__ void inside_at(uint32_t t, uint32_t &x, uint32_t &y,
                                              uint32_t &z) const {
        const uint32_t row = diw.div(t), zi = dih.div(row);
        x = lo[0] + 1 + (t - row * iw);
        y = lo[1] + 1 + (row - zi * ih);
        z = lo[2] + 1 + zi;
    }
};

// S: the non-empty children of box p go to the next level's table, one
// ballot and one atomic add per 64 children.
__device__ void emit_children(const Vol3 &v, const Level3 &L, const uint32_t p[3], uint32_t lane) {
    const uint32_t r = L.r, kids = r * r * r;
    const uint64_t G1 = L.G * r;
    for (uint32_t k0 = 0; k0 < kids; k0 += kLanes) {
        const uint32_t k = k0 + lane;
        uint32_t c[3] = {0, 0, 0}, clo[3], chi[3];
        bool ok = false;
        if (k < kids) {
            c[0] = p[0] * r + k % r;
            c[1] = p[1] * r + (k / r) % r;
            c[2] = p[2] * r + k / (r * r);
            ok = cell_box(v, G1, c, clo, chi);
        }
        const uint64_t mask = __ballot(ok);
        const uint64_t base = wave_base(&L.ctrl[kCountW + L.level + 1], mask, lane);
        if (ok) {
            const uint64_t at = base + lanes_below(mask, lane);
            if (at < L.cap)
                L.next[at] = cell_scalar(c, G1, L.curve);
            else
                atomicOr(&L.ctrl[kOverW], 1ull);
        }
    }
}

__device__ __forceinline__ void count_outcomes(const Level3 &L, unsigned long long nfill,
                                               unsigned long long nsplit,
                                               unsigned long long nleaf) {
    if (nfill)
        atomicAdd(&L.ctrl[kFillW + L.level], nfill);
    if (nsplit)
        atomicAdd(&L.ctrl[kSplitW + L.level], nsplit);
    if (nleaf)
        atomicAdd(&L.ctrl[kLeafW + L.level], nleaf);
}

// One level: each wave takes boxes from the level's table and decides them
// (surface uniform -> fill; every side <= B -> every voxel; else split).
// Every finished surface dwell is written: whatever follows, a voxel on a
// scanned surface ends with its own dwell, so a leaf box's stream goes on
// from its surface into its inside.
__global__ __launch_bounds__(kThreads) void level3_kernel(Vol3 v, Level3 L) {
    const uint32_t lane = threadIdx.x & (kLanes - 1);
    const uint64_t count = std::min((uint64_t)L.ctrl[kCountW + L.level], L.cap);
    // Entries per claim: one while the level has few boxes per wave (the best
    // balance), up to 64 when it has very many small ones, so that the
    // counters do not serialise the level.
    const uint64_t waves = (uint64_t)gridDim.x * kWavesPer;
    const uint64_t chunk = std::max<uint64_t>(1, std::min<uint64_t>(64, count / (waves * 16)));
    unsigned long long nfill = 0, nsplit = 0, nleaf = 0;
    claim_items(&L.ctrl[kClaimW + L.level * kXcds * kLineWords], kLineWords, count, chunk,
                [&](uint64_t e) {
        const Box bx = Box::decode(v, L, uniform64_3(L.in[e]));  // wave-uniform box
        if (!bx.ok) {
            if (lane == 0)
                atomicOr(&L.ctrl[kOverW], 2ull);
            return;
        }
        uint32_t first = 0;
        const uint32_t outcome = quat_stream<true>(
            v, bx.n_surf, bx.leaf_size ? bx.n_surf + bx.inside + 1u : bx.n_surf,
            [&](uint32_t j, uint32_t &x, uint32_t &y, uint32_t &z) {
                if (j < bx.n_surf)
                    return bx.surface_at(j, x, y, z);
                if (j - bx.n_surf >= bx.inside)
                    return false;
                bx.inside_at(j - bx.n_surf, x, y, z);
                return true;
            },
            [&](uint32_t x, uint32_t y, uint32_t z, uint32_t d, bool) { put_voxel(v, x, y, z, d); },
            first);
        if (outcome == 0) {
            fill_box(v, bx.lo, bx.w, bx.h, bx.l, first, lane);
            ++nfill;
        } else if (bx.leaf_size) {
            ++nleaf;
        } else {
            emit_children(v, L, bx.p, lane);
            ++nsplit;
        }
    });
    if (lane == 0)
        count_outcomes(L, nfill, nsplit, nleaf);
}

// The surface decision of a workgroup's waves sharing one box, in LDS: the
// first dwell proposed becomes v for all, and any wave that sees the surface
// mixed says so to the others.
constexpr uint32_t kNoVal = 0xffffffffu;

struct SharedDecision {
    uint32_t *val, *flag;
    __device__ uint32_t propose(uint32_t x) const {
        uint32_t old = kNoVal;
        if (first_lane3())
            old = atomicCAS(val, kNoVal, x);
        old = __builtin_amdgcn_readfirstlane(old);
        return old == kNoVal ? x : old;
    }
    __device__ bool known(uint32_t &x) const {
        const uint32_t y = __builtin_amdgcn_readfirstlane(*(volatile uint32_t *)val);
        if (y == kNoVal)
            return false;
        x = y;
        return true;
    }
    __device__ bool mixed() const {
        return __builtin_amdgcn_readfirstlane(*(volatile uint32_t *)flag) != 0;
    }
    __device__ void set_mixed() const {
        if (first_lane3())
            *(volatile uint32_t *)flag = 1u;
    }
};

// Levels of large boxes (kCoopSurface surface voxels or more): the four
// waves of a workgroup share one box. Each scans every fourth position of
// the surface order, and they decide the surface together through LDS (a
// mixed one stops every wave at its next round); then they fill the box
// together, stream a leaf box's inside together (the surface of a leaf box
// is always scanned whole), or one wave appends the children. A box's
// critical path is a quarter of one wave's.
constexpr uint32_t kCoopSurface = 1024;

__global__ __launch_bounds__(kThreads) void level3_coop_kernel(Vol3 v, Level3 L) {
    __shared__ unsigned long long sh_e;
    __shared__ uint32_t sh_val, sh_mixed;
    const uint32_t lane = threadIdx.x & (kLanes - 1), wave = threadIdx.x / kLanes;
    const uint64_t count = std::min((uint64_t)L.ctrl[kCountW + L.level], L.cap);
    unsigned long long *counters = &L.ctrl[kClaimW + L.level * kXcds * kLineWords];
    const SharedDecision dec{&sh_val, &sh_mixed};
    const uint32_t home = xcd_id();
    uint32_t q = 0;  // thread 0: the counter it claims from (home, then the others)
    unsigned long long nfill = 0, nsplit = 0, nleaf = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            unsigned long long e = ~0ull;
            while (q < kXcds) {
                const uint32_t x = (home + q) & (kXcds - 1);
                const uint64_t mine = count > x ? (count - x + kXcds - 1) / kXcds : 0;
                const uint64_t k = atomicAdd(&counters[x * kLineWords], 1ull);
                if (k < mine) {
                    e = x + k * kXcds;
                    break;
                }
                ++q;
            }
            sh_e = e;
            sh_val = kNoVal;
            sh_mixed = 0;
        }
        __syncthreads();
        const uint64_t e = uniform64_3(*(volatile unsigned long long *)&sh_e);
        if (e == ~0ull)
            break;
        const Box bx = Box::decode(v, L, uniform64_3(L.in[e]));
        if (bx.ok) {
            const uint32_t part = bx.n_surf > wave ? (bx.n_surf - wave + kWavesPer - 1) / kWavesPer : 0u;
            uint32_t vloc = 0;
            quat_stream<true>(
                v, part, bx.leaf_size ? part + 1u : part,
                [&](uint32_t i, uint32_t &x, uint32_t &y, uint32_t &z) {
                    return i < part && bx.surface_at(wave + i * kWavesPer, x, y, z);
                },
                [&](uint32_t x, uint32_t y, uint32_t z, uint32_t d, bool) { put_voxel(v, x, y, z, d); },
                vloc, dec);
        } else if (threadIdx.x == 0) {
            atomicOr(&L.ctrl[kOverW], 2ull);
        }
        __syncthreads();
        if (bx.ok) {
            const bool mixed = dec.mixed();
            uint32_t val = 0;
            dec.known(val);
            if (!mixed) {
                fill_box(v, bx.lo, bx.w, bx.h, bx.l, val, lane, wave, kWavesPer);
                ++nfill;
            } else if (bx.leaf_size) {
                const uint32_t part = bx.inside > wave ? (bx.inside - wave + kWavesPer - 1) / kWavesPer : 0u;
                uint32_t none = 0;
                quat_stream<false>(
                    v, 0u, part,
                    [&](uint32_t i, uint32_t &x, uint32_t &y, uint32_t &z) {
                        bx.inside_at(wave + i * kWavesPer, x, y, z);
                        return true;
                    },
                    [&](uint32_t x, uint32_t y, uint32_t z, uint32_t d, bool) { put_voxel(v, x, y, z, d); },
                    none);
                ++nleaf;
            } else {
                if (wave == 0)
                    emit_children(v, L, bx.p, lane);
                ++nsplit;
            }
        }
        __syncthreads();  // the LDS words are the next box's
    }
    if (threadIdx.x == 0)
        count_outcomes(L, nfill, nsplit, nleaf);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
bool volume_ok(const ask_volume *v) {
    if (!v)
        return false;
    const double c[8] = {v->x0, v->x1, v->y0, v->y1, v->z0, v->z1, v->cr, v->ci};
    for (double d : c)
        if (!std::isfinite(d))
            return false;
    if (!(v->x0 < v->x1 && v->y0 < v->y1 && v->z0 < v->z1))
        return false;
    const uint32_t n[3] = {v->W, v->H, v->L};
    for (uint32_t d : n)
        if (d < 1 || d > 65536)
            return false;
    // at most 2^31 voxels: the per-lane 32-bit voxel counters then never wrap
    return v->D >= 1 && (uint64_t)v->W * v->H * v->L <= (1ull << 31);
}

// Levels any box can reach: the first level whose cells all have sides <= B
// is the last; 0 when that takes more than ASK3_MAX_LEVELS levels or a grid
// wider than 2^21 cells.
uint32_t reachable_levels(const ask_volume *v, const ask3_params *p) {
    const uint32_t n = std::max(v->W, std::max(v->H, v->L));
    uint64_t G = p->g;
    for (uint32_t i = 0; i < ASK3_MAX_LEVELS; ++i) {
        if (G > (1ull << kMaxCoordBits))
            return 0;
        if ((n + G - 1) / G <= p->B)
            return i + 1;
        G *= p->r;
    }
    return 0;
}

bool params_ok(const ask_volume *v, const ask3_params *p) {
    if (!p || p->g < 1 || p->g > 1024 || p->r < 2 || p->r > 16 || p->B < 1 ||
        (p->curve != ASK_CURVE_CANONICAL && p->curve != ASK_CURVE_MORTON))
        return false;
    return reachable_levels(v, p) != 0;
}

uint64_t table_cap(const ask_volume *v, const ask3_params *p) {
    const uint64_t V = (uint64_t)v->W * v->H * v->L;
    const uint64_t level0 = (uint64_t)std::min(p->g, v->W) * std::min(p->g, v->H) *
                            std::min(p->g, v->L);
    const uint64_t r3 = (uint64_t)p->r * p->r * p->r;
    const uint64_t cap = std::min(V, std::max(level0, r3 * (V / ((uint64_t)p->B + 1))));
    return (cap + 31) / 32 * 32;
}

Vol3 make_vol(const ask_volume *v, uint32_t *out) {
    Vol3 o;
    o.cx = 0.5 * (v->x0 + v->x1);
    o.cy = 0.5 * (v->y0 + v->y1);
    o.cz = 0.5 * (v->z0 + v->z1);
    o.hx = (v->x1 - v->x0) / (2.0 * (double)v->W);
    o.hy = (v->y1 - v->y0) / (2.0 * (double)v->H);
    o.hz = (v->z1 - v->z0) / (2.0 * (double)v->L);
    o.cr = v->cr;
    o.ci = v->ci;
    o.n[0] = v->W, o.n[1] = v->H, o.n[2] = v->L;
    o.D = v->D;
    o.out = out;
    return o;
}

ask_status launched() {
    return hipGetLastError() == hipSuccess ? ASK_OK : ASK_EDEVICE;
}

}  // namespace

extern "C" ask_status ask3_validate(const ask_volume *v, const ask3_params *p) {
    if (!volume_ok(v))
        return ASK_EINVAL;
    if (p && !params_ok(v, p))
        return ASK_EINVAL;
    return ASK_OK;
}

extern "C" ask_status ask3_workspace_bytes(const ask_volume *v, const ask3_params *p,
                                           uint64_t *bytes) {
    if (!bytes || !volume_ok(v) || !params_ok(v, p))
        return ASK_EINVAL;
    *bytes = kTableOffset + 2 * table_cap(v, p) * sizeof(uint64_t);
    return ASK_OK;
}

extern "C" ask_status ask3_dwell_exhaustive(const ask_volume *v, uint32_t *d_out, void *d_work,
                                           uint64_t work_bytes, void *stream) {
    if (!volume_ok(v) || !d_out || !d_work || ((uintptr_t)d_work & 255) ||
        work_bytes < ASK3_EXHAUSTIVE_WORK_BYTES)
        return ASK_EINVAL;
    static_assert(kXcds * kLineWords * 8 <= ASK3_EXHAUSTIVE_WORK_BYTES, "exhaustive workspace");
    // at most 2^31 voxels, so fewer than 2^31 columns
    const uint32_t tx = (v->W + kTile3 - 1) / kTile3, ty = (v->H + kTile3 - 1) / kTile3;
    const uint64_t cols = (uint64_t)tx * ty * ((v->L + kCol3 - 1) / kCol3);
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        return ASK_EDEVICE;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, exhaustive3_kernel, kEx3Waves * kLanes,
                                                     0) != hipSuccess ||
        occ < 1) {
        (void)hipGetLastError();
        occ = 1;
    }
    const uint64_t blocks = std::min<uint64_t>((cols + kEx3Waves - 1) / kEx3Waves, (uint64_t)cus * occ);
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *counters = (unsigned long long *)d_work;
    hipLaunchKernelGGL(clear3_kernel, dim3(1), dim3(kThreads), 0, s, counters, kXcds * kLineWords);
    hipLaunchKernelGGL(exhaustive3_kernel, dim3((uint32_t)blocks), dim3(kEx3Waves * kLanes), 0, s,
                       make_vol(v, d_out), tx, ty, (uint32_t)cols, counters);
    return launched();
}

extern "C" ask_status ask3_dwell_subdiv(const ask_volume *v, const ask3_params *p,
                                        uint32_t *d_out, void *d_work, uint64_t work_bytes,
                                        void *stream, ask3_stats *stats) {
    uint64_t need = 0;
    if (!d_out || !d_work || ((uintptr_t)d_work & 255) ||
        ask3_workspace_bytes(v, p, &need) != ASK_OK || work_bytes < need)
        return ASK_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        return ASK_EDEVICE;
    // The level kernel's resident workgroups per CU: a grid larger than the
    // device holds at once would leave workgroups waiting for others to end.
    int occ = 0, occ_coop = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, level3_kernel, kThreads, 0) != hipSuccess ||
        occ < 1) {
        (void)hipGetLastError();
        occ = 1;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_coop, level3_coop_kernel, kThreads, 0) !=
            hipSuccess ||
        occ_coop < 1) {
        (void)hipGetLastError();
        occ_coop = 1;
    }
    const uint64_t cap = table_cap(v, p);
    const uint32_t levels = reachable_levels(v, p);
    unsigned long long *ctrl = (unsigned long long *)d_work;
    uint64_t *table[2] = {(uint64_t *)((char *)d_work + kTableOffset),
                          (uint64_t *)((char *)d_work + kTableOffset) + cap};
    const Vol3 vol = make_vol(v, d_out);
    hipLaunchKernelGGL(reset3_kernel, dim3(1), dim3(kThreads), 0, s, ctrl);
    const uint64_t cells = (uint64_t)p->g * p->g * p->g;
    const uint32_t seed_blocks = (uint32_t)std::min<uint64_t>((cells + kThreads - 1) / kThreads,
                                                              (uint64_t)cus * 16);
    hipLaunchKernelGGL(seed3_kernel, dim3(seed_blocks), dim3(kThreads), 0, s, vol, table[0], ctrl,
                       p->g, p->curve, cap);
    const uint64_t level0 = (uint64_t)std::min(p->g, v->W) * std::min(p->g, v->H) *
                            std::min(p->g, v->L);
    uint64_t G = p->g;
    for (uint32_t i = 0; i < levels; ++i, G *= p->r) {
        Level3 L;
        L.in = table[i & 1];
        L.next = table[(i + 1) & 1];
        L.ctrl = ctrl;
        L.G = G;
        L.cap = cap;
        L.r = p->r;
        L.B = p->B;
        L.curve = p->curve;
        L.level = i;
        const uint64_t bound = i == 0 ? level0 : cap;
        // The level's largest box: sides ceil(n / G) (floor partition).
        const uint32_t S_max = surface_count((uint32_t)((v->W + G - 1) / G),
                                             (uint32_t)((v->H + G - 1) / G),
                                             (uint32_t)((v->L + G - 1) / G));
        if (S_max >= kCoopSurface) {
            const uint32_t blocks = (uint32_t)std::max<uint64_t>(
                1, std::min<uint64_t>(bound, (uint64_t)cus * occ_coop));
            hipLaunchKernelGGL(level3_coop_kernel, dim3(blocks), dim3(kThreads), 0, s, vol, L);
        } else {
            const uint32_t blocks = (uint32_t)std::max<uint64_t>(
                1, std::min<uint64_t>((bound + kWavesPer - 1) / kWavesPer, (uint64_t)cus * occ));
            hipLaunchKernelGGL(level3_kernel, dim3(blocks), dim3(kThreads), 0, s, vol, L);
        }
    }
    ask_status st = launched();
    if (st != ASK_OK || !stats)
        return st;
    unsigned long long host[kStatWords];
    if (hipMemcpyAsync(host, ctrl, sizeof host, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return ASK_EDEVICE;
    *stats = ask3_stats{};
    for (uint32_t i = 0; i < levels; ++i) {
        const uint64_t n = std::min<uint64_t>(host[kCountW + i], cap);
        if (n == 0)
            break;
        stats->levels = i + 1;
        stats->regions[i] = n;
        stats->fills[i] = host[kFillW + i];
        stats->splits[i] = host[kSplitW + i];
        stats->leaves[i] = host[kLeafW + i];
    }
    stats->overflow = (uint32_t)host[kOverW];
    return stats->overflow ? ASK_EOVERFLOW : ASK_OK;
}
