// common.hpp -- internal definitions shared by the HIP sources of the walk
// engine: error reporting, the device graph view, the counter RNG, 128-bit
// multiply-high and wavefront (64-lane) primitives for CDNA.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/n2v.h"

namespace n2v {

constexpr uint32_t SENT = 0xFFFFFFFFu;
constexpr int WAVE = 64;
// Pair sketches.  A sketch of the move (t -> v) at a hub v splits N(v) into
// at most MEMO_SEGS segments of whole 512-entry tiles (nsup of them) and
// holds, per segment, one plus the number of members of N(t) in the segment
// (0 = not known yet), then per segment a start hint into N(t), then one plus
// the count in the segment's first half: three u16 arrays of nsp entries
// each, nsp = nsup rounded up to even (memo_segs).  Rows of weighted graphs
// append, as u32, per segment the weight sum of its members of N(t), the same
// over its first half, the weight sum of all its entries and the same over
// its first half.  Each row is sized for its own vertex: memo_row_words u16
// words for a vertex of degree d, a whole number of 4-byte words.
constexpr int MEMO_SEGS = 64;
__host__ __device__ inline uint32_t memo_segs(uint64_t d)
{
    const uint64_t tiles = (d + 511) / 512;
    const uint64_t per = tiles > 0 ? (tiles + MEMO_SEGS - 1) / MEMO_SEGS : 1;  // tiles per segment
    const uint32_t nsup = (uint32_t)((tiles + per - 1) / per);
    return (nsup + 1) & ~1u;
}
__host__ __device__ inline uint32_t memo_row_words(bool weighted, uint64_t d)
{
    return (weighted ? 11u : 3u) * memo_segs(d);
}
// Sketches serve rows of at most this degree: 127 tiles of 512 entries per
// segment, so count + 1 always fits the u16 entries (and a segment's weight
// sum, at most 65024 x 65535, a u32).
constexpr uint32_t MEMO_MAX_DEG = 127u * 512u * MEMO_SEGS;
// Walk counters a graph hands out round-robin to persistent launches: up to
// this many launches on one graph may overlap.
constexpr int CURSOR_SLOTS = 64;
constexpr int CURSOR_STRIDE = 64;  // words between counters (one per 256 bytes)

// ---------------------------------------------------------------- errors
int set_error(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

// Host bookkeeping of a graph's walk-counter slots (walk.hip).
void *cursor_slots_new();
void cursor_slots_free(void *slots);

#define N2V_HIP(call)                                              \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return ::n2v::hip_fail(e_, #call);   \
    } while (0)

// ------------------------------------------------------------ graph view
// Per-vertex record: row offset, degree and largest weight of the row.
// One 16-byte aligned load gives everything a move needs about a vertex.
struct alignas(16) VRec {
    uint64_t off;
    uint32_t deg;
    uint32_t wmax;
};

struct DevGraph {
    const VRec *vrec;      // n
    const uint2 *erec;     // m: (neighbour x, position of the reverse entry in N(x) or SENT)
    const uint32_t *adj;   // m, rows strictly ascending
    const uint16_t *wt;    // m, or null for an unweighted graph
    const uint64_t *wsum;  // n: row weight sums (weighted graphs only)
    const uint64_t *hbase; // n+1: u16 word offset of the sketch rows of each vertex of degree >= memo_min
    uint16_t *memo;        // pair sketches (hbase[n] u16 words; deg(v) rows of memo_row_words each) or null
    uint32_t *status;      // device flags: bit 0 = a start id was out of range
    uint32_t *cursors;     // CURSOR_SLOTS walk counters, one per concurrent call
    uint32_t n;
    uint64_t m;
    uint32_t d_rule;
    uint32_t memo_min;     // vertices of at least this degree (> d_rule) have sketch rows
    uint32_t a_cap;
    uint32_t wlo, whi;     // smallest and largest edge weight of the graph (1, 1 unweighted)
};

// ------------------------------------------------------------ counter RNG
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
struct R4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ R4 philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                                     uint32_t c3)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return R4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint64_t hi64(uint64_t x, uint64_t y) { return __umul64hi(x, y); }

__device__ __forceinline__ uint64_t join64(uint32_t hi, uint32_t lo)
{
    return ((uint64_t)hi << 32) | lo;
}

// --------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// LDS written by some lanes of a wave becomes visible to the other lanes.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t shfl32(uint32_t v, int src) { return __shfl(v, src, WAVE); }

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    uint32_t lo = __shfl((uint32_t)v, src, WAVE);
    uint32_t hi = __shfl((uint32_t)(v >> 32), src, WAVE);
    return join64(hi, lo);
}

__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, int d)
{
    uint32_t lo = __shfl_up((uint32_t)v, d, WAVE);
    uint32_t hi = __shfl_up((uint32_t)(v >> 32), d, WAVE);
    return join64(hi, lo);
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m)
{
    uint32_t lo = __shfl_xor((uint32_t)v, m, WAVE);
    uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, WAVE);
    return join64(hi, lo);
}

// Lane l - (shift) within its row of 16 (row_shr), or the last lane of the
// previous row (row_bcast:15) / of lanes 0..31 (row_bcast:31), by DPP; lanes
// the pattern leaves out, or whose rows are masked off, read 0.  These are
// register-to-register moves, with none of the LDS latency of a permute.
// They read every lane's register, so callers keep all 64 lanes active.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint32_t dpp0(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, true);
}

template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint64_t dpp0_64(uint64_t v)
{
    return join64(dpp0<CTRL, ROWS>((uint32_t)(v >> 32)), dpp0<CTRL, ROWS>((uint32_t)v));
}

// Inclusive prefix sums over the 64 lanes (Hillis-Steele within rows of 16,
// then the row totals carried across rows).
__device__ __forceinline__ uint32_t wave_incl_scan32(uint32_t v)
{
    v += dpp0<0x111>(v);        // row_shr:1
    v += dpp0<0x112>(v);        // row_shr:2
    v += dpp0<0x114>(v);        // row_shr:4
    v += dpp0<0x118>(v);        // row_shr:8
    v += dpp0<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp0<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v)
{
    v += dpp0_64<0x111>(v);
    v += dpp0_64<0x112>(v);
    v += dpp0_64<0x114>(v);
    v += dpp0_64<0x118>(v);
    v += dpp0_64<0x142, 0xa>(v);
    v += dpp0_64<0x143, 0xc>(v);
    return v;
}

// Wave-uniform values live in scalar registers.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t uni64(uint64_t v)
{
    return join64(__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)), __builtin_amdgcn_readfirstlane((uint32_t)v));
}

// Value of lane `src` (uniform) in a scalar register.
__device__ __forceinline__ uint32_t lane_val(uint32_t v, int src) { return __builtin_amdgcn_readlane(v, src); }

__device__ __forceinline__ uint64_t lane_val64(uint64_t v, int src)
{
    return join64(__builtin_amdgcn_readlane((uint32_t)(v >> 32), src), __builtin_amdgcn_readlane((uint32_t)v, src));
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) { return lane_val64(wave_incl_scan(v), WAVE - 1); }

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) { return lane_val(wave_incl_scan32(v), WAVE - 1); }

__device__ __forceinline__ int first_lane(uint64_t mask) { return __ffsll((unsigned long long)mask) - 1; }

// Lower bound of x in a[lo, hi) (global memory); returns the index.
__device__ __forceinline__ uint64_t lower_bound_g(const uint32_t *__restrict__ a, uint64_t lo, uint64_t hi,
                                                  uint32_t x)
{
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool contains_g(const uint32_t *__restrict__ a, uint64_t lo, uint64_t hi, uint32_t x)
{
    const uint64_t p = lower_bound_g(a, lo, hi, x);
    return p < hi && a[p] == x;
}

}  // namespace n2v

// Host-side graph handle.
struct n2v_graph {
    n2v::DevGraph dg;
    const uint64_t *off;
    int weighted;
    int validate;
    int device;
    bool has_tuned;
    n2v_exec_opts tuned;
    uint64_t hub_words;     // sketch words of the rows of degree > d_rule
    uint64_t hub_entries;   // entries of the rows of degree > d_rule
    uint64_t memo_words;    // sketch words of the rows of degree >= dg.memo_min
    void *scan;             // scan scratch of the graph's workspace
    unsigned long long *hist;  // 64 words of the graph's workspace for degree statistics
    uint32_t next_cursor;   // next walk-counter slot to try
    size_t memo_bytes;      // attached sketch memory (0: none)
    int servers;            // servers created on this graph and not yet destroyed
    void *slots;            // walk-counter slot bookkeeping (host; see walk.hip)
};
