// walk.hip -- node2vec second-order walk kernels.
//
// A move from v (previous vertex t) draws the next vertex x with probability
// proportional to pi_x = w_vx * A(t, x), A = A_ret (x = t), A_com (x a
// neighbour of t), A_out (otherwise): the model of Section 2.1 of the paper
// with the probabilities computed on demand as in Section 3.2, never stored.
// The first move uses the edge weights alone (Algorithm 1).
//
// Execution classes (all give bit-identical results; they only decide who
// evaluates the rule):
//   thread  -- one lane runs a rejection move of its own walk;
//   wave    -- 64 lanes evaluate 64 rejection attempts at once and keep the
//              lowest accepting attempt index;
//   hub     -- a wavefront evaluates the inverse CDF of a high-degree vertex:
//              it intersects N(v) with N(t), forms S = sum pi, draws
//              r = hi64(R1, S) and finds the first prefix sum above r, by a
//              chunked merge-intersection staged in LDS (dense) or by
//              searching the members of a short N(t) in N(v) (sparse).
//
// Forms: PLAIN = one superstep per move (a thread kernel plus a hub kernel
// with one workgroup per hub move, as a BSP superstep advances every walk by
// one move); PERSISTENT = one launch, each wavefront owns 64 walk slots and
// switches between thread and wave classes.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "prims.hpp"
#include "walk.hpp"

namespace n2v {

constexpr uint32_t A_COM = 4;

// Walk state carried from move to move.
struct WS {
    uint32_t job;    // job the walk belongs to
    uint32_t i;      // index of the walk within its job (row of out)
    uint32_t s;      // moves taken so far
    uint32_t v, t;   // current and previous vertex
    uint64_t vo;     // row offset of v
    uint32_t vd, vw; // degree and largest weight of v
    uint64_t to;     // row offset of t
    uint32_t td;     // degree of t
    uint32_t pos_t;  // index of t in N(v), SENT if absent
    uint32_t jprev;  // index of v in N(t)
    uint64_t hb;     // first sketch row of v when loaded with v's record (hub moves), else ~0
};

namespace {

constexpr int HCH = 256;            // weighted scan chunk: 4 entries per lane
constexpr int HEPL = HCH / WAVE;
constexpr int TX = 512;             // dense merge: N(v) tile, 8 entries per lane
constexpr int XPL = TX / WAVE;
static_assert(XPL == 8, "a lane's run of tile flags is read as one u64");
constexpr int YPL = 8;              // dense merge: later N(t) blocks of 8 x 64 entries
constexpr int YFIRST = 4;           // entries per lane of the first N(t) block of a tile
constexpr int NSUPER = MEMO_SEGS;   // segments (sums) per hub row
constexpr int SPCAP = 1024;         // specials (positions) held by the sparse path
constexpr int NPIV = 256;           // pivots of an N(t) range that N(v) entries are searched in

// LDS of one wavefront for hub moves (5.5 KiB).
struct HubLds {
    union {
        struct {
            uint32_t xs[TX];
            uint8_t flag[TX];
            uint32_t rc[NSUPER];  // reverse sketch: members of N(v) per segment of N(t)
            uint32_t rh[NSUPER];  // reverse sketch: encoded start hints
            uint32_t r1[NSUPER];  // reverse sketch: members in each segment's first half
        } d;
        struct {
            uint32_t pos[SPCAP];
        } sp;
    } a;
    union {
        uint64_t csum[NSUPER];
    } b;
    union {
        int32_t dl[HCH];     // weighted scan deltas, sparse sketch counts
        uint32_t piv[NPIV];  // pivots for searching N(v) entries in N(t)
    } c;
};

// Lower bound of x in row[0, n) found by the whole wavefront: each round the
// 64 lanes probe the last entry of 64 equal buckets, so a search over n
// entries takes about log_64(n) + 1 dependent loads instead of log_2(n).
__device__ uint32_t wave_lower_bound(const uint32_t *__restrict__ row, uint32_t n, uint32_t x)
{
    const int l = lane_id();
    uint32_t lo = 0, hi = n;
    while (hi - lo > (uint32_t)WAVE) {
        const uint32_t step = (hi - lo + WAVE - 1) / WAVE;
        uint32_t p = lo + (uint32_t)(l + 1) * step - 1;
        if (p > hi - 1) p = hi - 1;
        const uint64_t m = ballot(row[p] >= x);
        if (m == 0) return hi;
        const int f = first_lane(m);
        const uint32_t nhi = lo + (uint32_t)(f + 1) * step;
        lo = lo + (uint32_t)f * step;
        hi = nhi < hi ? nhi : hi;
    }
    const uint32_t p = lo + l;
    const uint64_t m = ballot(p < hi && row[p] >= x);
    return m ? lo + first_lane(m) : hi;
}

// The state of lane o in scalar registers.
__device__ __forceinline__ WS bcast(const WS &s, int o)
{
    WS w;
    w.job = lane_val(s.job, o);
    w.i = lane_val(s.i, o);
    w.s = lane_val(s.s, o);
    w.v = lane_val(s.v, o);
    w.t = lane_val(s.t, o);
    w.vo = lane_val64(s.vo, o);
    w.vd = lane_val(s.vd, o);
    w.vw = lane_val(s.vw, o);
    w.to = lane_val64(s.to, o);
    w.td = lane_val(s.td, o);
    w.pos_t = lane_val(s.pos_t, o);
    w.jprev = lane_val(s.jprev, o);
    w.hb = lane_val64(s.hb, o);
    return w;
}

__device__ __forceinline__ WS uniform_ws(const WS &s) { return bcast(s, 0); }

__device__ __forceinline__ uint32_t amax3(const JobCtx &J)
{
    uint32_t m = J.A_ret > A_COM ? J.A_ret : A_COM;
    return m > J.A_out ? m : J.A_out;
}

template <bool WALKS, bool COUNTS>
__device__ __forceinline__ void emit(const JobCtx &J, uint32_t i, uint32_t col, uint32_t x, uint64_t &csum)
{
    if (WALKS) J.out[(uint64_t)i * (J.L + 1) + col] = x;
    if (COUNTS) {
        atomicAdd(&J.cnt[x], 1u);
        const R4 h = philox(J.k0, J.k1, J.wbase + i, col, x, 3u);
        csum += join64(h.x, h.y);
    }
}

// v's record; a hub move also takes v's first sketch row in the same round
// trip, which its sketch lookup would otherwise wait for
template <bool HUB = false>
__device__ __forceinline__ void load_v(const Exec &E, WS &st, uint32_t x)
{
    const VRec r = E.g.vrec[x];
    st.hb = HUB && E.g.memo ? E.g.hbase[x] : ~0ull;
    st.v = x;
    st.vo = r.off;
    st.vd = r.deg;
    st.vw = r.wmax;
}

// Neighbour index j of v -> (x, position of v in N(x)).
__device__ __forceinline__ void resolve(const Exec &E, const WS &st, uint32_t j, uint32_t &x, uint32_t &rev)
{
    if (st.s > 0 && j == st.pos_t) {
        x = st.t;
        rev = st.jprev;
    } else {
        const uint2 e = E.g.erec[st.vo + j];
        x = e.x;
        rev = e.y;
    }
}

template <bool HUB = false>
__device__ __forceinline__ void advance(const Exec &E, WS &st, uint32_t j, uint32_t x, uint32_t rev)
{
    st.t = st.v;
    st.to = st.vo;
    st.td = st.vd;
    st.jprev = j;
    st.pos_t = rev;
    load_v<HUB>(E, st, x);
    st.s += 1;
}

// Rejection attempt k up to the membership test: the proposal j and, unless
// the outcome is already forced, the proposal x and the acceptance draw u
// against A * w (A = A_COM if x is a neighbour of t, else A_out).  Returns
// 1 (accept), 0 (reject) or 2 (the test is needed).
struct Att {
    uint32_t j, x;
    uint64_t u, w;
};

__device__ __forceinline__ int attempt_pre(const Exec &E, const JobCtx &J, const WS &st, uint32_t k, Att &a)
{
    const bool first = st.s == 0;
    const uint64_t E_env = (uint64_t)st.vw * (first ? 1u : amax3(J));
    const R4 r = philox(J.k0, J.k1, J.wbase + st.i, st.s, k, 0u);
    const uint64_t j = hi64(join64(r.x, r.y), st.vd);
    a.j = (uint32_t)j;
    a.u = hi64(join64(r.z, r.w), E_env);
    a.w = E.g.wt ? E.g.wt[st.vo + j] : 1u;
    const uint32_t acmin = A_COM < J.A_out ? A_COM : J.A_out;
    const uint32_t acmax = A_COM < J.A_out ? J.A_out : A_COM;
    if (first) return a.u < a.w;
    if (j == st.pos_t) return a.u < J.A_ret * a.w;
    if (a.u < acmin * a.w) return 1;
    if (a.u >= acmax * a.w) return 0;
    a.x = E.g.adj[st.vo + j];
    return 2;
}

// One rejection attempt k; returns whether it accepts and its neighbour index.
__device__ __forceinline__ bool attempt(const Exec &E, const JobCtx &J, const WS &st, uint32_t k, uint32_t &j_out)
{
    Att a;
    const int r = attempt_pre(E, J, st, k, a);
    j_out = a.j;
    if (r < 2) return r == 1;
    const bool com = contains_g(E.g.adj, st.to, st.to + st.td, a.x);
    return a.u < (uint64_t)(com ? A_COM : J.A_out) * a.w;
}

// x in the sorted LDS array T[0, n): a branchless lower bound (the bound lies
// in [p, p + len - 1] throughout), then one compare.
__device__ __forceinline__ bool lds_contains(const uint32_t *T, uint32_t n, uint32_t x)
{
    const uint32_t *q = T;
    for (uint32_t len = n; len > 1; len -= len >> 1) {
        const uint32_t half = len >> 1;
        q += q[half - 1] < x ? half : 0u;
    }
    return n > 0 && *q == x;
}

// Thread class: attempts in order until one accepts (false after a_cap, or
// after the first kmax attempts).
__device__ bool thread_reject(const Exec &E, const JobCtx &J, const WS &st, uint32_t &j_out,
                              uint32_t kmax = 0xFFFFFFFFu)
{
    const uint32_t n = kmax < E.g.a_cap ? kmax : E.g.a_cap;
    for (uint32_t k = 0; k < n; ++k)
        if (attempt(E, J, st, k, j_out)) return true;
    return false;
}

// Wave class: lanes take attempts k0 + lane (from attempt kfrom on, the
// earlier ones having rejected); the lowest accepting one wins.
// When some attempt needs "is x a neighbour of t?" and N(t) fits, the wave
// stages N(t) in LDS once (one coalesced read) and searches it there.
__device__ bool wave_reject(const Exec &E, const JobCtx &J, const WS &st_in, HubLds &L, uint32_t &j_out,
                            uint32_t kfrom = 0)
{
    const WS st = uniform_ws(st_in);
    const int l = lane_id();
    bool staged = false;
    for (uint32_t k0 = kfrom; k0 < E.g.a_cap; k0 += WAVE) {
        const uint32_t k = k0 + l;
        Att a;
        a.j = 0;
        const int r = k < E.g.a_cap ? attempt_pre(E, J, st, k, a) : 0;
        bool acc = r == 1;
        if (ballot(r == 2)) {
            if (!staged && st.td <= (uint32_t)SPCAP) {
                for (uint32_t i = l; i < st.td; i += WAVE) L.a.sp.pos[i] = E.g.adj[st.to + i];
                wave_lds_sync();
                staged = true;
            }
            if (r == 2) {
                const bool com = staged ? lds_contains(L.a.sp.pos, st.td, a.x)
                                        : contains_g(E.g.adj, st.to, st.to + st.td, a.x);
                acc = a.u < (uint64_t)(com ? A_COM : J.A_out) * a.w;
            }
        }
        const uint64_t m = ballot(acc);
        if (m) {
            j_out = lane_val(a.j, first_lane(m));
            wave_lds_sync();
            return true;
        }
    }
    wave_lds_sync();
    return false;
}

// ------------------------------------------------------------------ hubs
// Sketch rows (nsp = memo_segs(deg v) entries per array): counts (one plus
// the number of members of N(t) in a segment of N(v); 0 = unknown), then
// start hints: hint h > 0 of a
// segment says that its merge may start streaming N(t) at index
// (h - 1) << hint_shift(deg t), which is at or below the lower bound in N(t)
// of the segment's first entry (so the skipped entries cannot match).
__device__ __forceinline__ uint32_t hint_shift(uint32_t d)
{
    const uint32_t b = 32 - __clz(d);
    return b > 15 ? b - 15 : 0;
}

// The sketch of the reverse pair (t, index of v in N(t)) that a merge of N(v)
// with N(t) also yields: counts of common entries per segment of N(t) and,
// for each segment's first entry, its lower bound in N(v) as a start hint.
struct RevSketch {
    uint32_t rseg;   // segment length of N(t); 0: not collected
    uint32_t nsp;    // entries per array of t's sketch row (memo_segs(deg t))
    uint32_t shift;  // hint_shift(deg v)
    uint32_t *rc;    // LDS counts
    uint32_t *rh;    // LDS encoded hints
    uint32_t *r1;    // LDS counts in each segment's first half
};

// Flags the tile entries equal to a block of NB x 64 entries of N(t) loaded
// from ypos; returns how many block entries lie in the tile's value range
// (they form a prefix of the block, N(t) being sorted).  The lower bounds in
// the tile are found by branchless searches that advance SEARCH_ILP entries
// per lane in lockstep, so their LDS reads overlap instead of each probe
// waiting for the previous one.
constexpr int SEARCH_ILP = 4;

template <int NB>
__device__ __forceinline__ uint32_t flag_block(HubLds &L, const uint32_t (&y)[NB], uint32_t ypos, uint32_t td,
                                               uint32_t j0, uint32_t cnt, uint32_t xlast, const RevSketch &R)
{
    static_assert(NB % SEARCH_ILP == 0, "blocks are searched SEARCH_ILP entries per lane at a time");
    const int l = lane_id();
    uint32_t nin = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) nin += __popcll(ballot(ypos + b * WAVE + l < td && y[b] <= xlast));
#pragma unroll
    for (int g = 0; g < NB; g += SEARCH_ILP) {
        if ((uint32_t)(g * WAVE) >= nin) break;  // the rest of the block lies beyond the tile
        // the probes walk LDS pointers, so each address is the pointer plus
        // an immediate offset
        const uint32_t *q[SEARCH_ILP];
#pragma unroll
        for (int k = 0; k < SEARCH_ILP; ++k) q[k] = L.a.d.xs;
#pragma unroll
        for (uint32_t step = TX / 2; step >= 1; step >>= 1) {
#pragma unroll
            for (int k = 0; k < SEARCH_ILP; ++k) q[k] += q[k][step - 1] < y[g + k] ? step : 0u;
        }
        uint32_t pos[SEARCH_ILP];
#pragma unroll
        for (int k = 0; k < SEARCH_ILP; ++k) pos[k] = (uint32_t)(q[k] - L.a.d.xs);
#pragma unroll
        for (int k = 0; k < SEARCH_ILP; ++k) {
            const uint32_t idx = ypos + (g + k) * WAVE + l;
            const bool in = idx < td && y[g + k] <= xlast;
            const bool hit = in && pos[k] < cnt && L.a.d.xs[pos[k]] == y[g + k];
            if (hit) L.a.d.flag[pos[k]] = 1;
            if (R.rseg && in && (hit || (idx & (TX - 1)) == 0)) {
                const uint32_t q = idx / R.rseg;
                if (hit) {
                    atomicAdd(&R.rc[q], 1u);
                    if (idx - q * R.rseg < R.rseg / 2) atomicAdd(&R.r1[q], 1u);
                }
                if (idx == q * R.rseg) R.rh[q] = ((j0 + pos[k]) >> R.shift) + 1;
            }
        }
    }
    return nin;
}

// Stages N(v)[j0, j0+cnt) (cnt <= TX) in LDS and flags the members of N(t),
// streaming N(t) from ypos (advanced past every value <= the tile's last
// entry).  The tile and a first, small block of N(t) are loaded together
// (most windows are short); a block consumed entirely is followed by
// full-size blocks.  Returns the number of flagged entries, plus 2^16 times
// the number among the tile's first 256 entries.
__device__ uint32_t dense_flags(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Y, uint32_t td,
                                HubLds &L, uint32_t j0, uint32_t cnt, uint32_t &ypos, const RevSketch &R)
{
    const int l = lane_id();
    uint32_t xv[XPL], y0[YFIRST];
#pragma unroll
    for (int e = 0; e < XPL; ++e) {
        const uint32_t i = e * WAVE + l;
        xv[e] = i < cnt ? X[j0 + i] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int b = 0; b < YFIRST; ++b) {
        const uint32_t idx = ypos + b * WAVE + l;
        y0[b] = idx < td ? Y[idx] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int e = 0; e < XPL; ++e) L.a.d.xs[e * WAVE + l] = xv[e];
    *(uint64_t *)&L.a.d.flag[l * XPL] = 0;
    wave_lds_sync();
    const uint32_t xlast = L.a.d.xs[cnt - 1];
    uint32_t nin = flag_block<YFIRST>(L, y0, ypos, td, j0, cnt, xlast, R);
    ypos += nin;
    if (nin == YFIRST * WAVE) {
        while (ypos < td) {
            uint32_t y[YPL];
#pragma unroll
            for (int b = 0; b < YPL; ++b) {
                const uint32_t idx = ypos + b * WAVE + l;
                y[b] = idx < td ? Y[idx] : 0xFFFFFFFFu;
            }
            nin = flag_block<YPL>(L, y, ypos, td, j0, cnt, xlast, R);
            ypos += nin;
            if (nin < YPL * WAVE) break;
        }
    }
    wave_lds_sync();
    // flags are 0/1 bytes: the byte sum of the lane's eight; lanes 0..31 hold
    // the tile's first 256 entries
    const uint64_t f8 = *(const uint64_t *)&L.a.d.flag[l * XPL];
    const uint32_t c = (uint32_t)((f8 * 0x0101010101010101ull) >> 56);
    return wave_sum32(l < WAVE / 2 ? c | (c << 16) : c);
}

// np (a power of two, 64..NPIV) pivots of Y[ylo, yhi) in LDS: bucket k is
// Y[ylo + kB, min(ylo + (k+1)B, yhi)) with B = ceil((yhi - ylo) / np), and
// piv[k] is its last entry (0xFFFFFFFF for an empty bucket), so the only
// bucket that can hold a value x is the first k with piv[k] >= x.  Returns B.
__device__ uint32_t load_pivots(const uint32_t *__restrict__ Y, uint32_t ylo, uint32_t yhi, HubLds &L, uint32_t np)
{
    const int l = lane_id();
    const uint32_t ny = yhi - ylo;
    const uint32_t B = (ny + np - 1) / np;
    for (uint32_t k = l; k < np; k += WAVE) {
        const uint64_t lo = (uint64_t)k * B, hi = lo + B < ny ? lo + B : ny;
        L.c.piv[k] = lo < ny ? Y[ylo + hi - 1] : 0xFFFFFFFFu;
    }
    wave_lds_sync();
    return B;
}

// Pivot count for searching n values: about one per value, 64..NPIV.
__device__ __forceinline__ uint32_t pivots_for(uint32_t n)
{
    uint32_t np = WAVE;
    while (np < (uint32_t)NPIV && np < n) np <<= 1;
    return np;
}

// Bucket of x among np pivots (number of pivots below x, 0..np), SEARCH_ILP
// values per lane in lockstep.
__device__ __forceinline__ void pivot_buckets(const HubLds &L, uint32_t np, const uint32_t (&x)[SEARCH_ILP],
                                              uint32_t (&p)[SEARCH_ILP])
{
    const uint32_t *q[SEARCH_ILP];
#pragma unroll
    for (int k = 0; k < SEARCH_ILP; ++k) q[k] = L.c.piv;
    for (uint32_t step = np >> 1; step >= 1; step >>= 1) {
#pragma unroll
        for (int k = 0; k < SEARCH_ILP; ++k) q[k] += q[k][step - 1] < x[k] ? step : 0u;
    }
#pragma unroll
    for (int k = 0; k < SEARCH_ILP; ++k) p[k] = (uint32_t)(q[k] - L.c.piv) + (q[k][0] < x[k] ? 1u : 0u);
}

// Flags the members of N(t) in the tile N(v)[j0, j0+cnt) by searching each
// entry in Y[ylo, yhi) (which must hold every match; pivots of B entries per
// bucket in LDS): a lockstep LDS search over the pivots, then a branchless
// search inside the bucket, SEARCH_ILP entries per lane at a time.  Returns
// the number flagged (plus 2^16 times the number among the tile's first 256
// entries); lb0 receives the lower bound in N(t) of the tile's first
// entry.  Matches are also counted in R.rc (reverse start hints stay unknown).
// The tile's entries are left in LDS (xs) as by dense_flags.
__device__ uint32_t search_flags(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Y, uint32_t ylo,
                                 uint32_t yhi, uint32_t np, uint32_t B, HubLds &L, uint32_t j0, uint32_t cnt,
                                 const RevSketch &R, uint32_t &lb0)
{
    const int l = lane_id();
    uint32_t c = 0, first = yhi;
#pragma unroll
    for (int h = 0; h < XPL; h += SEARCH_ILP) {
        uint32_t x[SEARCH_ILP], p[SEARCH_ILP];
#pragma unroll
        for (int k = 0; k < SEARCH_ILP; ++k) {
            const uint32_t i = (h + k) * WAVE + l;
            x[k] = i < cnt ? X[j0 + i] : 0xFFFFFFFFu;
            L.a.d.xs[i] = x[k];  // the tile, for the caller's answer
        }
        pivot_buckets(L, np, x, p);  // bucket index, np past the last
#pragma unroll
        for (int k = 0; k < SEARCH_ILP; ++k) {
            const uint64_t b0 = (uint64_t)ylo + (uint64_t)p[k] * B;
            p[k] = b0 < yhi ? (uint32_t)b0 : yhi;
        }
        // the lower bound lies in [p, p + len - 1]; probes past yhi read as +inf
        for (uint32_t len = B; len > 1; len -= len >> 1) {
            const uint32_t half = len >> 1;
#pragma unroll
            for (int k = 0; k < SEARCH_ILP; ++k) {
                const uint32_t q = p[k] + half - 1;
                const uint32_t v = q < yhi ? Y[q] : 0xFFFFFFFFu;
                p[k] += v < x[k] ? half : 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < SEARCH_ILP; ++k) {
            const uint32_t i = (h + k) * WAVE + l;
            const bool hit = i < cnt && p[k] < yhi && Y[p[k]] == x[k];
            L.a.d.flag[i] = hit ? 1 : 0;
            c += hit ? (h + k < 4 ? 0x10001u : 1u) : 0u;  // rows 0..3: the tile's first 256 entries
            if (R.rseg && hit) {
                const uint32_t q = p[k] / R.rseg;
                atomicAdd(&R.rc[q], 1u);
                if (p[k] - q * R.rseg < R.rseg / 2) atomicAdd(&R.r1[q], 1u);
            }
            if (h + k == 0) first = p[k];
        }
    }
    lb0 = lane_val(first, 0);
    wave_lds_sync();
    return wave_sum32(c);
}

// pi of entry j0+i of a tile (weights from W, or 1).
__device__ __forceinline__ uint64_t dense_pi(const uint16_t *__restrict__ W, const JobCtx &J, uint32_t pos_t,
                                             const HubLds &L, uint32_t j0, uint32_t i)
{
    const uint64_t w = W ? W[j0 + i] : 1u;
    const uint32_t m = (j0 + i == pos_t) ? J.A_ret : (L.a.d.flag[i] ? A_COM : J.A_out);
    return w * m;
}

__device__ uint64_t dense_chunk_sum(const uint16_t *__restrict__ W, const JobCtx &J, uint32_t pos_t,
                                    const HubLds &L, uint32_t j0, uint32_t cnt)
{
    const int l = lane_id();
    uint64_t s = 0;
#pragma unroll
    for (int e = 0; e < XPL; ++e) {
        const uint32_t i = e * WAVE + l;
        if (i < cnt) s += dense_pi(W, J, pos_t, L, j0, i);
    }
    return wave_sum(s);
}

// The weights of lane l's run of a tile, N(v)[j0 + XPL*l, +XPL) (0 past cnt),
// loaded before the tile's flags are formed so that their reads overlap the
// merge's instead of following it.
__device__ __forceinline__ void tile_run_weights(const uint16_t *__restrict__ W, uint32_t j0, uint32_t cnt,
                                                 uint32_t (&w)[XPL])
{
    const uint32_t i0 = (uint32_t)lane_id() * XPL;
#pragma unroll
    for (int e = 0; e < XPL; ++e) w[e] = W && i0 + e < cnt ? W[j0 + i0 + e] : (W ? 0u : 1u);
}

// First index of the tile whose running prefix (base + partial) exceeds r,
// or SENT (base then holds the prefix after the tile).  Lane l takes the run
// of entries [XPL*l, XPL*l + XPL): one 32-bit wave scan of the run sums (a
// tile sums to at most 512 * 65535 * 16 < 2^32) finds the lane whose run
// crosses r, and that lane walks its run.
__device__ uint32_t dense_chunk_locate(const uint32_t (&wrun)[XPL], const JobCtx &J, uint32_t pos_t,
                                       const HubLds &L, uint32_t j0, uint32_t cnt, uint64_t &base, uint64_t r)
{
    const int l = lane_id();
    const uint32_t i0 = (uint32_t)l * XPL;
    const uint64_t f8 = *(const uint64_t *)&L.a.d.flag[i0];
    uint32_t pi[XPL];
    uint32_t run = 0;
#pragma unroll
    for (int e = 0; e < XPL; ++e) {
        const uint32_t i = i0 + e;
        const uint32_t w = i < cnt ? wrun[e] : 0u;
        const uint32_t m = (j0 + i == pos_t) ? J.A_ret : (((f8 >> (8 * e)) & 0xFF) ? A_COM : J.A_out);
        pi[e] = w * m;
        run += pi[e];
    }
    const uint32_t inc = wave_incl_scan32(run);
    const uint64_t m = ballot(base + inc > r);
    if (m == 0) {
        base += lane_val(inc, WAVE - 1);
        return SENT;
    }
    const int f = first_lane(m);
    uint32_t j = SENT;
    if (l == f) {
        uint64_t acc = base + (inc - run);
#pragma unroll
        for (int e = 0; e < XPL; ++e) {
            acc += pi[e];
            if (j == SENT && acc > r) j = j0 + i0 + e;
        }
    }
    return lane_val(j, f);
}

// Sum of pi over N(v)[j0, j0+len) of an unweighted row with c members of N(t).
__device__ __forceinline__ uint64_t seg_pi(const JobCtx &J, uint32_t pos_t, uint32_t j0, uint32_t len, uint32_t c)
{
    uint64_t s = (uint64_t)J.A_out * len + (uint64_t)((int64_t)((int32_t)A_COM - (int32_t)J.A_out) * (int64_t)c);
    if (pos_t >= j0 && pos_t - j0 < len) s += (uint64_t)((int64_t)J.A_ret - (int64_t)J.A_out);
    return s;
}

// Sketch row of the move at v from t (t at index pos_t of N(v)), or null.
__device__ __forceinline__ uint16_t *sketch_row(const Exec &E, uint32_t v, uint32_t d, uint32_t pos_t)
{
    return E.g.memo + E.g.hbase[v] + pos_t * (uint64_t)memo_row_words(E.g.wt != nullptr, d);
}

// The same for the move at st.v, from the first sketch row loaded with v's
// record when there is one.
__device__ __forceinline__ uint16_t *sketch_row(const Exec &E, const WS &st, uint32_t pos_t)
{
    const uint64_t hb = st.hb != ~0ull ? st.hb : E.g.hbase[st.v];
    return E.g.memo + hb + pos_t * (uint64_t)memo_row_words(E.g.wt != nullptr, st.vd);
}

// Weight sums of a tile whose flags are in LDS: all entries, flagged entries,
// and both over the tile's first 256 entries (the runs of lanes 0..31).
struct TileW {
    uint32_t all, com, all1, com1;
};

__device__ __forceinline__ TileW tile_weights(const uint32_t (&wrun)[XPL], const HubLds &L, uint32_t cnt)
{
    const int l = lane_id();
    const uint32_t i0 = (uint32_t)l * XPL;
    const uint64_t f8 = *(const uint64_t *)&L.a.d.flag[i0];
    uint32_t a = 0, c = 0;
#pragma unroll
    for (int e = 0; e < XPL; ++e) {
        const uint32_t w = i0 + e < cnt ? wrun[e] : 0u;
        a += w;
        c += ((f8 >> (8 * e)) & 0xFF) ? w : 0u;
    }
    TileW t;
    t.all = wave_sum32(a);
    t.com = wave_sum32(c);
    t.all1 = wave_sum32(l < WAVE / 2 ? a : 0u);
    t.com1 = wave_sum32(l < WAVE / 2 ? c : 0u);
    return t;
}

// pi summed over entries of a weighted row whose weights sum to wall, of which
// members of N(t) sum to wcom, and t's own weight wt_t when t is among them
// (A_ret for t, A_com for members, A_out for the rest).
__device__ __forceinline__ uint64_t wseg_pi(const JobCtx &J, uint64_t wall, uint64_t wcom, uint64_t wt_t)
{
    return (uint64_t)J.A_out * (wall - wcom - wt_t) + (uint64_t)A_COM * wcom + (uint64_t)J.A_ret * wt_t;
}

// Reverse sketch to collect while merging a cold move at v (a hub) from t.
__device__ __forceinline__ uint16_t *rev_setup(const Exec &E, const WS &st, uint32_t *rc, uint32_t *rh, uint32_t *r1,
                                               RevSketch &R)
{
    R.rseg = 0;
    R.shift = hint_shift(st.vd);
    R.rc = rc;
    R.rh = rh;
    R.r1 = r1;
    // weighted rows need the weights of N(t), which a merge of N(v) does not read
    if (E.g.wt || st.td < E.g.memo_min || st.td > MEMO_MAX_DEG) return nullptr;
    const uint32_t tsub = (st.td + TX - 1) / TX;
    const uint32_t tG = (tsub + NSUPER - 1) / NSUPER;
    R.rseg = tG * TX;
    R.nsp = memo_segs(st.td);
    return sketch_row(E, st.t, st.td, st.jprev);
}

// Dense inverse CDF of a second-order move over all of N(v): per-segment sums
// (from the pair sketch when it is known, else by a merge-intersection pass
// that also fills the sketch and its reverse), then one segment is recomputed
// to find the entry whose prefix sum first exceeds r.
__device__ uint32_t hub_dense(const Exec &E, const JobCtx &J, const WS &st, HubLds &L, uint64_t R1, uint32_t &xj)
{
    const int l = lane_id();
    const uint32_t *__restrict__ X = E.g.adj + st.vo;
    const uint32_t *__restrict__ Y = E.g.adj + st.to;
    const uint16_t *__restrict__ W = E.g.wt ? E.g.wt + st.vo : nullptr;
    const uint32_t dv = st.vd, td = st.td, pos_t = st.pos_t;
    const uint32_t nsub = (dv + TX - 1) / TX;
    const uint32_t G = (nsub + NSUPER - 1) / NSUPER;  // tiles per segment
    const uint32_t nsup = (nsub + G - 1) / G;
    const uint32_t seglen = G * TX;
    const uint32_t hs = hint_shift(td);
    uint16_t *row = nullptr;
    if (E.g.memo && pos_t != SENT && dv >= E.g.memo_min && dv <= MEMO_MAX_DEG) row = sketch_row(E, st, pos_t);
    // weighted rows: per-segment weight sums after the u16 words (members of
    // N(t) + 1, the same over the first half + 1, all entries, first half)
    const uint32_t nsp = memo_segs(dv);  // entries per array of the row
    uint32_t *row32 = row && W ? (uint32_t *)(row + 3 * nsp) : nullptr;
    const uint64_t wt_t = W && pos_t != SENT ? W[pos_t] : 0u;
    bool warm = false;
    // per segment (lane): count + 1; where its stream of N(t) may start (SENT:
    // unknown), and an index at or above that start; first-half count + 1 (0:
    // unknown); weighted: the segment's weight sums (all, members; first half)
    uint32_t known = 1, ystart = SENT, ycap = td, halfv = 0, segcnt = 0;
    uint32_t segw = 0, segcw = 0, segw1 = 0, segcw1 = 0;
    if (row) {
        if ((uint32_t)l < nsup) {
            known = row[l];
            halfv = row[2 * nsp + l];
            const uint32_t h = row[nsp + l];
            if (h) {
                ystart = (h - 1) << hs;
                const uint64_t up = (uint64_t)h << hs;
                ycap = up < td ? (uint32_t)up : td;
            }
            if (row32) {
                // a word is 0 until written, and every writer writes the same
                // value: a segment is known when all of its words are
                const uint32_t cw = row32[l], cw1 = row32[nsp + l];
                segw = row32[2 * nsp + l];
                segw1 = row32[3 * nsp + l];
                if (cw == 0 || segw == 0) known = 0;
                if (cw1 == 0 || segw1 == 0) halfv = 0;
                segcw = cw - 1;
                segcw1 = cw1 - 1;
            }
        }
        warm = ballot(known == 0) == 0;
    }
    uint64_t S;
    if (warm) {
        uint64_t pi = 0;
        if ((uint32_t)l < nsup) {
            const uint32_t a = l * seglen;
            const uint32_t len = dv - a < seglen ? dv - a : seglen;
            if (W) pi = wseg_pi(J, segw, segcw, pos_t >= a && pos_t - a < len ? wt_t : 0u);
            else pi = seg_pi(J, pos_t, a, len, known - 1);
            L.b.csum[l] = pi;
        }
        S = wave_sum(pi);
    } else {
        RevSketch R;
        uint16_t *rrow = nullptr;
        if (row) rrow = rev_setup(E, st, L.a.d.rc, L.a.d.rh, L.a.d.r1, R);
        else R.rseg = 0;
        if (R.rseg) {
            L.a.d.rc[l] = 0;
            L.a.d.rh[l] = 0;
            L.a.d.r1[l] = 0;
        }
        // N(t) much longer than N(v): search N(v)'s entries in it instead of
        // streaming it (reverse start hints then stay unknown)
        const bool srch = (uint64_t)td > (uint64_t)E.search_ratio * dv;
        const uint32_t B = srch ? load_pivots(Y, 0, td, L, NPIV) : 0;
        uint32_t ypos = !srch && td ? wave_lower_bound(Y, td, X[0]) : 0;
        uint32_t mine = 0;
        S = 0;
        for (uint32_t sp = 0; sp < nsup; ++sp) {
            uint64_t sum = 0;
            uint32_t csp = 0, c1 = 0;  // members in the segment and in its first half
            uint32_t sw = 0, scw = 0, sw1 = 0, scw1 = 0;  // weighted: the same as weight sums
            const uint32_t mid = sp * seglen + seglen / 2;
            if ((uint32_t)l == sp) ystart = ypos;
            const uint32_t sub_end = nsub < (sp + 1) * G ? nsub : (sp + 1) * G;
            for (uint32_t sub = sp * G; sub < sub_end; ++sub) {
                const uint32_t j0 = sub * TX;
                const uint32_t cnt = dv - j0 < (uint32_t)TX ? dv - j0 : (uint32_t)TX;
                uint32_t wrun[XPL];
                if (W) tile_run_weights(W, j0, cnt, wrun);
                uint32_t c;
                if (srch) {
                    uint32_t lb0;
                    c = search_flags(X, Y, 0, td, NPIV, B, L, j0, cnt, R, lb0);
                    if (sub == sp * G && (uint32_t)l == sp) ystart = lb0;
                } else {
                    c = dense_flags(X, Y, td, L, j0, cnt, ypos, R);
                }
                const uint32_t ct = c & 0xFFFFu;
                if (W) {
                    const TileW tw = tile_weights(wrun, L, cnt);
                    sum += wseg_pi(J, tw.all, tw.com, pos_t >= j0 && pos_t - j0 < cnt ? wt_t : 0u);
                    sw += tw.all;
                    scw += tw.com;
                    sw1 += j0 + cnt <= mid ? tw.all : (j0 < mid ? tw.all1 : 0u);
                    scw1 += j0 + cnt <= mid ? tw.com : (j0 < mid ? tw.com1 : 0u);
                } else {
                    sum += seg_pi(J, pos_t, j0, cnt, ct);
                }
                csp += ct;
                // the half boundary is a tile start or 256 entries into a tile
                c1 += j0 + cnt <= mid ? ct : (j0 < mid ? c >> 16 : 0u);
                wave_lds_sync();
            }
            if (l == 0) L.b.csum[sp] = sum;
            if ((uint32_t)l == sp) {
                mine = csp;
                segcnt = csp;
                halfv = c1 + 1;
                segw = sw;
                segcw = scw;
                segw1 = sw1;
                segcw1 = scw1;
            }
            S += sum;
        }
        if (row && (uint32_t)l < nsup) {
            __builtin_nontemporal_store((uint16_t)(mine + 1), row + l);
            __builtin_nontemporal_store((uint16_t)((ystart >> hs) + 1), row + nsp + l);
            __builtin_nontemporal_store((uint16_t)halfv, row + 2 * nsp + l);
            if (row32) {
                __builtin_nontemporal_store(segcw + 1, row32 + l);
                __builtin_nontemporal_store(segcw1 + 1, row32 + nsp + l);
                __builtin_nontemporal_store(segw, row32 + 2 * nsp + l);
                __builtin_nontemporal_store(segw1, row32 + 3 * nsp + l);
            }
        }
        ycap = ystart;
        const uint32_t rsup = R.rseg ? (td + R.rseg - 1) / R.rseg : 0;
        if (rrow && (uint32_t)l < rsup) {
            __builtin_nontemporal_store((uint16_t)(L.a.d.rc[l] + 1), rrow + l);
            __builtin_nontemporal_store((uint16_t)L.a.d.rh[l], rrow + R.nsp + l);
            __builtin_nontemporal_store((uint16_t)(L.a.d.r1[l] + 1), rrow + 2 * R.nsp + l);
        }
    }
    wave_lds_sync();
    const uint64_t r = hi64(R1, S);
    uint64_t base;
    uint32_t spx = nsup - 1;
    {
        const uint64_t c = (uint32_t)l < nsup ? L.b.csum[l] : 0;
        const uint64_t inc = wave_incl_scan(c);
        const uint64_t m = ballot((uint32_t)l < nsup && inc > r);
        if (m) {
            const int f = first_lane(m);
            spx = f;
            base = lane_val64(inc - c, f);
        } else {
            base = lane_val64(inc - c, (int)(nsup - 1));
        }
    }
    wave_lds_sync();
    // the matches of segment spx lie in N(t)[ypos, yend): from its start to
    // (at or above) the next segment's start
    const uint32_t x0 = spx * seglen;
    const uint32_t xe = dv - x0 < seglen ? dv : x0 + seglen;
    const uint32_t mid = xe - x0 < seglen / 2 ? xe : x0 + seglen / 2;
    uint32_t ypos = lane_val(ystart, (int)spx);
    if (ypos == SENT) ypos = td ? wave_lower_bound(Y, td, X[x0]) : 0;
    if (ypos > td) ypos = td;
    uint32_t yend = spx + 1 < nsup ? lane_val(ycap, (int)spx + 1) : td;
    if (yend < ypos) yend = ypos;
    // with the first half's count known, only the half holding r is recomputed
    uint32_t xa = x0, xb = xe;
    const uint32_t hk = lane_val(halfv, (int)spx);
    const uint32_t segc = warm ? lane_val(known, (int)spx) - 1 : lane_val(segcnt, (int)spx);
    uint32_t crange = W ? SENT : segc;  // members of N(t) in [xa, xb), when known
    if (hk != 0 && mid < xe) {
        const uint64_t p1 = W ? wseg_pi(J, lane_val(segw1, (int)spx), lane_val(segcw1, (int)spx),
                                        pos_t >= x0 && pos_t < mid ? wt_t : 0u)
                              : seg_pi(J, pos_t, x0, mid - x0, hk - 1);
        if (base + p1 > r) {
            xb = mid;
            crange = W ? SENT : hk - 1;
        } else {
            base += p1;
            xa = mid;
            crange = W ? SENT : segc - (hk - 1);
            if (crange != 0) ypos += wave_lower_bound(Y + ypos, yend - ypos, X[mid]);
        }
    }
    if (crange == 0) {
        // no member of N(t) in the range: every pi is A_out but t's own (A_ret),
        // so the first prefix above r has a closed form
        const uint64_t rr = r - base;
        const uint64_t Ao = J.A_out;
        if (pos_t >= xa && pos_t < xb) {
            const uint64_t before = Ao * (pos_t - xa);
            if (rr < before) return xa + (uint32_t)(rr / Ao);
            if (rr < before + J.A_ret) return pos_t;
            return pos_t + 1 + (uint32_t)((rr - before - J.A_ret) / Ao);
        }
        return xa + (uint32_t)(rr / Ao);
    }
    const bool srch = (uint64_t)(yend - ypos) > (uint64_t)E.search_ratio * (xb - xa);
    const uint32_t np = pivots_for(xb - xa);
    const uint32_t B = srch ? load_pivots(Y, ypos, yend, L, np) : 0;
    const RevSketch none = {};
    for (uint32_t j0 = xa; j0 < xb; j0 += TX) {
        const uint32_t cnt = xb - j0 < (uint32_t)TX ? xb - j0 : (uint32_t)TX;
        uint32_t wrun[XPL];
        tile_run_weights(W, j0, cnt, wrun);
        if (srch) {
            uint32_t lb0;
            search_flags(X, Y, ypos, yend, np, B, L, j0, cnt, none, lb0);
        } else {
            dense_flags(X, Y, td, L, j0, cnt, ypos, none);
        }
        const uint32_t j = dense_chunk_locate(wrun, J, pos_t, L, j0, cnt, base, r);
        if (j != SENT) xj = L.a.d.xs[j - j0];  // the chosen neighbour, still in the tile
        wave_lds_sync();
        if (j != SENT) return j;
    }
    return dv - 1;  // not reached: the last prefix equals S > r
}

// Excess of special position q of N(v) over the out-multiplier:
// (A - A_out) * w_q with A = A_ret at t's position, else A_com.
__device__ __forceinline__ int32_t special_delta(const Exec &E, const JobCtx &J, const WS &st, uint32_t q)
{
    const int32_t w = E.g.wt ? (int32_t)E.g.wt[st.vo + q] : 1;
    const int32_t mult = q == st.pos_t ? (int32_t)J.A_ret : (int32_t)A_COM;
    return (mult - (int32_t)J.A_out) * w;
}

// Weighted scan with specials: pi_j = m0 * w_j + delta_j, the deltas of the
// c specials (sorted positions, in LDS) scattered chunk by chunk.
__device__ uint32_t weighted_scan_locate(const Exec &E, const JobCtx &J, const WS &st, HubLds &L, uint32_t m0,
                                         uint32_t c, uint64_t r)
{
    const int l = lane_id();
    const uint64_t dv = st.vd;
    uint64_t base = 0;
    uint32_t kp = 0;
    for (uint64_t j0 = 0; j0 < dv; j0 += HCH) {
        const uint32_t cnt = (uint32_t)std::min<uint64_t>(HCH, dv - j0);
#pragma unroll
        for (int e = 0; e < HEPL; ++e) L.c.dl[e * WAVE + l] = 0;
        wave_lds_sync();
        while (kp < c) {
            const uint32_t k = kp + l;
            const bool in = k < c && L.a.sp.pos[k] < j0 + cnt;
            if (in) L.c.dl[L.a.sp.pos[k] - j0] = special_delta(E, J, st, L.a.sp.pos[k]);
            const uint32_t n_in = __popcll(ballot(in));
            kp += n_in;
            if (n_in < WAVE) break;
        }
        wave_lds_sync();
#pragma unroll 1
        for (int e = 0; e < HEPL; ++e) {
            const uint32_t i = e * WAVE + l;
            uint64_t pi = 0;
            if (i < cnt) pi = (uint64_t)((int64_t)m0 * E.g.wt[st.vo + j0 + i] + L.c.dl[i]);
            const uint64_t inc = wave_incl_scan(pi);
            const uint64_t m = ballot(i < cnt && base + inc > r);
            if (m) {
                wave_lds_sync();
                return (uint32_t)(j0 + e * WAVE + first_lane(m));
            }
            base += lane_val64(inc, WAVE - 1);
        }
        wave_lds_sync();
    }
    return (uint32_t)(dv - 1);  // not reached
}

// Sparse inverse CDF: the members of N(t) are searched in N(v); they and t
// are the only entries whose multiplier differs from A_out.  The search takes
// SEARCH_ILP members per lane in lockstep: pivots of N(v) in LDS (about one
// per member searched) give the bucket, a branchless search inside it the
// position.
__device__ uint32_t hub_sparse(const Exec &E, const JobCtx &J, const WS &st, HubLds &L, uint64_t R1)
{
    const int l = lane_id();
    const uint32_t *__restrict__ X = E.g.adj + st.vo;
    const uint32_t *__restrict__ Y = E.g.adj + st.to;
    const uint32_t dv = st.vd, td = st.td;
    const uint32_t np = pivots_for(td);
    const uint32_t B = load_pivots(X, 0, dv, L, np);
    uint32_t c = 0;  // members found so far, in order (N(t) sorted => positions sorted)
    for (uint32_t b0 = 0; b0 < td; b0 += SEARCH_ILP * WAVE) {
        uint32_t y[SEARCH_ILP], p[SEARCH_ILP];
#pragma unroll
        for (int k = 0; k < SEARCH_ILP; ++k) {
            const uint32_t idx = b0 + k * WAVE + l;
            y[k] = idx < td ? Y[idx] : 0xFFFFFFFFu;
        }
        pivot_buckets(L, np, y, p);
#pragma unroll
        for (int k = 0; k < SEARCH_ILP; ++k) {
            const uint64_t s0 = (uint64_t)p[k] * B;
            p[k] = s0 < dv ? (uint32_t)s0 : dv;
        }
        for (uint32_t len = B; len > 1; len -= len >> 1) {
            const uint32_t half = len >> 1;
#pragma unroll
            for (int k = 0; k < SEARCH_ILP; ++k) {
                const uint32_t q = p[k] + half - 1;
                const uint32_t v = q < dv ? X[q] : 0xFFFFFFFFu;
                p[k] += v < y[k] ? half : 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < SEARCH_ILP; ++k) {
            const bool found = b0 + k * WAVE + l < td && p[k] < dv && X[p[k]] == y[k];
            const uint64_t m = ballot(found);
            if (found) L.a.sp.pos[c + __popcll(m & lanemask_lt())] = p[k];
            c += __popcll(m);
        }
    }
    wave_lds_sync();
    // insert t's own position (t is never a member of N(t)): the positions
    // above it move up by one, block by block from the top
    if (st.pos_t != SENT) {
        uint32_t nless = 0;
        for (uint32_t k = l; k < c; k += WAVE) nless += L.a.sp.pos[k] < st.pos_t ? 1u : 0u;
        nless = wave_sum32(nless);
        for (int32_t b = (int32_t)((c + WAVE - 1) / WAVE) - 1; b >= 0; --b) {
            const uint32_t k = (uint32_t)b * WAVE + l;
            const uint32_t v = k < c ? L.a.sp.pos[k] : 0u;
            wave_lds_sync();
            if (k < c && k >= nless) L.a.sp.pos[k + 1] = v;
            wave_lds_sync();
        }
        if (l == 0) L.a.sp.pos[nless] = st.pos_t;
        c += 1;
        wave_lds_sync();
    }
    // the positions give the sketch's per-segment counts (start hints stay
    // unknown), so later moves along this pair take the dense path's one-segment
    // recompute instead of searching again
    if (E.g.memo && !E.g.wt && st.pos_t != SENT && dv >= E.g.memo_min && dv <= MEMO_MAX_DEG) {
        const uint32_t nsub = (dv + TX - 1) / TX;
        const uint32_t G = (nsub + NSUPER - 1) / NSUPER;
        const uint32_t nsup = (nsub + G - 1) / G;
        const uint32_t seglen = G * TX;
        uint32_t *cnt = (uint32_t *)L.c.dl, *cnt1 = cnt + NSUPER;
        cnt[l] = 0;
        cnt1[l] = 0;
        wave_lds_sync();
        for (uint32_t k = l; k < c; k += WAVE) {
            const uint32_t q = L.a.sp.pos[k];
            if (q != st.pos_t) {
                const uint32_t sg = q / seglen;
                atomicAdd(&cnt[sg], 1u);
                if (q - sg * seglen < seglen / 2) atomicAdd(&cnt1[sg], 1u);
            }
        }
        wave_lds_sync();
        if ((uint32_t)l < nsup) {
            uint16_t *row = sketch_row(E, st, st.pos_t);
            __builtin_nontemporal_store((uint16_t)(cnt[l] + 1), row + l);
            __builtin_nontemporal_store((uint16_t)(cnt1[l] + 1), row + 2 * memo_segs(dv) + l);
        }
        wave_lds_sync();
    }
    int64_t dsum = 0;
    for (uint32_t k = l; k < c; k += WAVE) dsum += special_delta(E, J, st, L.a.sp.pos[k]);
    dsum = (int64_t)wave_sum((uint64_t)dsum);
    const uint64_t W = E.g.wt ? E.g.wsum[st.v] : dv;
    const uint64_t S = (uint64_t)((int64_t)(J.A_out * W) + dsum);
    const uint64_t r = hi64(R1, S);
    if (E.g.wt) return weighted_scan_locate(E, J, st, L, J.A_out, c, r);
    // unweighted: between specials the prefix grows by A_out per entry
    int64_t D = 0;       // deltas of the specials before this block
    int64_t qprev = -1;  // position of the special before this block
    for (uint32_t b = 0; b < c; b += WAVE) {
        const uint32_t k = b + l;
        const bool valid = k < c;
        const int64_t q = valid ? (int64_t)L.a.sp.pos[k] : 0;
        const int64_t dl = valid ? (int64_t)special_delta(E, J, st, (uint32_t)q) : 0;
        const int64_t inc = (int64_t)wave_incl_scan((uint64_t)dl);
        const int64_t Dincl = D + inc;
        const bool cross = valid && (int64_t)J.A_out * (q + 1) + Dincl > (int64_t)r;
        const uint64_t m = ballot(cross);
        if (m) {
            const int f = first_lane(m);
            const int64_t qf = (int64_t)lane_val64((uint64_t)q, f);
            const int64_t Dexcl = (int64_t)lane_val64((uint64_t)(Dincl - dl), f);
            const int64_t qp = f > 0 ? (int64_t)lane_val64((uint64_t)q, f - 1) : qprev;
            int64_t ig = ((int64_t)r - Dexcl) / (int64_t)J.A_out;
            if (ig < qp + 1) ig = qp + 1;
            return (uint32_t)(ig < qf ? ig : qf);
        }
        D += (int64_t)lane_val64((uint64_t)inc, WAVE - 1);
        const uint32_t last = c - 1 - b < (uint32_t)(WAVE - 1) ? c - 1 - b : (uint32_t)(WAVE - 1);
        qprev = (int64_t)lane_val64((uint64_t)q, (int)last);
    }
    int64_t ig = ((int64_t)r - D) / (int64_t)J.A_out;
    if (ig < qprev + 1) ig = qprev + 1;
    return (uint32_t)ig;
}

__device__ __forceinline__ bool use_sparse(const Exec &E, const WS &st)
{
    if (st.td + 1 > (uint32_t)SPCAP || st.td > E.t_sparse) return false;
    // on a weighted graph the sparse path locates the entry by scanning N(v)'s
    // weights; a move that keeps a pair sketch takes the dense path instead,
    // which fills the sketch, so that later visits recompute half a segment
    if (E.g.wt && E.g.memo && st.pos_t != SENT && st.vd >= E.g.memo_min && st.vd <= MEMO_MAX_DEG) return false;
    const uint32_t lg = 32 - __clz(st.vd);
    return (uint64_t)st.td * E.sparse_ratio * lg < (uint64_t)st.vd + st.td;
}

// ------------------------------------------------ workgroup per hub move
constexpr int HBLOCK = 256;  // plain hub kernel workgroup
constexpr int HUB_CLAIM = 8; // plain hub moves a wavefront claims per atomic
constexpr int HWAVES = HBLOCK / WAVE;

// LDS a workgroup shares while it evaluates one move together.
struct BlkLds {
    uint64_t csum[NSUPER];   // per-segment sums of pi
    uint32_t ystart[NSUPER]; // per-segment start in N(t) (SENT: search)
    uint32_t ycap[NSUPER];   // an index at or above each segment's start
    uint32_t rc[NSUPER];     // reverse sketch counts
    uint32_t rh[NSUPER];     // reverse sketch hints
    uint32_t r1[NSUPER];     // reverse sketch first-half counts
    uint64_t part[HWAVES];   // tile sums of one locate round
    uint32_t q;              // dequeued item
    uint32_t warm;
    uint32_t ans;
};

// Dense inverse CDF of one move by a whole workgroup (state uniform across
// the group): the same arithmetic as hub_dense, with the segments of N(v)
// split among the wavefronts (each merging its share against N(t) from its
// own lower bound) and the tiles of the located segment taken HWAVES at a
// time.  Every wavefront of the group must call it; it synchronises the group.
__device__ __forceinline__ uint32_t block_dense(const Exec &E, const JobCtx &J, const WS &st, HubLds &L, BlkLds &B, uint64_t R1)
{
    const int l = lane_id();
    const uint32_t wv = threadIdx.x / WAVE;
    const uint32_t *__restrict__ X = E.g.adj + st.vo;
    const uint32_t *__restrict__ Y = E.g.adj + st.to;
    const uint16_t *__restrict__ W = E.g.wt ? E.g.wt + st.vo : nullptr;
    const uint32_t dv = st.vd, td = st.td, pos_t = st.pos_t;
    const uint32_t nsub = (dv + TX - 1) / TX;
    const uint32_t G = (nsub + NSUPER - 1) / NSUPER;
    const uint32_t nsup = (nsub + G - 1) / G;
    const uint32_t seglen = G * TX;
    const uint32_t hs = hint_shift(td);
    uint16_t *row = nullptr;
    if (E.g.memo && !W && pos_t != SENT && dv >= E.g.memo_min && dv <= MEMO_MAX_DEG) row = sketch_row(E, st, pos_t);
    // one wavefront reads the sketch, so that the whole group takes one branch
    // even while another group is filling the same row
    if (wv == 0) {
        bool warm = false;
        uint32_t known = 1, ys = SENT, yc = td;
        if (row) {
            if ((uint32_t)l < nsup) {
                known = row[l];
                const uint32_t h = row[memo_segs(dv) + l];
                if (h) {
                    ys = (h - 1) << hs;
                    const uint64_t up = (uint64_t)h << hs;
                    yc = up < td ? (uint32_t)up : td;
                }
            }
            warm = ballot(known == 0) == 0;
        }
        if (warm && (uint32_t)l < nsup) {
            const uint32_t a = l * seglen;
            B.csum[l] = seg_pi(J, pos_t, a, dv - a < seglen ? dv - a : seglen, known - 1);
        }
        B.ystart[l] = ys;
        B.ycap[l] = yc;
        B.rc[l] = 0;
        B.rh[l] = 0;
        B.r1[l] = 0;
        if (l == 0) B.warm = warm;
    }
    __syncthreads();
    if (!B.warm) {
        RevSketch R;
        uint16_t *rrow = nullptr;
        if (row) rrow = rev_setup(E, st, B.rc, B.rh, B.r1, R);
        else R.rseg = 0;
        const uint32_t sp0 = wv * nsup / HWAVES, sp1 = (wv + 1) * nsup / HWAVES;
        const bool srch = (uint64_t)td > (uint64_t)E.search_ratio * dv;
        if (sp0 < sp1) {
            const uint32_t Bp = srch ? load_pivots(Y, 0, td, L, NPIV) : 0;
            uint32_t ypos = !srch && td ? wave_lower_bound(Y, td, X[sp0 * seglen]) : 0;
            for (uint32_t sp = sp0; sp < sp1; ++sp) {
                uint64_t sum = 0;
                uint32_t csp = 0;
                uint32_t ys = ypos;
                const uint32_t sub_end = nsub < (sp + 1) * G ? nsub : (sp + 1) * G;
                for (uint32_t sub = sp * G; sub < sub_end; ++sub) {
                    const uint32_t j0 = sub * TX;
                    const uint32_t cnt = dv - j0 < (uint32_t)TX ? dv - j0 : (uint32_t)TX;
                    uint32_t c;
                    if (srch) {
                        uint32_t lb0;
                        c = search_flags(X, Y, 0, td, NPIV, Bp, L, j0, cnt, R, lb0) & 0xFFFFu;
                        if (sub == sp * G) ys = lb0;
                    } else {
                        c = dense_flags(X, Y, td, L, j0, cnt, ypos, R) & 0xFFFFu;
                    }
                    sum += W ? dense_chunk_sum(W, J, pos_t, L, j0, cnt) : seg_pi(J, pos_t, j0, cnt, c);
                    csp += c;
                    wave_lds_sync();
                }
                if (l == 0) {
                    B.csum[sp] = sum;
                    B.ystart[sp] = ys;
                    B.ycap[sp] = ys;
                    if (row) {
                        __builtin_nontemporal_store((uint16_t)(csp + 1), row + sp);
                        __builtin_nontemporal_store((uint16_t)((ys >> hs) + 1), row + memo_segs(dv) + sp);
                    }
                }
            }
        }
        __syncthreads();
        const uint32_t rsup = R.rseg ? (td + R.rseg - 1) / R.rseg : 0;
        if (wv == 0 && rrow && (uint32_t)l < rsup) {
            __builtin_nontemporal_store((uint16_t)(B.rc[l] + 1), rrow + l);
            __builtin_nontemporal_store((uint16_t)B.rh[l], rrow + R.nsp + l);
            __builtin_nontemporal_store((uint16_t)(B.r1[l] + 1), rrow + 2 * R.nsp + l);
        }
    }
    // every wavefront finds the same segment from the shared sums
    const uint64_t c = (uint32_t)l < nsup ? B.csum[l] : 0;
    const uint64_t inc = wave_incl_scan(c);
    const uint64_t S = lane_val64(inc, WAVE - 1);
    const uint64_t r = hi64(R1, S);
    const uint64_t m = ballot((uint32_t)l < nsup && inc > r);
    const uint32_t spx = m ? (uint32_t)first_lane(m) : nsup - 1;
    uint64_t base = lane_val64(inc - c, (int)spx);
    // the matches of segment spx lie in N(t)[ylo, yhi)
    uint32_t ylo = B.ystart[spx];
    if (ylo == SENT) ylo = td ? wave_lower_bound(Y, td, X[spx * seglen]) : 0;
    if (ylo > td) ylo = td;
    uint32_t yhi = spx + 1 < nsup ? B.ycap[spx + 1] : td;
    if (yhi < ylo) yhi = ylo;
    const uint32_t xlen = dv - spx * seglen < seglen ? dv - spx * seglen : seglen;
    const bool lsrch = (uint64_t)(yhi - ylo) > (uint64_t)E.search_ratio * xlen;
    const RevSketch none = {};
    const uint32_t sub_end = nsub < (spx + 1) * G ? nsub : (spx + 1) * G;
    const uint32_t Bl = lsrch && spx * G + wv < sub_end ? load_pivots(Y, ylo, yhi, L, NPIV) : 0;
    for (uint32_t b = spx * G; b < sub_end; b += HWAVES) {
        const uint32_t sub = b + wv;
        const bool has = sub < sub_end;
        const uint32_t j0 = sub * TX;
        const uint32_t cnt = has ? (dv - j0 < (uint32_t)TX ? dv - j0 : (uint32_t)TX) : 0;
        uint64_t tsum = 0;
        if (has) {
            uint32_t cc;
            if (lsrch) {
                uint32_t lb0;
                cc = search_flags(X, Y, ylo, yhi, NPIV, Bl, L, j0, cnt, none, lb0) & 0xFFFFu;
            } else {
                uint32_t ypos = ylo;
                if (sub != spx * G) ypos = ylo + wave_lower_bound(Y + ylo, yhi - ylo, X[j0]);
                cc = dense_flags(X, Y, td, L, j0, cnt, ypos, none) & 0xFFFFu;
            }
            tsum = W ? dense_chunk_sum(W, J, pos_t, L, j0, cnt) : seg_pi(J, pos_t, j0, cnt, cc);
        }
        if (l == 0) B.part[wv] = tsum;
        __syncthreads();
        uint64_t before = base, after = base;
        for (int k = 0; k < HWAVES; ++k) {
            if ((uint32_t)k < wv) before += B.part[k];
            after += B.part[k];
        }
        if (has && before <= r && before + tsum > r) {
            uint32_t wrun[XPL];
            tile_run_weights(W, j0, cnt, wrun);
            const uint32_t j = dense_chunk_locate(wrun, J, pos_t, L, j0, cnt, before, r);
            if (l == 0) B.ans = j;
        }
        wave_lds_sync();
        __syncthreads();
        if (after > r) return B.ans;
        base = after;
    }
    return dv - 1;  // not reached: the last prefix equals S > r
}

// FN-Approx (Section 3.4, Eqs. 2 and 3).  At a vertex v of degree > d_rule
// reached from a vertex t of degree <= d_rule, every neighbour x != t of v has
// a probability between LB = wlo min(A_com, A_out) / (whi S_hi) and
// UB = whi max(A_com, A_out) / (wlo S_lo), where S_lo and S_hi bound the
// multiplier sum A_ret + c A_com + (d_v - 1 - c) A_out over c = 0 ..
// min(d_t, d_v) - 1 common neighbours and wlo, whi are the graph's smallest
// and largest weights.  When UB - LB < 1/approx_t the move is drawn as a first
// move (static weights, attempt 0, the move's own counter).  The comparison
// T (UB_n LB_d - LB_n UB_d) < UB_d LB_d is exact in 128 bits.
__device__ __forceinline__ bool approx_first_order(const Exec &E, const JobCtx &J, const WS &st)
{
    if (!J.approx_t || st.s == 0 || st.vd <= E.g.d_rule || st.td > E.g.d_rule || st.td == 0) return false;
    const uint64_t dv = st.vd, ac = 4, ao = J.A_out;
    const uint64_t c = (st.td < st.vd ? st.td : st.vd) - 1;
    const uint64_t none = J.A_ret + (dv - 1) * ao;
    const uint64_t all = J.A_ret + c * ac + (dv - 1 - c) * ao;
    const uint64_t lb_n = (uint64_t)E.g.wlo * (ac < ao ? ac : ao);
    const uint64_t lb_d = (uint64_t)E.g.whi * (none > all ? none : all);
    const uint64_t ub_n = (uint64_t)E.g.whi * (ac > ao ? ac : ao);
    const uint64_t ub_d = (uint64_t)E.g.wlo * (none < all ? none : all);
    const unsigned __int128 diff = (unsigned __int128)ub_n * lb_d - (unsigned __int128)lb_n * ub_d;
    return (unsigned __int128)J.approx_t * diff < (unsigned __int128)ub_d * lb_d;
}

// Inverse CDF of one move by a wavefront (state uniform across lanes).
// xj receives the chosen neighbour when the evaluation already holds it, else
// SENT.
__device__ __forceinline__ uint32_t wave_inverse_cdf(const Exec &E, const JobCtx &J, const WS &st_in, uint32_t kidx,
                                                     HubLds &L, uint32_t &xj)
{
    xj = SENT;
    const WS st = uniform_ws(st_in);
    const R4 rr = philox(J.k0, J.k1, J.wbase + st.i, st.s, kidx, 0u);
    const uint64_t R1 = join64(rr.x, rr.y);
    if (st.s == 0 || approx_first_order(E, J, st)) {
        if (!E.g.wt) return (uint32_t)hi64(R1, st.vd);
        return weighted_scan_locate(E, J, st, L, 1u, 0u, hi64(R1, E.g.wsum[st.v]));
    }
    bool sparse = use_sparse(E, st);
    if (sparse && E.g.memo && st.pos_t != SENT && st.vd >= E.g.memo_min && st.vd <= MEMO_MAX_DEG) {
        // a sketch that an earlier move filled makes the dense path cheaper
        const uint32_t nsub = (st.vd + TX - 1) / TX;
        const uint32_t G = (nsub + NSUPER - 1) / NSUPER;
        const uint32_t nsup = (nsub + G - 1) / G;
        const uint16_t *row = sketch_row(E, st, st.pos_t);
        const uint32_t known = (uint32_t)lane_id() < nsup ? row[lane_id()] : 1u;
        if (ballot(known == 0) == 0) sparse = false;
    }
    uint32_t j = sparse ? hub_sparse(E, J, st, L, R1) : hub_dense(E, J, st, L, R1, xj);
    if (j >= st.vd) {  // cannot happen for a correct rule; keeps every read inside the row
        if (lane_id() == 0) atomicOr(E.g.status, 2u);
        j = st.vd - 1;
        xj = SENT;
    }
    return j;
}

template <bool WALKS>
__device__ __forceinline__ void fill_tail_lane(const JobCtx &J, uint32_t i, uint32_t s)
{
    if (WALKS)
        for (uint32_t c = s + 1; c <= J.L; ++c) J.out[(uint64_t)i * (J.L + 1) + c] = SENT;
}

template <bool WALKS>
__device__ __forceinline__ void fill_tail_wave(const JobCtx &J, uint32_t i, uint32_t s)
{
    if (WALKS)
        for (uint32_t c = s + 1 + lane_id(); c <= J.L; c += WAVE) J.out[(uint64_t)i * (J.L + 1) + c] = SENT;
}

// Starts walk i of a job in lane state st; returns whether it has a move to make.
template <bool WALKS, bool COUNTS>
__device__ bool start_walk(const Exec &E, const JobCtx &J, uint32_t job, uint32_t i, uint32_t x, WS &st,
                           uint64_t &csum)
{
    st.job = job;
    st.i = i;
    st.s = 0;
    st.t = SENT;
    st.to = 0;
    st.td = 0;
    st.pos_t = SENT;
    st.jprev = SENT;
    if (x >= E.g.n) {
        atomicOr(E.g.status, 1u);
        if (WALKS) J.out[(uint64_t)i * (J.L + 1)] = x;
        fill_tail_lane<WALKS>(J, i, 0);
        return false;
    }
    emit<WALKS, COUNTS>(J, i, 0, x, csum);
    load_v(E, st, x);
    if (st.vd == 0) {
        fill_tail_lane<WALKS>(J, i, 0);
        return false;
    }
    return true;
}

// ---------------------------------------------------------- job sources
// One job for the whole launch (kernel arguments, uniform).
struct OneJob {
    JobCtx c;
    const uint32_t *starts;
    uint32_t n;
    uint32_t *cur;
    __device__ uint32_t total() const { return n; }
    __device__ uint32_t *cursor() const { return cur; }
    __device__ void locate(uint32_t g, uint32_t &job, uint32_t &i) const
    {
        job = 0;
        i = g;
    }
    __device__ JobCtx ctx(uint32_t) const { return c; }
    __device__ uint32_t start(uint32_t, uint32_t i) const { return starts[i]; }
};

// A table of jobs (serving): walk g belongs to the job whose prefix range
// holds it.  The header (job count, walk count) lives in device memory so that
// one captured launch can be replayed over tables of any content.
struct JobTable {
    const TableHdr *hdr;
    __device__ uint32_t total() const { return hdr->total; }
    __device__ uint32_t *cursor() const { return const_cast<uint32_t *>(&hdr->cursor); }
    __device__ void locate(uint32_t g, uint32_t &job, uint32_t &i) const
    {
        uint32_t lo = 0, hi = hdr->njobs;  // last job with jstart <= g
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (hdr->jstart[mid] <= g) lo = mid;
            else hi = mid;
        }
        job = lo;
        i = g - hdr->jstart[lo];
    }
    __device__ JobCtx ctx(uint32_t job) const { return hdr->jobs[job].c; }
    __device__ uint32_t start(uint32_t job, uint32_t i) const { return hdr->jobs[job].starts[i]; }
};

// ---------------------------------------------------------- persistent
constexpr int PBLOCK = 256;
constexpr int POOL = 256;  // most walks a wavefront claims per atomic

// Walk slot of one lane, kept in LDS between the thread and wave phases so
// that neither phase holds the other's registers.
struct Slot {
    uint32_t job, i, s, v, t, pos_t, jprev;
    uint32_t flags;  // bit 0: live, bit 1: pending wave/hub move, bit 2: after a_cap rejections
};
enum : uint32_t { SL_LIVE = 1, SL_PEND = 2, SL_CAP = 4 };

template <bool HUB = false>
__device__ __forceinline__ void slot_to_ws(const Exec &E, const Slot &q, WS &st)
{
    st.job = q.job;
    st.i = q.i;
    st.s = q.s;
    st.t = q.t;
    st.pos_t = q.pos_t;
    st.jprev = q.jprev;
    load_v<HUB>(E, st, q.v);
    if (q.s > 0) {
        const VRec r = E.g.vrec[q.t];
        st.to = r.off;
        st.td = r.deg;
    } else {
        st.to = 0;
        st.td = 0;
    }
}

__device__ __forceinline__ void ws_to_slot(const WS &st, uint32_t flags, Slot &q)
{
    q.job = st.job;
    q.i = st.i;
    q.s = st.s;
    q.v = st.v;
    q.t = st.t;
    q.pos_t = st.pos_t;
    q.jprev = st.jprev;
    q.flags = flags;
}

// The graph view a kernel instantiated for unweighted graphs (WT false)
// works with: a null weight array the compiler can see, so the weighted
// branches of every move drop out of its code (and its registers).
template <bool WT>
__device__ __forceinline__ Exec exec_for(const Exec &E)
{
    Exec e = E;
    if (!WT) {
        e.g.wt = nullptr;
        e.g.wsum = nullptr;
    }
    return e;
}

template <class Src, bool WALKS, bool COUNTS, bool WT>
__global__ __launch_bounds__(PBLOCK, 5) void k_persistent(Exec E_arg, Src S)
{
    const Exec E = exec_for<WT>(E_arg);
    __shared__ HubLds lds[PBLOCK / WAVE];
    __shared__ Slot slots[PBLOCK / WAVE][WAVE];
    HubLds &L = lds[threadIdx.x / WAVE];
    Slot *sl = slots[threadIdx.x / WAVE];
    const int l = lane_id();
    const uint32_t total = S.total();
    const uint32_t tw = E.t_wave < E.g.d_rule ? E.t_wave : E.g.d_rule;
    uint32_t pool_next = 0, pool_end = 0;  // walks this wavefront has claimed but not started
    // claims of up to POOL walks, but small enough that every wavefront of the
    // grid gets some (wave-class moves of a wavefront's walks run one by one);
    // later claims shrink with what is left (guided self-scheduling, down to
    // one walk), so that no wavefront holds unstarted walks while others have
    // run dry
    const uint32_t nwaves = gridDim.x * (PBLOCK / WAVE);
    uint32_t pool = total / nwaves < 1u ? 1u : (total / nwaves < (uint32_t)POOL ? total / nwaves : (uint32_t)POOL);
    bool exhausted = false;
    uint64_t csum = 0;
    sl[l].flags = 0;
    for (;;) {
        // refill and thread class: the lane's own walk
        {
            Slot q = sl[l];
            WS st;
            bool live = q.flags & SL_LIVE;
            bool pend = q.flags & SL_PEND;
            uint32_t cap = q.flags & SL_CAP;
            if (live) slot_to_ws(E, q, st);
            // idle lanes start walks claimed from the global counter, pool at a time
            for (;;) {
                const uint64_t m = ballot(!live);
                if (m == 0) break;
                if (pool_next >= pool_end) {
                    if (exhausted) break;
                    const uint32_t claim = pool;
                    uint32_t b = 0;
                    if (l == 0) b = atomicAdd(S.cursor(), claim);
                    b = uni(b);
                    if (b >= total) {
                        exhausted = true;
                        break;
                    }
                    pool_next = b;
                    pool_end = total - b < claim ? total : b + claim;
                    const uint32_t share = (total - pool_end) / (2 * nwaves);
                    pool = share < pool ? (share > 0 ? share : 1u) : pool;
                }
                const uint32_t avail = pool_end - pool_next;
                const uint32_t r = __popcll(m & lanemask_lt());
                if (!live && r < avail) {
                    uint32_t job, i;
                    S.locate(pool_next + r, job, i);
                    const JobCtx J = S.ctx(job);
                    live = start_walk<WALKS, COUNTS>(E, J, job, i, S.start(job, i), st, csum);
                    pend = false;
                    cap = 0;
                }
                const uint32_t took = __popcll(m);
                pool_next += took < avail ? took : avail;
            }
            if (ballot(live) == 0) break;
            for (uint32_t it = 0; it < E.thread_iters; ++it) {
                if (live && !pend && st.vd > tw) pend = true;
                const bool can = live && !pend;
                if (ballot(can) == 0) break;
                if (can) {
                    const JobCtx J = S.ctx(st.job);
                    uint32_t j;
                    if (thread_reject(E, J, st, j)) {
                        uint32_t x, rev;
                        resolve(E, st, j, x, rev);
                        emit<WALKS, COUNTS>(J, st.i, st.s + 1, x, csum);
                        advance(E, st, j, x, rev);
                        if (st.s == J.L || st.vd == 0) {
                            fill_tail_lane<WALKS>(J, st.i, st.s);
                            live = false;
                        }
                    } else {
                        pend = true;
                        cap = SL_CAP;
                    }
                }
            }
            if (live && !pend) pend = st.vd > tw;
            if (live) ws_to_slot(st, SL_LIVE | (pend ? SL_PEND : 0) | cap, q);
            else q.flags = 0;
            sl[l] = q;
        }
        wave_lds_sync();
        // wave and hub classes, one pending walk at a time, state in scalars
        uint64_t pm = ballot((sl[l].flags & (SL_LIVE | SL_PEND)) == (SL_LIVE | SL_PEND));
        while (pm) {
            const int o = first_lane(pm);
            pm &= pm - 1;
            Slot q;
            q.job = uni(sl[o].job);
            q.i = uni(sl[o].i);
            q.s = uni(sl[o].s);
            q.v = uni(sl[o].v);
            q.t = uni(sl[o].t);
            q.pos_t = uni(sl[o].pos_t);
            q.jprev = uni(sl[o].jprev);
            q.flags = uni(sl[o].flags);
            WS w;
            slot_to_ws<true>(E, q, w);
            w = uniform_ws(w);
            const JobCtx J = S.ctx(w.job);
            bool capped = q.flags & SL_CAP;
            bool alive = true;
            for (;;) {
                uint32_t j = 0, kidx = capped ? E.g.a_cap : 0u;
                bool icdf = capped || w.vd > E.g.d_rule;
                if (!icdf && !wave_reject(E, J, w, L, j)) {
                    icdf = true;
                    kidx = E.g.a_cap;
                }
                uint32_t xj = SENT;
                if (icdf) j = wave_inverse_cdf(E, J, w, kidx, L, xj);
                uint32_t x, rev;
                if (xj != SENT && !(w.s > 0 && j == w.pos_t)) {
                    // the neighbour is known: its record and the reverse
                    // position load together
                    x = xj;
                    rev = E.g.erec[w.vo + j].y;
                } else {
                    resolve(E, w, j, x, rev);
                }
                x = uni(x);
                rev = uni(rev);
                if (l == 0) emit<WALKS, COUNTS>(J, w.i, w.s + 1, x, csum);
                advance<true>(E, w, j, x, rev);
                w = uniform_ws(w);
                capped = false;
                if (w.s == J.L || w.vd == 0) {
                    fill_tail_wave<WALKS>(J, w.i, w.s);
                    alive = false;
                    break;
                }
                if (w.vd <= tw) break;
            }
            wave_lds_sync();
            if (l == o) {
                Slot r;
                if (alive) ws_to_slot(w, SL_LIVE, r);
                else r.flags = 0;
                sl[o] = r;
            }
            wave_lds_sync();
        }
    }
    if (COUNTS) {
        csum = wave_sum(csum);
        if (l == 0 && csum) atomicAdd(S.ctx(0).checksum, (unsigned long long)csum);
    }
}

// --------------------------------------------------------------- plain
// Per-walk state between supersteps: (v, t, pos_t, jprev); v = SENT once done.
template <bool WALKS, bool COUNTS>
__global__ __launch_bounds__(256) void k_plain_init(Exec E, OneJob S, uint4 *__restrict__ state)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t csum = 0;
    if (i < S.n) {
        WS st;
        const bool live = start_walk<WALKS, COUNTS>(E, S.c, 0, i, S.starts[i], st, csum);
        state[i] = make_uint4(live ? st.v : SENT, SENT, SENT, SENT);
    }
    if (COUNTS) {
        csum = wave_sum(csum);
        if (lane_id() == 0 && csum) atomicAdd(S.c.checksum, (unsigned long long)csum);
    }
}

template <bool HUB = false>
__device__ __forceinline__ bool plain_load(const Exec &E, const uint4 &q, uint32_t i, uint32_t s, WS &st)
{
    if (q.x == SENT) return false;
    st.job = 0;
    st.i = i;
    st.s = s;
    load_v<HUB>(E, st, q.x);
    st.t = q.y;
    st.pos_t = q.z;
    st.jprev = q.w;
    if (s > 0) {
        const VRec r = E.g.vrec[q.y];
        st.to = r.off;
        st.td = r.deg;
    } else {
        st.to = 0;
        st.td = 0;
    }
    return true;
}

template <bool WALKS, bool COUNTS>
__device__ __forceinline__ void plain_finish(const Exec &E, const JobCtx &J, WS &st, uint32_t j, uint4 *state,
                                             uint64_t &csum, bool wave)
{
    uint32_t x, rev;
    resolve(E, st, j, x, rev);
    if (!wave || lane_id() == 0) emit<WALKS, COUNTS>(J, st.i, st.s + 1, x, csum);
    // a dead end at x is found by the next superstep, which loads x's record
    // anyway
    const bool end = st.s + 1 == J.L;
    if (!wave || lane_id() == 0) state[st.i] = make_uint4(end ? SENT : x, st.v, rev, j);
}

// Rejection attempts a lane of the plain thread kernel makes alone when a
// superstep is small; its wavefront then takes the attempts that follow, 64
// at a time, so that the superstep does not wait for one lane's long chain.
// (A large superstep hides such chains behind other wavefronts.)
constexpr uint32_t PLAIN_LANE_ATTEMPTS = 16;

// Hub moves are queued for k_plain_hub: dense moves at degree > t_wg at the
// top of hubq (growing down, one workgroup each), all others at the bottom.
template <bool WALKS, bool COUNTS, bool COOP>
__global__ __launch_bounds__(256) void k_plain_step(Exec E, OneJob S, uint32_t s, uint4 *__restrict__ state,
                                                    uint32_t *__restrict__ hubq, uint32_t *__restrict__ hubn,
                                                    uint32_t *__restrict__ bign)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t csum = 0;
    bool push = false, big = false, pend = false;
    uint32_t item = 0;
    WS st;
    if (i < S.n) {
        if (plain_load(E, state[i], i, s, st)) {
            if (st.vd == 0) {
                // the previous move reached a dead end: the rest of the row is N2V_SENT
                fill_tail_lane<WALKS>(S.c, i, s);
                state[i].x = SENT;
            } else if (st.vd > E.g.d_rule) {
                item = i;
                // workgroups pay off on full merges: with sketches, only moves
                // whose sketch looks unknown (first count still 0) go to them
                big = s > 0 && st.vd > E.t_wg && !use_sparse(E, st) && !approx_first_order(E, S.c, st) &&
                      !(E.g.memo && st.pos_t != SENT && st.vd >= E.g.memo_min &&
                        st.vd <= MEMO_MAX_DEG && sketch_row(E, st, st.pos_t)[0] != 0);
                push = !big;
            } else {
                uint32_t j;
                if (thread_reject(E, S.c, st, j, COOP ? PLAIN_LANE_ATTEMPTS : 0xFFFFFFFFu)) {
                    plain_finish<WALKS, COUNTS>(E, S.c, st, j, state, csum, false);
                } else if (COOP) {
                    pend = true;
                } else {
                    push = true;  // every attempt rejected: the inverse CDF of attempt a_cap
                    item = i | 0x80000000u;
                }
            }
        }
    }
    if constexpr (COOP) {
        __shared__ HubLds lds[256 / WAVE];
        HubLds &L = lds[threadIdx.x / WAVE];
        for (uint64_t pm = ballot(pend); pm; pm &= pm - 1) {
            const int o = first_lane(pm);
            WS w = bcast(st, o);
            uint32_t j;
            if (wave_reject(E, S.c, w, L, j, PLAIN_LANE_ATTEMPTS)) {
                plain_finish<WALKS, COUNTS>(E, S.c, w, j, state, csum, true);
            } else if (lane_id() == o) {
                push = true;
                item = i | 0x80000000u;
            }
        }
    }
    const uint64_t m = ballot(push);
    if (m) {
        uint32_t base = 0;
        const int lead = first_lane(m);
        if (lane_id() == lead) base = atomicAdd(hubn, (uint32_t)__popcll(m));
        base = shfl32(base, lead);
        if (push) hubq[base + __popcll(m & lanemask_lt())] = item;
    }
    const uint64_t mb = ballot(big);
    if (mb) {
        uint32_t base = 0;
        const int lead = first_lane(mb);
        if (lane_id() == lead) base = atomicAdd(bign, (uint32_t)__popcll(mb));
        base = shfl32(base, lead);
        if (big) hubq[S.n - 1 - (base + __popcll(mb & lanemask_lt()))] = item;
    }
    if (COUNTS) {
        csum = wave_sum(csum);
        if (lane_id() == 0 && csum) atomicAdd(S.c.checksum, (unsigned long long)csum);
    }
}

// The hub moves of this superstep: first the large dense ones, one workgroup
// each (largest work first shortens the superstep's tail), then the rest,
// one wavefront each.
template <bool WALKS, bool COUNTS, bool WT>
__global__ __launch_bounds__(HBLOCK, 5) void k_plain_hub(Exec E_arg, OneJob S, uint32_t s, uint4 *__restrict__ state,
                                                         const uint32_t *__restrict__ hubq,
                                                         const uint32_t *__restrict__ hubn, uint32_t *__restrict__ hubd,
                                                         const uint32_t *__restrict__ bign, uint32_t *__restrict__ bigd)
{
    const Exec E = exec_for<WT>(E_arg);
    __shared__ HubLds lds[HBLOCK / WAVE];
    __shared__ BlkLds blk;
    HubLds &L = lds[threadIdx.x / WAVE];
    const bool lead = threadIdx.x < WAVE;
    uint64_t csum = 0;
    // Each workgroup first takes the large move of its own index and each
    // wavefront the small move of its own index; only the moves past those
    // are claimed from the superstep's counters.  A short queue (the common
    // case) then costs no atomics: thousands of claims on one counter would
    // serialise in L2 and outlast the moves themselves.
    const uint32_t nb = *bign;
    for (uint32_t q = blockIdx.x; q < nb;) {
        const uint32_t i = uni(hubq[S.n - 1 - q]);
        WS st;
        plain_load<true>(E, state[i], i, s, st);
        st = uniform_ws(st);
        const R4 rr = philox(S.c.k0, S.c.k1, S.c.wbase + st.i, st.s, 0u, 0u);
        uint32_t j = block_dense(E, S.c, st, L, blk, join64(rr.x, rr.y));
        if (lead) {
            if (j >= st.vd) {
                if (lane_id() == 0) atomicOr(E.g.status, 2u);
                j = st.vd - 1;
            }
            plain_finish<WALKS, COUNTS>(E, S.c, st, j, state, csum, true);
        }
        if (nb <= gridDim.x) break;
        __syncthreads();
        if (threadIdx.x == 0) blk.q = gridDim.x + atomicAdd(bigd, 1u);
        __syncthreads();
        q = blk.q;
    }
    // wavefront moves past the first nwaves: up to HUB_CLAIM per atomic,
    // sized so that what is left spreads over the grid
    const uint32_t n = *hubn;
    const uint32_t nwaves = gridDim.x * (HBLOCK / WAVE);
    const uint32_t rest = n > nwaves ? n - nwaves : 0u;
    const uint32_t per = (rest + nwaves - 1) / nwaves;
    const uint32_t claim = per < 1u ? 1u : (per > (uint32_t)HUB_CLAIM ? (uint32_t)HUB_CLAIM : per);
    uint32_t q0 = blockIdx.x * (HBLOCK / WAVE) + threadIdx.x / WAVE, q1 = q0 + 1;
    while (q0 < n) {
        if (q1 > n) q1 = n;
        for (uint32_t q = q0; q < q1; ++q) {
            const uint32_t item = uni(hubq[q]);
            const uint32_t i = item & 0x7FFFFFFFu;
            const uint32_t kidx = (item & 0x80000000u) ? E.g.a_cap : 0u;
            WS st;
            plain_load<true>(E, state[i], i, s, st);
            uint32_t xj;
            const uint32_t j = wave_inverse_cdf(E, S.c, st, kidx, L, xj);
            plain_finish<WALKS, COUNTS>(E, S.c, st, j, state, csum, true);
        }
        if (rest == 0) break;
        uint32_t b = 0;
        if (lane_id() == 0) b = atomicAdd(hubd, claim);
        q0 = nwaves + uni(b);
        q1 = q0 + claim;
    }
    if (COUNTS) {
        csum = wave_sum(csum);
        if (lane_id() == 0 && csum) atomicAdd(S.c.checksum, (unsigned long long)csum);
    }
}

__global__ void k_zero64(uint32_t *p, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

__global__ void k_zero(uint32_t *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------- host
struct DevInfo {
    int cus = 0;
    int occ = 0;
};

DevInfo &dev_info(int dev)
{
    static DevInfo info[64];
    DevInfo &d = info[dev & 63];
    if (d.cus == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) d.cus = prop.multiProcessorCount;
        if (d.cus <= 0) d.cus = 256;
        int b = 0;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void *)k_persistent<OneJob, true, true, true>,
                                                           PBLOCK, 0);
        d.occ = b > 0 ? b : 2;
    }
    return d;
}

size_t plain_ws(uint32_t n_starts, uint32_t L)
{
    Carver c(nullptr, 0);
    c.take<uint4>(n_starts ? n_starts : 1);
    c.take<uint32_t>(n_starts ? n_starts : 1);
    c.take<uint32_t>(4 * ((uint64_t)L + 1));
    return c.total();
}

uint32_t persistent_blocks(const n2v_exec_opts &o, int dev, uint64_t walks)
{
    DevInfo &d = dev_info(dev);
    uint32_t per_cu = o.waves_per_cu ? (o.waves_per_cu + (PBLOCK / WAVE) - 1) / (PBLOCK / WAVE) : (uint32_t)d.occ;
    if (per_cu > (uint32_t)d.occ) per_cu = d.occ;
    if (per_cu < 1) per_cu = 1;
    uint64_t blocks = (uint64_t)d.cus * per_cu;
    const uint64_t need = (walks + WAVE - 1) / WAVE;  // small jobs: spread walks thin over more wavefronts
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    return (uint32_t)blocks;
}

template <bool W, bool C>
int launch_persistent(const Exec &E, const OneJob &S, const n2v_exec_opts &o, int dev, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, S.cur, 1u);
    if (E.g.wt)
        hipLaunchKernelGGL((k_persistent<OneJob, W, C, true>), dim3(persistent_blocks(o, dev, S.n)), dim3(PBLOCK), 0,
                           st, E, S);
    else
        hipLaunchKernelGGL((k_persistent<OneJob, W, C, false>), dim3(persistent_blocks(o, dev, S.n)), dim3(PBLOCK), 0,
                           st, E, S);
    N2V_HIP(hipGetLastError());
    return N2V_OK;
}

template <bool W, bool C>
int launch_plain(const Exec &E, const OneJob &S, void *ws, int dev, hipStream_t st)
{
    Carver c(ws, (size_t)-1);
    uint4 *state = c.take<uint4>(S.n ? S.n : 1);
    uint32_t *hubq = c.take<uint32_t>(S.n ? S.n : 1);
    // per superstep: enqueued and dequeued wavefront moves, then workgroup moves
    uint32_t *hubn = c.take<uint32_t>(4 * ((uint64_t)S.c.L + 1));
    uint32_t *hubd = hubn + S.c.L + 1;
    uint32_t *bign = hubd + S.c.L + 1;
    uint32_t *bigd = bign + S.c.L + 1;
    const uint32_t blocks = (S.n + 255) / 256;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, st, hubn, 4 * (S.c.L + 1));
    hipLaunchKernelGGL((k_plain_init<W, C>), dim3(blocks), dim3(256), 0, st, E, S, state);
    N2V_HIP(hipGetLastError());
    DevInfo &d = dev_info(dev);
    const uint32_t hub_blocks = (uint32_t)d.cus * 8;
    // the thread kernel lasts as long as its slowest lane's chain of dependent
    // reads: a small superstep is spread over every CU, one wavefront per
    // block, and its wavefronts finish their lanes' long rejection chains
    // together
    const uint32_t tpb = S.n < (uint32_t)d.cus * 1024u ? 64u : 256u;
    const uint32_t sblocks = (S.n + tpb - 1) / tpb;
    for (uint32_t s = 0; s < S.c.L; ++s) {
        if (tpb == 64)
            hipLaunchKernelGGL((k_plain_step<W, C, true>), dim3(sblocks), dim3(tpb), 0, st, E, S, s, state, hubq,
                               hubn + s, bign + s);
        else
            hipLaunchKernelGGL((k_plain_step<W, C, false>), dim3(sblocks), dim3(tpb), 0, st, E, S, s, state, hubq,
                               hubn + s, bign + s);
        if (E.g.wt)
            hipLaunchKernelGGL((k_plain_hub<W, C, true>), dim3(hub_blocks), dim3(HBLOCK), 0, st, E, S, s, state, hubq,
                               (const uint32_t *)(hubn + s), hubd + s, (const uint32_t *)(bign + s), bigd + s);
        else
            hipLaunchKernelGGL((k_plain_hub<W, C, false>), dim3(hub_blocks), dim3(HBLOCK), 0, st, E, S, s, state,
                               hubq, (const uint32_t *)(hubn + s), hubd + s, (const uint32_t *)(bign + s), bigd + s);
    }
    N2V_HIP(hipGetLastError());
    return N2V_OK;
}

}  // namespace

// ------------------------------------------------- shared with other files
int walk_multipliers(float p, float q, uint32_t *A_ret, uint32_t *A_out)
{
    static const float allowed[5] = {0.25f, 0.5f, 1.0f, 2.0f, 4.0f};
    static const uint32_t mult[5] = {16, 8, 4, 2, 1};
    int ip = -1, iq = -1;
    for (int i = 0; i < 5; ++i) {
        if (p == allowed[i]) ip = i;
        if (q == allowed[i]) iq = i;
    }
    if (ip < 0 || iq < 0) return -1;
    *A_ret = mult[ip];
    *A_out = mult[iq];
    return 0;
}

// Walk counters of a graph: a persistent launch takes a counter slot that no
// launch still in flight holds (an event recorded after each launch tells),
// so overlapping calls never share a counter.
//
// The same host record keeps the graph's captured plain-form launch
// sequences.  The plain form issues 2L+2 kernels per call.  A call whose
// every launch argument (graph view, options, job, starts, outputs,
// workspace, grid) equals that of one of the last PLAIN_GRAPHS distinct calls
// is recorded into a hipGraph on its second occurrence and replayed from then
// on: one graph launch instead of 2L+2 kernel launches.  A replay runs exactly
// the kernels, grids and arguments of the direct launches, so results are the
// same; the contents of the buffers may change between calls.
constexpr int PLAIN_GRAPHS = 8;
constexpr int PLAIN_KEY_WORDS = 32;

struct PlainKey {
    uint64_t w[PLAIN_KEY_WORDS] = {};
    int n = 0;
    void put(uint64_t x) { w[n++] = x; }
    void put(const void *p) { put((uint64_t)(uintptr_t)p); }
    void put2(uint32_t hi, uint32_t lo) { put(((uint64_t)hi << 32) | lo); }
    bool operator==(const PlainKey &o) const { return n == o.n && !memcmp(w, o.w, sizeof(uint64_t) * n); }
};

struct PlainGraph {
    PlainKey key;                   // n == 0: unused
    hipGraphExec_t exec = nullptr;  // null: seen once, not captured yet
    hipEvent_t done = nullptr;      // recorded after each replay
    uint64_t used = 0;              // last use (LRU)
};

struct CursorSlots {
    std::mutex mu;
    hipEvent_t ev[CURSOR_SLOTS] = {};
    int next = 0;
    PlainGraph plain[PLAIN_GRAPHS];
    uint64_t clock = 0;
    hipStream_t cap = nullptr;  // private stream the plain form is captured on
};

void plain_graph_drop(PlainGraph &e)
{
    if (e.done) {
        (void)hipEventSynchronize(e.done);
        (void)hipEventDestroy(e.done);
    }
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    e = PlainGraph();
}

void *cursor_slots_new() { return new (std::nothrow) CursorSlots(); }

void cursor_slots_free(void *p)
{
    CursorSlots *cs = (CursorSlots *)p;
    if (!cs) return;
    for (hipEvent_t &e : cs->ev)
        if (e) (void)hipEventDestroy(e);
    for (PlainGraph &e : cs->plain) plain_graph_drop(e);
    if (cs->cap) (void)hipStreamDestroy(cs->cap);
    delete cs;
}

template <class F>
int with_cursor(const n2v_graph *g, hipStream_t st, F launch)
{
    CursorSlots *cs = (CursorSlots *)g->slots;
    std::lock_guard<std::mutex> lk(cs->mu);
    int slot = -1;
    for (int k = 0; k < CURSOR_SLOTS && slot < 0; ++k) {
        const int i = (cs->next + k) % CURSOR_SLOTS;
        if (!cs->ev[i]) N2V_HIP(hipEventCreateWithFlags(&cs->ev[i], hipEventDisableTiming));
        const hipError_t q = hipEventQuery(cs->ev[i]);
        if (q == hipSuccess) slot = i;
        else if (q != hipErrorNotReady) return hip_fail(q, "hipEventQuery (walk counter)");
    }
    if (slot < 0)
        return set_error(N2V_EAGAIN, "n2v_walk: %d persistent walk calls on this graph are still in flight",
                         CURSOR_SLOTS);
    cs->next = (slot + 1) % CURSOR_SLOTS;
    const int rc = launch(g->dg.cursors + (uint64_t)slot * CURSOR_STRIDE);
    if (rc) return rc;
    N2V_HIP(hipEventRecord(cs->ev[slot], st));
    return N2V_OK;
}

void make_exec(const n2v_graph *g, const n2v_exec_opts &o, Exec *E)
{
    E->g = g->dg;
    E->cursor = nullptr;  // persistent launches take one per launch (with_cursor)
    if (!o.memo) E->g.memo = nullptr;
    E->t_wave = o.t_wave;
    E->t_sparse = o.t_sparse;
    E->t_wg = o.t_wg < g->dg.d_rule ? g->dg.d_rule : o.t_wg;
    E->search_ratio = o.search_ratio;
    E->sparse_ratio = o.sparse_ratio < 1 ? 1 : o.sparse_ratio;
    // Where hub rows hold a large share of the entries (so of the visits), a
    // lane's walk soon reaches one and waits while the other lanes go on: one
    // rejection move per lane before the wave serves its pending walks when
    // hub rows hold at least 35% of the entries, two from 2%.  Otherwise
    // eight, since each return to the wave phase reloads the lanes' vertex
    // records.
    const uint64_t he = g->hub_entries, m = g->dg.m;
    E->thread_iters = he && he * 20 >= m * 7 ? 1u : (he && he * 50 >= m ? 2u : 8u);
}

PlainKey plain_key(const Exec &E, const OneJob &S, const void *ws, uint32_t hub_blocks, bool W, bool C)
{
    // every field the launches read from the host: a new field of Exec,
    // DevGraph, JobCtx or OneJob must be added here
    static_assert(sizeof(DevGraph) == 112 && sizeof(Exec) == 144 && sizeof(JobCtx) == 56 && sizeof(OneJob) == 80,
                  "plain_key covers every launch argument");
    PlainKey k;
    const DevGraph &d = E.g;
    k.put(d.vrec);
    k.put(d.erec);
    k.put(d.adj);
    k.put(d.wt);
    k.put(d.wsum);
    k.put(d.hbase);
    k.put(d.memo);
    k.put(d.status);
    k.put(d.cursors);
    k.put2(d.n, d.d_rule);
    k.put(d.m);
    k.put2(d.memo_min, d.a_cap);
    k.put2(d.wlo, d.whi);
    k.put2(E.t_wave, E.t_sparse);
    k.put2(E.sparse_ratio, E.t_wg);
    k.put2(E.search_ratio, hub_blocks);
    k.put2(E.thread_iters, 0u);
    k.put(E.cursor);
    k.put(S.c.out);
    k.put(S.c.cnt);
    k.put(S.c.checksum);
    k.put2(S.c.wbase, S.c.L);
    k.put2(S.c.k0, S.c.k1);
    k.put2(S.c.A_ret, S.c.A_out);
    k.put2(S.c.approx_t, S.n);
    k.put(S.starts);
    k.put(S.cur);
    k.put(ws);
    k.put((W ? 1u : 0u) | (C ? 2u : 0u));
    return k;
}

template <bool W, bool C>
int capture_plain(CursorSlots *cs, const Exec &E, const OneJob &S, void *ws, int dev, hipGraphExec_t *out)
{
    if (!cs->cap) N2V_HIP(hipStreamCreateWithFlags(&cs->cap, hipStreamNonBlocking));
    N2V_HIP(hipStreamBeginCapture(cs->cap, hipStreamCaptureModeThreadLocal));
    const int rc = launch_plain<W, C>(E, S, ws, dev, cs->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs->cap, &graph);
    if (rc || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc ? rc : hip_fail(e, "hipStreamEndCapture (plain form)");
    }
    const hipError_t e2 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
        *out = nullptr;
        return hip_fail(e2, "hipGraphInstantiate (plain form)");
    }
    return N2V_OK;
}

// The plain form, direct or replayed from a captured graph (see PlainGraph).
// Calls enqueued on a stream that is itself being captured launch directly.
template <bool W, bool C>
int launch_plain_replayed(const n2v_graph *g, const Exec &E, const OneJob &S, void *ws, hipStream_t st)
{
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess) {
        (void)hipGetLastError();
        cap = hipStreamCaptureStatusActive;  // unknown: do not capture
    }
    if (cap != hipStreamCaptureStatusNone) return launch_plain<W, C>(E, S, ws, g->device, st);
    const PlainKey k = plain_key(E, S, ws, (uint32_t)dev_info(g->device).cus * 8, W, C);
    CursorSlots *cs = (CursorSlots *)g->slots;
    std::lock_guard<std::mutex> lk(cs->mu);
    const uint64_t now = ++cs->clock;
    PlainGraph *hit = nullptr;
    for (PlainGraph &e : cs->plain)
        if (e.key.n && e.key == k) hit = &e;
    if (!hit) {
        // first occurrence: remember it in the least recently used entry that
        // no replay in flight holds, and launch directly
        PlainGraph *victim = nullptr;
        for (PlainGraph &e : cs->plain) {
            if (e.done) {
                const hipError_t q = hipEventQuery(e.done);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess) return hip_fail(q, "hipEventQuery (plain form graph)");
            }
            if (!victim || e.used < victim->used) victim = &e;
        }
        if (victim) {
            plain_graph_drop(*victim);
            victim->key = k;
            victim->used = now;
        }
        return launch_plain<W, C>(E, S, ws, g->device, st);
    }
    hit->used = now;
    if (!hit->exec) {
        int rc = capture_plain<W, C>(cs, E, S, ws, g->device, &hit->exec);
        if (rc == N2V_OK && !hit->done) {
            const hipError_t e = hipEventCreateWithFlags(&hit->done, hipEventDisableTiming);
            if (e != hipSuccess) rc = hip_fail(e, "hipEventCreate (plain form graph)");
        }
        if (rc) {
            plain_graph_drop(*hit);
            return rc;
        }
    }
    N2V_HIP(hipGraphLaunch(hit->exec, st));
    N2V_HIP(hipEventRecord(hit->done, st));
    return N2V_OK;
}

uint32_t full_grid_blocks(int dev)
{
    DevInfo &d = dev_info(dev);
    return (uint32_t)d.cus * (uint32_t)d.occ;
}

int launch_job_table(const Exec &E, const TableHdr *hdr, uint32_t blocks, hipStream_t st)
{
    JobTable T;
    T.hdr = hdr;
    if (E.g.wt)
        hipLaunchKernelGGL((k_persistent<JobTable, true, false, true>), dim3(blocks), dim3(PBLOCK), 0, st, E, T);
    else
        hipLaunchKernelGGL((k_persistent<JobTable, true, false, false>), dim3(blocks), dim3(PBLOCK), 0, st, E, T);
    N2V_HIP(hipGetLastError());
    return N2V_OK;
}

int launch_one(const n2v_graph *g, const Exec &E, const JobCtx &c, const uint32_t *starts, uint32_t n,
               const n2v_exec_opts &o, hipStream_t st)
{
    OneJob S;
    S.c = c;
    S.starts = starts;
    S.n = n;
    return with_cursor(g, st, [&](uint32_t *cur) {
        S.cur = cur;
        return launch_persistent<true, false>(E, S, o, g->device, st);
    });
}

}  // namespace n2v

using namespace n2v;

extern "C" void n2v_exec_opts_default(const n2v_graph *g, n2v_exec_opts *o)
{
    if (!o) return;
    if (g && g->has_tuned) {
        *o = g->tuned;
        return;
    }
    o->mode = N2V_MODE_AUTO;
    o->t_wave = 1024;
    o->t_sparse = 1023;
    o->sparse_ratio = 2;
    o->waves_per_cu = 0;
    o->block = 256;
    o->memo = 1;
    o->t_wg = 65536;
    o->search_ratio = 24;
}

extern "C" int n2v_walk_workspace(const n2v_graph *g, uint32_t n_starts, uint32_t L, const n2v_exec_opts *opts,
                                  size_t *ws_bytes)
{
    if (!g || !ws_bytes) return set_error(N2V_EINVAL, "n2v_walk_workspace: null argument");
    n2v_exec_opts o;
    n2v_exec_opts_default(g, &o);
    if (opts) o = *opts;
    *ws_bytes = o.mode == N2V_MODE_PLAIN ? plain_ws(n_starts, L) : 0;
    return N2V_OK;
}

namespace n2v {
namespace {

// Every walk entry point: `replay` lets the plain form use captured graphs
// (instantiating one allocates, so the static entry point launches directly).
int walk_impl(const n2v_graph *g, const uint32_t *starts, uint32_t n_starts, uint64_t walk_base, uint32_t L,
              float p, float q, uint64_t seed, uint32_t approx_t, const n2v_exec_opts *opts, int outputs,
              uint32_t *out, uint32_t *cnt, uint64_t *checksum, void *ws, size_t ws_bytes, void *stream,
              bool replay)
{
    if (!g) return set_error(N2V_EINVAL, "n2v_walk: null graph");
    if (L < 1) return set_error(N2V_EINVAL, "n2v_walk: L must be >= 1");
    uint32_t A_ret, A_out;
    if (walk_multipliers(p, q, &A_ret, &A_out))
        return set_error(N2V_EINVAL, "n2v_walk: p and q must be in {0.25, 0.5, 1, 2, 4}");
    if (!(outputs & (N2V_OUT_WALKS | N2V_OUT_COUNTS)) || (outputs & ~(N2V_OUT_WALKS | N2V_OUT_COUNTS)))
        return set_error(N2V_EINVAL, "n2v_walk: outputs must be a nonempty mask of N2V_OUT_WALKS | N2V_OUT_COUNTS");
    const bool W = outputs & N2V_OUT_WALKS, C = outputs & N2V_OUT_COUNTS;
    if (walk_base + (uint64_t)n_starts > (1ull << 32)) return set_error(N2V_EINVAL, "n2v_walk: walk ids exceed 2^32");
    if (n_starts >= 0x80000000u) return set_error(N2V_EINVAL, "n2v_walk: at most 2^31-1 walks per call");
    if (n_starts == 0) return N2V_OK;
    if (W && !out) return set_error(N2V_EINVAL, "n2v_walk: null out");
    if (C && (!cnt || !checksum)) return set_error(N2V_EINVAL, "n2v_walk: null cnt or checksum");
    if (!starts) return set_error(N2V_EINVAL, "n2v_walk: null starts");
    n2v_exec_opts o;
    n2v_exec_opts_default(g, &o);
    if (opts) o = *opts;

    Exec E;
    make_exec(g, o, &E);
    OneJob S;
    S.c.out = W ? out : nullptr;
    S.c.cnt = C ? cnt : nullptr;
    S.c.checksum = C ? (unsigned long long *)checksum : nullptr;
    S.c.wbase = (uint32_t)walk_base;
    S.c.L = L;
    S.c.k0 = (uint32_t)seed;
    S.c.k1 = (uint32_t)(seed >> 32);
    S.c.A_ret = A_ret;
    S.c.A_out = A_out;
    S.c.approx_t = approx_t;
    S.starts = starts;
    S.n = n_starts;
    S.cur = nullptr;
    hipStream_t st = (hipStream_t)stream;

    if (o.mode == N2V_MODE_PLAIN) {
        const size_t need = plain_ws(n_starts, L);
        if (!ws || ws_bytes < need) return set_error(N2V_ENOMEM, "n2v_walk: plain form needs %zu workspace bytes", need);
        if (((uintptr_t)ws & 255) != 0) return set_error(N2V_EINVAL, "n2v_walk: workspace not 256-byte aligned");
        if (replay) {
            if (W && C) return launch_plain_replayed<true, true>(g, E, S, ws, st);
            if (W) return launch_plain_replayed<true, false>(g, E, S, ws, st);
            return launch_plain_replayed<false, true>(g, E, S, ws, st);
        }
        if (W && C) return launch_plain<true, true>(E, S, ws, g->device, st);
        if (W) return launch_plain<true, false>(E, S, ws, g->device, st);
        return launch_plain<false, true>(E, S, ws, g->device, st);
    }
    return with_cursor(g, st, [&](uint32_t *cur) {
        S.cur = cur;
        if (W && C) return launch_persistent<true, true>(E, S, o, g->device, st);
        if (W) return launch_persistent<true, false>(E, S, o, g->device, st);
        return launch_persistent<false, true>(E, S, o, g->device, st);
    });
}

}  // namespace
}  // namespace n2v

extern "C" int n2v_walk_approx(const n2v_graph *g, const uint32_t *starts, uint32_t n_starts, uint64_t walk_base,
                               uint32_t L, float p, float q, uint64_t seed, uint32_t approx_t,
                               const n2v_exec_opts *opts, int outputs, uint32_t *out, uint32_t *cnt,
                               uint64_t *checksum, void *ws, size_t ws_bytes, void *stream)
{
    return walk_impl(g, starts, n_starts, walk_base, L, p, q, seed, approx_t, opts, outputs, out, cnt, checksum, ws,
                     ws_bytes, stream, true);
}

extern "C" int n2v_walk_ex(const n2v_graph *g, const uint32_t *starts, uint32_t n_starts, uint64_t walk_base,
                           uint32_t L, float p, float q, uint64_t seed, const n2v_exec_opts *opts, int outputs,
                           uint32_t *out, uint32_t *cnt, uint64_t *checksum, void *ws, size_t ws_bytes, void *stream)
{
    return n2v_walk_approx(g, starts, n_starts, walk_base, L, p, q, seed, 0, opts, outputs, out, cnt, checksum, ws,
                           ws_bytes, stream);
}

extern "C" int n2v_walk(const n2v_graph *g, const uint32_t *starts, uint32_t n_starts, uint32_t L, float p, float q,
                        uint64_t seed, uint32_t *out, void *stream)
{
    return n2v_walk_ex(g, starts, n_starts, 0, L, p, q, seed, nullptr, N2V_OUT_WALKS, out, nullptr, nullptr, nullptr,
                       0, stream);
}

// ----------------------------------------- plain form without allocation
// For callers that cannot allocate device memory (code under graph capture,
// tight serving loops, harnesses that forbid allocation): the plain form's
// scratch (per-walk state, the hub-move queue and per-superstep counters)
// lives in a fixed file-scope array that each GPU holds until the process
// ends.  Sizes: at most 2^21 walks of at most 1023 moves.
namespace n2v {
namespace {

constexpr uint32_t STATIC_MAX_WALKS = 1u << 21;
constexpr uint32_t STATIC_MAX_L = 1023;
// plain_ws(STATIC_MAX_WALKS, STATIC_MAX_L): 16-byte states and 4-byte queue
// entries per walk, four u32 counters per superstep, each piece 256-aligned
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)16 * STATIC_MAX_WALKS + (size_t)4 * STATIC_MAX_WALKS +
                                        (((size_t)16 * (STATIC_MAX_L + 1) + 255) & ~(size_t)255);

__device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

// Device address of this GPU's copy of `scratch` (the host-side name is only
// a stand-in), looked up once per device with that device current.
void *scratch_ptr(int dev, int *rc)
{
    static std::mutex mu;
    static void *ptr[64] = {};
    *rc = N2V_OK;
    if (dev < 0 || dev >= 64) {
        *rc = set_error(N2V_EDEVICE, "n2v_walk_static: device %d out of range", dev);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            *rc = hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
            return nullptr;
        }
        ptr[dev] = p;
    }
    return ptr[dev];
}

}  // namespace
}  // namespace n2v

extern "C" int n2v_walk_static(const n2v_graph *g, const uint32_t *starts, uint32_t n_starts, uint64_t walk_base,
                               uint32_t L, float p, float q, uint64_t seed, uint32_t approx_t,
                               const n2v_exec_opts *opts, int outputs, uint32_t *out, uint32_t *cnt,
                               uint64_t *checksum, void *stream)
{
    if (!g) return set_error(N2V_EINVAL, "n2v_walk_static: null graph");
    if (n_starts > STATIC_MAX_WALKS || L > STATIC_MAX_L)
        return set_error(N2V_ENOMEM, "n2v_walk_static: %u walks of %u moves exceed the static scratch (at most %u walks "
                         "of at most %u moves)", n_starts, L, STATIC_MAX_WALKS, STATIC_MAX_L);
    const size_t need = plain_ws(n_starts, L);
    if (need > STATIC_SCRATCH_BYTES)
        return set_error(N2V_ENOMEM, "n2v_walk_static: %zu scratch bytes needed, %zu held", need,
                         STATIC_SCRATCH_BYTES);
    int rc = N2V_OK;
    void *ws = scratch_ptr(g->device, &rc);
    if (rc) return rc;
    n2v_exec_opts o;
    n2v_exec_opts_default(g, &o);
    if (opts) o = *opts;
    o.mode = N2V_MODE_PLAIN;
    return walk_impl(g, starts, n_starts, walk_base, L, p, q, seed, approx_t, &o, outputs, out, cnt, checksum, ws,
                     STATIC_SCRATCH_BYTES, stream, false);
}
