// graph.hip -- graph handle: validation of a caller's CSR and the derived
// arrays the walk kernels read (per-vertex records, reverse-entry positions,
// row weight sums and maxima).
#include <stdlib.h>

#include <algorithm>

#include "prims.hpp"

namespace n2v {

namespace {

enum : uint32_t { BAD_OFF = 1, BAD_ROW = 2, BAD_ASYM = 4, BAD_ENDS = 8 };

__global__ __launch_bounds__(256) void k_validate(const uint64_t *__restrict__ off, const uint32_t *__restrict__ adj,
                                                  const uint16_t *__restrict__ wt, uint32_t n, uint64_t m,
                                                  uint32_t *__restrict__ bad)
{
    const int l = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint64_t nw = (uint64_t)gridDim.x * blockDim.x / WAVE;
    if (wave == 0 && l == 0 && (off[0] != 0 || off[n] != m)) atomicOr(bad, BAD_ENDS);
    uint32_t flags = 0;
    for (uint64_t v = wave; v < n; v += nw) {
        const uint64_t lo = off[v], hi = off[v + 1];
        if (hi < lo || hi > m) {
            flags |= BAD_OFF;
            continue;
        }
        for (uint64_t e = lo + l; e < hi; e += WAVE) {
            const uint32_t x = adj[e];
            if (x >= n || x == (uint32_t)v) flags |= BAD_ROW;
            if (e > lo && adj[e - 1] >= x) flags |= BAD_ROW;
            if (wt && wt[e] == 0) flags |= BAD_ROW;
        }
    }
    if (flags) atomicOr(bad, flags);
}

__global__ __launch_bounds__(256) void k_derive(const uint64_t *__restrict__ off, const uint32_t *__restrict__ adj,
                                                const uint16_t *__restrict__ wt, uint32_t n, VRec *__restrict__ vrec,
                                                uint2 *__restrict__ erec, uint64_t *__restrict__ wsum,
                                                uint32_t *__restrict__ bad, uint32_t *__restrict__ wrange,
                                                int check_sym)
{
    const int l = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint64_t nw = (uint64_t)gridDim.x * blockDim.x / WAVE;
    uint32_t flags = 0;
    // graph-wide weight range: wrange[0] = max(0xFFFF - w), wrange[1] = max(w)
    uint32_t winv = 0, wall = 0;
    for (uint64_t v = wave; v < n; v += nw) {
        const uint64_t lo = off[v], hi = off[v + 1];
        uint32_t wm = 0;
        uint64_t ws = 0;
        for (uint64_t e = lo + l; e < hi; e += WAVE) {
            const uint32_t x = adj[e];
            const uint64_t xlo = off[x], xhi = off[x + 1];
            const uint64_t p = lower_bound_g(adj, xlo, xhi, (uint32_t)v);
            const bool found = p < xhi && adj[p] == (uint32_t)v;
            if (!found && check_sym) flags |= BAD_ASYM;
            erec[e] = make_uint2(x, found ? (uint32_t)(p - xlo) : SENT);
            const uint32_t w = wt ? wt[e] : 1u;
            wm = w > wm ? w : wm;
            winv = 0xFFFFu - w > winv ? 0xFFFFu - w : winv;
            ws += w;
        }
#pragma unroll
        for (int msk = 32; msk >= 1; msk >>= 1) {
            const uint32_t o = __shfl_xor(wm, msk, WAVE);
            wm = o > wm ? o : wm;
        }
        ws = wave_sum(ws);
        wall = wm > wall ? wm : wall;
        if (l == 0) {
            VRec r;
            r.off = lo;
            r.deg = (uint32_t)(hi - lo);
            r.wmax = hi > lo ? wm : 0u;
            vrec[v] = r;
            if (wsum) wsum[v] = ws;
        }
    }
#pragma unroll
    for (int msk = 32; msk >= 1; msk >>= 1) {
        const uint32_t o = __shfl_xor(winv, msk, WAVE);
        winv = o > winv ? o : winv;
    }
    if (l == 0) {
        if (winv) atomicMax(wrange, winv);
        if (wall) atomicMax(wrange + 1, wall);
    }
    if (flags) atomicOr(bad, flags);
}

// Sketch words of a vertex of degree d: d rows of memo_row_words(d).
__device__ __forceinline__ uint64_t sketch_words(uint64_t d, bool weighted) { return d * memo_row_words(weighted, d); }

// hbase[v] = sketch words of v when deg(v) >= dmin, else 0 (scanned afterwards).
__global__ void k_hub_len(const uint64_t *__restrict__ off, uint32_t n, uint64_t dmin, bool weighted,
                          uint64_t *__restrict__ hb)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
        const uint64_t d = v < n ? off[v + 1] - off[v] : 0;
        hb[v] = d >= dmin && d > 0 ? sketch_words(d, weighted) : 0;
    }
}

// Sketch words of the rows of degree in [2^k, 2^(k+1)), k = 0..63, over rows
// of degree >= dmin (a per-block histogram, then one atomic per bin).
__global__ __launch_bounds__(256) void k_deg_hist(const uint64_t *__restrict__ off, uint32_t n, uint64_t dmin,
                                                  bool weighted, unsigned long long *__restrict__ hist)
{
    __shared__ unsigned long long h[64];
    if (threadIdx.x < 64) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint64_t d = off[v + 1] - off[v];
        if (d >= dmin && d > 0) atomicAdd(&h[63 - __clzll((long long)d)], (unsigned long long)sketch_words(d, weighted));
    }
    __syncthreads();
    if (threadIdx.x < 64 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Entries of the rows of degree >= dmin (per-block reduction, one atomic
// per block).
__global__ __launch_bounds__(256) void k_deg_entries_ge(const uint64_t *__restrict__ off, uint32_t n, uint64_t dmin,
                                                        unsigned long long *__restrict__ out)
{
    unsigned long long acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint64_t d = off[v + 1] - off[v];
        if (d >= dmin) acc += d;
    }
    acc = wave_sum(acc);
    __shared__ unsigned long long part[256 / WAVE];
    if (lane_id() == 0) part[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < 256 / WAVE; ++i) t += part[i];
        if (t) atomicAdd(out, t);
    }
}

__global__ void k_zero_u64w(unsigned long long *p, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Sketch words of the rows of degree >= dmin (per-block reduction, one
// atomic per block).
__global__ __launch_bounds__(256) void k_deg_sum_ge(const uint64_t *__restrict__ off, uint32_t n, uint64_t dmin,
                                                    bool weighted, unsigned long long *__restrict__ out)
{
    unsigned long long acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint64_t d = off[v + 1] - off[v];
        if (d >= dmin && d > 0) acc += sketch_words(d, weighted);
    }
    acc = wave_sum(acc);
    __shared__ unsigned long long part[256 / WAVE];
    if (lane_id() == 0) part[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < 256 / WAVE; ++i) t += part[i];
        if (t) atomicAdd(out, t);
    }
}

__global__ void k_zero_u32(uint32_t *p, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

struct GraphLayout {
    VRec *vrec;
    uint2 *erec;
    uint64_t *wsum;
    uint64_t *hbase;
    void *scan;
    unsigned long long *hist;
    uint32_t *status;
    uint32_t *cursors;
};

size_t graph_layout(uint32_t n, uint64_t m, int weighted, void *ws, size_t ws_bytes, GraphLayout *L)
{
    Carver c(ws, ws_bytes);
    L->status = c.take<uint32_t>(64);
    L->cursors = c.take<uint32_t>((uint64_t)CURSOR_SLOTS * CURSOR_STRIDE);
    L->vrec = c.take<VRec>((uint64_t)n + 1);
    L->erec = c.take<uint2>(m ? m : 1);
    L->wsum = weighted ? c.take<uint64_t>((uint64_t)n + 1) : nullptr;
    L->hbase = c.take<uint64_t>((uint64_t)n + 1);
    L->scan = c.take<char>(scan_scratch_bytes((uint64_t)n + 1));
    L->hist = c.take<unsigned long long>(64);
    return c.total();
}

uint32_t grid_for_waves(uint64_t waves)
{
    uint64_t blocks = (waves + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    return (uint32_t)blocks;
}

}  // namespace

}  // namespace n2v

using namespace n2v;

extern "C" void n2v_graph_opts_default(n2v_graph_opts *o)
{
    if (!o) return;
    o->d_rule = 1024;
    o->a_cap = 1024;
    o->validate = 1;
}

extern "C" int n2v_graph_workspace(uint32_t n, uint64_t m, int weighted, size_t *ws_bytes)
{
    if (!ws_bytes) return set_error(N2V_EINVAL, "n2v_graph_workspace: null ws_bytes");
    if (n == 0 || n > 0xFFFFFFFEu) return set_error(N2V_EINVAL, "n2v_graph_workspace: n out of range");
    GraphLayout L;
    *ws_bytes = graph_layout(n, m, weighted, nullptr, 0, &L);
    return N2V_OK;
}

extern "C" int n2v_graph_create(const uint64_t *off, const uint32_t *adj, const uint16_t *wt, uint32_t n, uint64_t m,
                                const n2v_graph_opts *opts, void *ws, size_t ws_bytes, void *stream,
                                n2v_graph **out)
{
    if (!out) return set_error(N2V_EINVAL, "n2v_graph_create: null out");
    *out = nullptr;
    if (!off || (!adj && m) || !ws) return set_error(N2V_EINVAL, "n2v_graph_create: null pointer");
    if (n == 0 || n > 0xFFFFFFFEu) return set_error(N2V_EINVAL, "n2v_graph_create: n out of range");
    if (((uintptr_t)ws & 255) != 0) return set_error(N2V_EINVAL, "n2v_graph_create: workspace not 256-byte aligned");
    n2v_graph_opts o;
    n2v_graph_opts_default(&o);
    if (opts) o = *opts;
    if (o.a_cap < 1) return set_error(N2V_EINVAL, "n2v_graph_create: a_cap must be >= 1");
    GraphLayout L;
    size_t need = graph_layout(n, m, wt != nullptr, ws, ws_bytes, &L);
    if (need > ws_bytes) return set_error(N2V_ENOMEM, "n2v_graph_create: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;

    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, L.status, 64u);
    N2V_HIP(hipGetLastError());
    if (o.validate >= 1) {
        hipLaunchKernelGGL(k_validate, dim3(grid_for_waves(n)), dim3(256), 0, st, off, adj, wt, n, m, L.status + 1);
        N2V_HIP(hipGetLastError());
        uint32_t bad = 0;
        N2V_HIP(hipMemcpyAsync(&bad, L.status + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        N2V_HIP(hipStreamSynchronize(st));
        if (bad)
            return set_error(N2V_EGRAPH,
                             "n2v_graph_create: CSR violates the contract (flags 0x%x: 1 offsets, 2 row order/loop/"
                             "id/weight, 8 off[0] or off[n])",
                             bad);
    }
    hipLaunchKernelGGL(k_derive, dim3(grid_for_waves(n)), dim3(256), 0, st, off, adj, wt, n, L.vrec, L.erec, L.wsum,
                       L.status + 1, L.status + 2, o.validate >= 2 ? 1 : 0);
    N2V_HIP(hipGetLastError());
    if (o.validate >= 2) {
        uint32_t bad = 0;
        N2V_HIP(hipMemcpyAsync(&bad, L.status + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        N2V_HIP(hipStreamSynchronize(st));
        if (bad) return set_error(N2V_EGRAPH, "n2v_graph_create: CSR is not symmetric (flags 0x%x)", bad);
    }
    const uint64_t memo_min = (uint64_t)o.d_rule + 1;
    hipLaunchKernelGGL(k_hub_len, dim3(grid_for_waves(n)), dim3(256), 0, st, off, n, memo_min, wt != nullptr,
                       L.hbase);
    N2V_HIP(hipGetLastError());
    int rc = exclusive_scan_u64(L.hbase, (uint64_t)n + 1, L.scan, st);
    if (rc) return rc;
    uint64_t hub_words = 0;
    unsigned long long hub_entries = 0;
    uint32_t wrange[2] = {0, 0};
    hipLaunchKernelGGL(k_zero_u64w, dim3(1), dim3(64), 0, st, L.hist, 1u);
    hipLaunchKernelGGL(k_deg_entries_ge, dim3(grid_for_waves(n)), dim3(256), 0, st, off, n, memo_min, L.hist);
    N2V_HIP(hipGetLastError());
    N2V_HIP(hipMemcpyAsync(&hub_entries, L.hist, sizeof(hub_entries), hipMemcpyDeviceToHost, st));
    N2V_HIP(hipMemcpyAsync(&hub_words, L.hbase + n, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    N2V_HIP(hipMemcpyAsync(wrange, L.status + 2, sizeof(wrange), hipMemcpyDeviceToHost, st));
    N2V_HIP(hipStreamSynchronize(st));
    n2v_graph *g = (n2v_graph *)calloc(1, sizeof(n2v_graph));
    if (!g) return set_error(N2V_ENOMEM, "n2v_graph_create: host allocation failed");
    g->slots = cursor_slots_new();
    if (!g->slots) {
        free(g);
        return set_error(N2V_ENOMEM, "n2v_graph_create: host allocation failed");
    }
    g->hist = L.hist;
    g->servers = 0;
    g->dg.hbase = L.hbase;
    g->dg.memo = nullptr;
    g->hub_words = hub_words;
    g->hub_entries = hub_entries;
    g->memo_words = hub_words;
    g->scan = L.scan;
    g->memo_bytes = 0;
    g->dg.vrec = L.vrec;
    g->dg.erec = L.erec;
    g->dg.adj = adj;
    g->dg.wt = wt;
    g->dg.wsum = L.wsum;
    g->dg.status = L.status;
    g->dg.cursors = L.cursors;
    g->next_cursor = 0;
    g->dg.n = n;
    g->dg.m = m;
    g->dg.d_rule = o.d_rule;
    g->dg.memo_min = memo_min > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)memo_min;
    g->dg.a_cap = o.a_cap;
    g->dg.wlo = 1;
    g->dg.whi = 1;
    if (wt && m > 0) {
        g->dg.wlo = 0xFFFFu - wrange[0];
        g->dg.whi = wrange[1];
    }
    g->off = off;
    g->weighted = wt != nullptr;
    g->validate = o.validate;
    if (hipGetDevice(&g->device) != hipSuccess) g->device = 0;
    g->has_tuned = false;
    *out = g;
    return N2V_OK;
}

extern "C" int n2v_graph_destroy(n2v_graph *g)
{
    if (!g) return N2V_OK;
    if (__atomic_load_n(&g->servers, __ATOMIC_ACQUIRE) > 0)
        return set_error(N2V_EINVAL, "n2v_graph_destroy: %d server(s) still use this graph", g->servers);
    cursor_slots_free(g->slots);
    free(g);
    return N2V_OK;
}

extern "C" int n2v_graph_info(const n2v_graph *g, uint32_t *n, uint64_t *m, uint32_t *d_rule, uint32_t *a_cap,
                              int *weighted)
{
    if (!g) return set_error(N2V_EINVAL, "n2v_graph_info: null graph");
    if (n) *n = g->dg.n;
    if (m) *m = g->dg.m;
    if (d_rule) *d_rule = g->dg.d_rule;
    if (a_cap) *a_cap = g->dg.a_cap;
    if (weighted) *weighted = g->weighted;
    return N2V_OK;
}

extern "C" int n2v_graph_memo_bytes(const n2v_graph *g, size_t *bytes)
{
    if (!g || !bytes) return set_error(N2V_EINVAL, "n2v_graph_memo_bytes: null argument");
    *bytes = (size_t)g->hub_words * sizeof(uint16_t);
    return N2V_OK;
}

namespace {

// Sketch words of the rows of degree >= dmin, through the graph's statistics
// words (synchronous on the default stream).
unsigned long long deg_sum_ge(const n2v_graph *g, uint64_t dmin, int *rc)
{
    unsigned long long e = 0;
    *rc = N2V_OK;
    hipLaunchKernelGGL(k_zero_u64w, dim3(1), dim3(64), 0, 0, g->hist, 1u);
    hipLaunchKernelGGL(k_deg_sum_ge, dim3(grid_for_waves(g->dg.n)), dim3(256), 0, 0, g->off, g->dg.n, dmin,
                       g->weighted != 0, g->hist);
    hipError_t err = hipGetLastError();
    if (err == hipSuccess) err = hipMemcpy(&e, g->hist, sizeof(e), hipMemcpyDeviceToHost);
    if (err != hipSuccess) *rc = hip_fail(err, "degree sum");
    return e;
}

}  // namespace

extern "C" int n2v_graph_memo_plan(const n2v_graph *g, size_t budget, uint32_t *min_degree, size_t *bytes)
{
    if (!g || !min_degree || !bytes) return set_error(N2V_EINVAL, "n2v_graph_memo_plan: null argument");
    const size_t row = sizeof(uint16_t);  // bytes per sketch word
    const uint64_t dmin = (uint64_t)g->dg.d_rule + 1;
    if (g->hub_words * row <= budget) {
        *min_degree = (uint32_t)std::min<uint64_t>(dmin, 0xFFFFFFFFull);
        *bytes = g->hub_words * row;
        return N2V_OK;
    }
    // degree statistics go through 64 words of the graph's own workspace
    unsigned long long *hist = g->hist;
    unsigned long long h[64];
    hipLaunchKernelGGL(k_zero_u64w, dim3(1), dim3(64), 0, 0, hist, 64u);
    hipLaunchKernelGGL(k_deg_hist, dim3(grid_for_waves(g->dg.n)), dim3(256), 0, 0, g->off, g->dg.n, dmin,
                       g->weighted != 0, hist);
    N2V_HIP(hipGetLastError());
    N2V_HIP(hipMemcpy(h, hist, sizeof(h), hipMemcpyDeviceToHost));
    int rc = N2V_OK;
    // the first power of two above d_rule whose rows fit brackets the answer:
    // the threshold below it (half of it, or d_rule + 1) does not fit
    uint64_t lo = 0, hi = 0, hi_e = 0;
    for (int k = 0; k < 64 && !hi; ++k) {
        const uint64_t t = 1ull << k;
        if (t <= dmin) continue;
        uint64_t e = 0;
        for (int b = k; b < 64; ++b) e += h[b];
        if (e * row <= budget) {
            lo = std::max<uint64_t>(dmin, t / 2);
            hi = t;
            hi_e = e;
        }
    }
    // then the smallest threshold in (lo, hi] whose rows fit, by bisection
    // over one-pass sums of the degrees at or above a candidate
    while (!rc && hi && hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        const unsigned long long e = deg_sum_ge(g, mid, &rc);
        if (rc) break;
        if (e * row <= budget) {
            hi = mid;
            hi_e = e;
        } else {
            lo = mid;
        }
    }
    if (rc) return rc;
    if (hi && hi <= 0xFFFFFFFFull) {
        *min_degree = (uint32_t)hi;
        *bytes = hi_e * row;
        return N2V_OK;
    }
    *min_degree = 0xFFFFFFFFu;
    *bytes = 0;
    return N2V_OK;
}

namespace {

__global__ void k_clear_words(uint32_t *p, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

int clear_memo(void *mem, size_t bytes, hipStream_t st)
{
    const uint64_t words = (uint64_t)bytes / 4;
    if (words == 0) return N2V_OK;
    hipLaunchKernelGGL(k_clear_words, dim3((uint32_t)std::min<uint64_t>((words + 255) / 256, 65536)), dim3(256), 0,
                       st, (uint32_t *)mem, words);
    N2V_HIP(hipGetLastError());
    return N2V_OK;
}

}  // namespace

extern "C" int n2v_graph_set_memo_min(n2v_graph *g, void *mem, size_t bytes, uint32_t min_degree)
{
    if (!g) return set_error(N2V_EINVAL, "n2v_graph_set_memo_min: null graph");
    if (__atomic_load_n(&g->servers, __ATOMIC_ACQUIRE) > 0)
        return set_error(N2V_EINVAL, "n2v_graph_set_memo: %d server(s) use this graph's sketches", g->servers);
    if (!mem) {
        g->dg.memo = nullptr;
        g->memo_bytes = 0;
        return N2V_OK;
    }
    if (((uintptr_t)mem & 255) != 0) return set_error(N2V_EINVAL, "n2v_graph_set_memo: memory not 256-byte aligned");
    const uint64_t dmin = std::max<uint64_t>(min_degree, (uint64_t)g->dg.d_rule + 1);
    // the rows the threshold keeps are counted before anything changes, so a
    // refusal leaves the handle exactly as it was
    uint64_t words = g->memo_words;
    if (dmin != g->dg.memo_min) {
        int rc = N2V_OK;
        words = deg_sum_ge(g, dmin, &rc);
        if (rc) return rc;
    }
    const size_t need = (size_t)words * sizeof(uint16_t);
    if (bytes < need) return set_error(N2V_ENOMEM, "n2v_graph_set_memo: %zu < %zu bytes", bytes, need);
    // detached while the rows are re-indexed: a failure below leaves no
    // memory attached rather than memory indexed for another threshold
    g->dg.memo = nullptr;
    g->memo_bytes = 0;
    if (dmin != g->dg.memo_min) {
        hipLaunchKernelGGL(k_hub_len, dim3(grid_for_waves(g->dg.n)), dim3(256), 0, 0, g->off, g->dg.n, dmin,
                           g->weighted != 0, (uint64_t *)g->dg.hbase);
        N2V_HIP(hipGetLastError());
        int rc = exclusive_scan_u64((uint64_t *)g->dg.hbase, (uint64_t)g->dg.n + 1, g->scan, 0);
        if (rc) return rc;
        g->memo_words = words;
        g->dg.memo_min = (uint32_t)std::min<uint64_t>(dmin, 0xFFFFFFFFull);
    }
    // every entry starts unknown
    int rc = clear_memo(mem, bytes, 0);
    if (rc) return rc;
    N2V_HIP(hipDeviceSynchronize());
    g->dg.memo = (uint16_t *)mem;
    g->memo_bytes = bytes;
    return N2V_OK;
}

extern "C" int n2v_graph_memo_clear(n2v_graph *g, void *stream)
{
    if (!g) return set_error(N2V_EINVAL, "n2v_graph_memo_clear: null graph");
    if (!g->dg.memo) return N2V_OK;
    return clear_memo(g->dg.memo, g->memo_bytes, (hipStream_t)stream);
}

extern "C" int n2v_graph_set_memo(n2v_graph *g, void *mem, size_t bytes)
{
    if (!g) return set_error(N2V_EINVAL, "n2v_graph_set_memo: null graph");
    if (!mem) return n2v_graph_set_memo_min(g, nullptr, 0, 0);
    size_t need = 0;
    n2v_graph_memo_bytes(g, &need);
    if (need == 0)
        return set_error(N2V_EINVAL, "n2v_graph_set_memo: no pair sketches (no row above d_rule)");
    if (bytes < need) return set_error(N2V_ENOMEM, "n2v_graph_set_memo: %zu < %zu bytes", bytes, need);
    return n2v_graph_set_memo_min(g, mem, bytes, g->dg.d_rule + 1 > g->dg.d_rule ? g->dg.d_rule + 1 : g->dg.d_rule);
}

// Visit profile: vertices and summed visit counts per equi-width degree
// bucket (bucket k >= 1 holds degrees in ((k-1) width, k width], bucket 0 the
// isolated vertices, the last bucket everything above).  Per-block LDS
// histograms, then one atomic per nonzero bin.
constexpr uint32_t PROFILE_MAX_BUCKETS = 2048;

__global__ __launch_bounds__(256) void k_visit_profile(const VRec *__restrict__ vrec, const uint32_t *__restrict__ cnt,
                                                       uint32_t n, uint32_t width, uint32_t nb,
                                                       unsigned long long *__restrict__ verts,
                                                       unsigned long long *__restrict__ visits)
{
    __shared__ unsigned long long hv[PROFILE_MAX_BUCKETS], hc[PROFILE_MAX_BUCKETS];
    for (uint32_t k = threadIdx.x; k < nb; k += blockDim.x) {
        hv[k] = 0;
        hc[k] = 0;
    }
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint64_t d = vrec[v].deg;
        const uint64_t k = (d + width - 1) / width;
        const uint32_t b = k < nb - 1 ? (uint32_t)k : nb - 1;
        atomicAdd(&hv[b], 1ull);
        const uint32_t c = cnt[v];
        if (c) atomicAdd(&hc[b], (unsigned long long)c);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < nb; k += blockDim.x) {
        if (hv[k]) atomicAdd(&verts[k], hv[k]);
        if (hc[k]) atomicAdd(&visits[k], hc[k]);
    }
}

__global__ void k_zero_u64(unsigned long long *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

extern "C" int n2v_visit_profile(const n2v_graph *g, const uint32_t *cnt, uint32_t width, uint32_t nbuckets,
                                 uint64_t *vertices, uint64_t *visits, void *stream)
{
    if (!g || !cnt || !vertices || !visits) return set_error(N2V_EINVAL, "n2v_visit_profile: null argument");
    if (width < 1 || nbuckets < 2 || nbuckets > PROFILE_MAX_BUCKETS)
        return set_error(N2V_EINVAL, "n2v_visit_profile: width >= 1 and 2 <= nbuckets <= %u", PROFILE_MAX_BUCKETS);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_u64, dim3((nbuckets + 255) / 256), dim3(256), 0, st, (unsigned long long *)vertices,
                       nbuckets);
    hipLaunchKernelGGL(k_zero_u64, dim3((nbuckets + 255) / 256), dim3(256), 0, st, (unsigned long long *)visits,
                       nbuckets);
    N2V_HIP(hipGetLastError());
    if (g->dg.n == 0) return N2V_OK;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(((uint64_t)g->dg.n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_visit_profile, dim3(blocks), dim3(256), 0, st, g->dg.vrec, cnt, g->dg.n, width, nbuckets,
                       (unsigned long long *)vertices, (unsigned long long *)visits);
    N2V_HIP(hipGetLastError());
    return N2V_OK;
}

extern "C" int n2v_graph_check(const n2v_graph *g, void *stream)
{
    if (!g) return set_error(N2V_EINVAL, "n2v_graph_check: null graph");
    hipStream_t st = (hipStream_t)stream;
    uint32_t flag = 0;
    N2V_HIP(hipMemcpyAsync(&flag, g->dg.status, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    N2V_HIP(hipStreamSynchronize(st));
    if (flag) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, g->dg.status, 1u);
        N2V_HIP(hipGetLastError());
        N2V_HIP(hipStreamSynchronize(st));
        if (flag & 2u) return set_error(N2V_EDEVICE, "n2v_graph_check: internal error in an inverse-CDF move");
        return set_error(N2V_EINVAL, "n2v_graph_check: a walk had a start id >= n");
    }
    return N2V_OK;
}
