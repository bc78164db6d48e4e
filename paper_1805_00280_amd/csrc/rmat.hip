// rmat.hip -- on-device R-MAT generator and CSR builder.
//
// R-MAT (Section 4.1 of the paper): each of edge_factor * 2^scale edges picks
// one of the four quadrants of the adjacency matrix with probabilities a, b,
// c, d, recursively from the top level down to single cells.  Every edge is
// generated independently from a counter-based Philox draw, so the kernel is
// a pure map over edge indices.
//
// CSR build: both directions of every non-loop edge become a packed key
// (u << scale) | v of 2*scale bits, LSD radix-sorted (8-bit digits, one
// wavefront per 4096-key tile, stable ranks from ballot-based digit matching),
// de-duplicated, counted per source (row offsets by exclusive scan) and
// compacted into adj (and wt).  A self-loop key of vertex n-1 is all ones, so
// dropped edges are written as that key and sort to the end.
#include "prims.hpp"

namespace n2v {

namespace {

constexpr int RS_KPT = 64;                           // keys per lane per tile
constexpr uint64_t RS_TILE = (uint64_t)WAVE * RS_KPT;  // keys per tile (one wavefront)

struct RmatDev {
    uint32_t scale;
    uint64_t M;
    uint64_t T0, T1, T2;
    uint32_t k0, k1;
};

__global__ __launch_bounds__(256) void k_rmat_keys(RmatDev p, uint64_t *__restrict__ keys)
{
    const uint64_t dead = (p.scale == 32) ? ~0ull : ((1ull << (2 * p.scale)) - 1ull);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < p.M; e += stride) {
        uint32_t u = 0, v = 0;
        R4 r{0, 0, 0, 0};
        for (uint32_t l = 0; l < p.scale; ++l) {
            if ((l & 3u) == 0) r = philox(p.k0, p.k1, (uint32_t)e, (uint32_t)(e >> 32), l >> 2, 1u);
            const uint32_t sel = l & 3u;
            const uint64_t w = sel == 0 ? r.x : sel == 1 ? r.y : sel == 2 ? r.z : r.w;
            const uint32_t q = (uint32_t)(w >= p.T0) + (uint32_t)(w >= p.T1) + (uint32_t)(w >= p.T2);
            u |= (q >> 1) << (p.scale - 1 - l);
            v |= (q & 1u) << (p.scale - 1 - l);
        }
        uint64_t a = dead, b = dead;
        if (u != v) {
            a = ((uint64_t)u << p.scale) | v;
            b = ((uint64_t)v << p.scale) | u;
        }
        keys[2 * e] = a;
        keys[2 * e + 1] = b;
    }
}

// Digit counts of one tile, stored digit-major: hist[d * ntiles + tile].
__global__ __launch_bounds__(WAVE) void k_rs_hist(const uint64_t *__restrict__ keys, uint64_t nkeys, int shift,
                                                  uint64_t *__restrict__ hist, uint64_t ntiles)
{
    __shared__ uint32_t cnt[256];
    const int l = lane_id();
    const uint64_t tile = blockIdx.x;
    for (int d = l; d < 256; d += WAVE) cnt[d] = 0;
    __syncthreads();
    const uint64_t base = tile * RS_TILE;
    for (int r = 0; r < RS_KPT; ++r) {
        const uint64_t i = base + (uint64_t)r * WAVE + l;
        if (i < nkeys) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (int d = l; d < 256; d += WAVE) hist[(uint64_t)d * ntiles + tile] = cnt[d];
}

// Stable scatter of one tile to the scanned digit offsets.
__global__ __launch_bounds__(WAVE) void k_rs_scatter(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                     uint64_t nkeys, int shift, const uint64_t *__restrict__ hoff,
                                                     uint64_t ntiles)
{
    __shared__ uint64_t base[256];
    const int l = lane_id();
    const uint64_t tile = blockIdx.x;
    for (int d = l; d < 256; d += WAVE) base[d] = hoff[(uint64_t)d * ntiles + tile];
    __syncthreads();
    const uint64_t t0 = tile * RS_TILE;
    for (int r = 0; r < RS_KPT; ++r) {
        const uint64_t i = t0 + (uint64_t)r * WAVE + l;
        const bool valid = i < nkeys;
        const uint64_t key = valid ? in[i] : 0;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lanemask_lt());
        const uint64_t pos = base[d] + rank;
        wave_lds_sync();
        if (valid) {
            out[pos] = key;
            if (l == first_lane(peers)) base[d] = pos - rank + __popcll(peers);
        }
        wave_lds_sync();
    }
}

// Per tile: number of distinct live keys.
__global__ __launch_bounds__(WAVE) void k_dd_count(const uint64_t *__restrict__ keys, uint64_t nkeys, uint64_t dead,
                                                   uint64_t *__restrict__ tcnt)
{
    const int l = lane_id();
    const uint64_t t0 = (uint64_t)blockIdx.x * RS_TILE;
    uint32_t c = 0;
    for (int r = 0; r < RS_KPT; ++r) {
        const uint64_t i = t0 + (uint64_t)r * WAVE + l;
        if (i < nkeys) {
            const uint64_t k = keys[i];
            c += (k != dead) && (i == 0 || keys[i - 1] != k);
        }
    }
    c = wave_sum32(c);
    if (l == 0) tcnt[blockIdx.x] = c;
}

// Per tile: write the distinct live keys to adj (and wt), count row lengths.
__global__ __launch_bounds__(WAVE) void k_dd_write(const uint64_t *__restrict__ keys, uint64_t nkeys, uint64_t dead,
                                                   uint32_t scale, const uint64_t *__restrict__ tbase,
                                                   uint32_t *__restrict__ adj, uint16_t *__restrict__ wt,
                                                   unsigned long long *__restrict__ deg, uint32_t k0, uint32_t k1)
{
    const int l = lane_id();
    const uint64_t t0 = (uint64_t)blockIdx.x * RS_TILE;
    const uint64_t vmask = (1ull << scale) - 1ull;
    uint64_t run = tbase[blockIdx.x];
    for (int r = 0; r < RS_KPT; ++r) {
        const uint64_t i = t0 + (uint64_t)r * WAVE + l;
        bool keep = false;
        uint64_t k = 0;
        if (i < nkeys) {
            k = keys[i];
            keep = (k != dead) && (i == 0 || keys[i - 1] != k);
        }
        const uint64_t m = ballot(keep);
        if (keep) {
            const uint64_t pos = run + __popcll(m & lanemask_lt());
            const uint32_t u = (uint32_t)(k >> scale), v = (uint32_t)(k & vmask);
            adj[pos] = v;
            if (wt) {
                const uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
                const R4 q = philox(k0, k1, lo, hi, 0u, 2u);
                wt[pos] = (uint16_t)(1u + (uint32_t)(((uint64_t)q.x * 1000u) >> 32));
            }
            atomicAdd(&deg[u], 1ull);
        }
        run += __popcll(m);
    }
}

__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

bool rmat_valid(const n2v_rmat_params *p)
{
    if (!p) return false;
    if (p->scale < 1 || p->scale > 31 || p->edge_factor < 1) return false;
    if (!(p->a >= 0 && p->b >= 0 && p->c >= 0 && p->a + p->b + p->c <= 1.0 + 1e-12)) return false;
    const uint64_t M = (uint64_t)p->edge_factor << p->scale;
    return M < (1ull << 40);
}

uint64_t threshold(double x)
{
    double y = x * 4294967296.0;
    if (y < 0.0) y = 0.0;
    if (y > 4294967296.0) y = 4294967296.0;
    return (uint64_t)llround(y);
}

struct RmatLayout {
    uint64_t nkeys, ntiles, n;
    uint64_t *kA, *kB, *hist, *tcnt, *deg;
    void *scan;
};

size_t rmat_layout(const n2v_rmat_params *p, void *ws, size_t ws_bytes, RmatLayout *L)
{
    const uint64_t M = (uint64_t)p->edge_factor << p->scale;
    L->n = 1ull << p->scale;
    L->nkeys = 2 * M;
    L->ntiles = (L->nkeys + RS_TILE - 1) / RS_TILE;
    Carver c(ws, ws_bytes);
    L->kA = c.take<uint64_t>(L->nkeys);
    L->kB = c.take<uint64_t>(L->nkeys);
    L->hist = c.take<uint64_t>(256 * L->ntiles);
    L->tcnt = c.take<uint64_t>(L->ntiles + 1);
    L->deg = c.take<uint64_t>(L->n + 1);
    uint64_t biggest = 256 * L->ntiles > L->n + 1 ? 256 * L->ntiles : L->n + 1;
    L->scan = c.take<char>(scan_scratch_bytes(biggest));
    return c.total();
}

}  // namespace

}  // namespace n2v

using namespace n2v;

extern "C" int n2v_rmat_workspace(const n2v_rmat_params *prm, size_t *ws_bytes, uint64_t *m_max)
{
    if (!rmat_valid(prm) || !ws_bytes) return set_error(N2V_EINVAL, "n2v_rmat_workspace: bad parameters");
    RmatLayout L;
    *ws_bytes = rmat_layout(prm, nullptr, 0, &L);
    if (m_max) *m_max = L.nkeys;
    return N2V_OK;
}

extern "C" int n2v_rmat_generate(const n2v_rmat_params *prm, void *ws, size_t ws_bytes, uint64_t *off, uint32_t *adj,
                                 uint16_t *wt, uint64_t *m_out, void *stream)
{
    if (!rmat_valid(prm)) return set_error(N2V_EINVAL, "n2v_rmat_generate: bad parameters");
    if (!off || !adj || !m_out || !ws) return set_error(N2V_EINVAL, "n2v_rmat_generate: null pointer");
    if (prm->weighted && !wt) return set_error(N2V_EINVAL, "n2v_rmat_generate: weighted graph needs wt");
    if (((uintptr_t)ws & 255) != 0) return set_error(N2V_EINVAL, "n2v_rmat_generate: workspace not 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    RmatLayout L;
    size_t need = rmat_layout(prm, ws, ws_bytes, &L);
    if (need > ws_bytes) return set_error(N2V_ENOMEM, "n2v_rmat_generate: workspace %zu < %zu bytes", ws_bytes, need);

    const uint32_t S = prm->scale;
    const uint64_t dead = (1ull << (2 * S)) - 1ull;
    RmatDev d;
    d.scale = S;
    d.M = (uint64_t)prm->edge_factor << S;
    d.T0 = threshold(prm->a);
    d.T1 = threshold(prm->a + prm->b);
    d.T2 = threshold(prm->a + prm->b + prm->c);
    d.k0 = (uint32_t)prm->seed;
    d.k1 = (uint32_t)(prm->seed >> 32);

    const uint32_t gen_blocks = (uint32_t)std::min<uint64_t>((d.M + 255) / 256, 1u << 20);
    hipLaunchKernelGGL(k_rmat_keys, dim3(gen_blocks), dim3(256), 0, st, d, L.kA);
    N2V_HIP(hipGetLastError());

    // LSD radix sort over the 2*scale significant bits
    uint64_t *src = L.kA, *dst = L.kB;
    const int bits = 2 * (int)S;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3((uint32_t)L.ntiles), dim3(WAVE), 0, st, src, L.nkeys, shift, L.hist,
                           L.ntiles);
        N2V_HIP(hipGetLastError());
        int rc = exclusive_scan_u64(L.hist, 256 * L.ntiles, L.scan, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_rs_scatter, dim3((uint32_t)L.ntiles), dim3(WAVE), 0, st, src, dst, L.nkeys, shift,
                           L.hist, L.ntiles);
        N2V_HIP(hipGetLastError());
        std::swap(src, dst);
    }

    // distinct live keys -> adj, wt and row lengths
    hipLaunchKernelGGL(k_dd_count, dim3((uint32_t)L.ntiles), dim3(WAVE), 0, st, src, L.nkeys, dead, L.tcnt);
    N2V_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, L.tcnt + L.ntiles, (uint64_t)1, (uint64_t)0);
    int rc = exclusive_scan_u64(L.tcnt, L.ntiles + 1, L.scan, st);
    if (rc) return rc;
    const uint32_t fb = (uint32_t)std::min<uint64_t>((L.n + 1 + 255) / 256, 1u << 16);
    hipLaunchKernelGGL(k_fill_u64, dim3(fb), dim3(256), 0, st, L.deg, L.n + 1, (uint64_t)0);
    hipLaunchKernelGGL(k_dd_write, dim3((uint32_t)L.ntiles), dim3(WAVE), 0, st, src, L.nkeys, dead, S, L.tcnt, adj,
                       prm->weighted ? wt : (uint16_t *)nullptr, (unsigned long long *)L.deg, d.k0, d.k1);
    N2V_HIP(hipGetLastError());
    rc = exclusive_scan_u64(L.deg, L.n + 1, L.scan, st);
    if (rc) return rc;
    N2V_HIP(hipMemcpyAsync(off, L.deg, (L.n + 1) * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    uint64_t m = 0;
    N2V_HIP(hipMemcpyAsync(&m, L.tcnt + L.ntiles, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    N2V_HIP(hipStreamSynchronize(st));
    *m_out = m;
    return N2V_OK;
}
