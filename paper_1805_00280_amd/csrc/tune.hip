// tune.hip -- autotuner of the persistent kernel's execution parameters.
//
// It times the persistent kernel on a seeded sample of walks (start vertices
// drawn uniformly over all vertices, the same distribution as walks from
// every vertex) under candidate settings of the degree thresholds, the
// sparse/dense hub cost weight, the grid size and the stream/search switch of
// dense merges, by coordinate descent, and
// stores the fastest setting in the graph.  Execution parameters never change
// outputs, so tuning cannot change any result.
#include <vector>

#include "prims.hpp"
#include "walk.hpp"

namespace n2v {

namespace {

__global__ void k_sample_starts(uint32_t *starts, uint32_t count, uint32_t n, uint32_t k0)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const R4 r = philox(k0, 0x6e327674u, i, 0u, 0u, 7u);
        starts[i] = (uint32_t)(((uint64_t)r.x * n) >> 32);
    }
}

struct TuneLayout {
    uint32_t *starts;
    uint32_t *out;
};

size_t tune_layout(uint32_t n_walks, uint32_t L, void *ws, size_t ws_bytes, TuneLayout *T)
{
    Carver c(ws, ws_bytes);
    T->starts = c.take<uint32_t>(n_walks);
    T->out = c.take<uint32_t>((uint64_t)n_walks * (L + 1));
    return c.total();
}

}  // namespace

}  // namespace n2v

using namespace n2v;

extern "C" int n2v_autotune_workspace(const n2v_graph *g, uint32_t n_walks, uint32_t L, size_t *ws_bytes)
{
    if (!g || !ws_bytes || n_walks == 0 || L == 0) return set_error(N2V_EINVAL, "n2v_autotune_workspace: bad argument");
    TuneLayout T;
    *ws_bytes = tune_layout(n_walks, L, nullptr, 0, &T);
    return N2V_OK;
}

extern "C" int n2v_autotune(n2v_graph *g, uint32_t n_walks, uint32_t L, float p, float q, void *ws, size_t ws_bytes,
                            void *stream, n2v_exec_opts *best, double *best_ms)
{
    if (!g || !ws || n_walks == 0 || L == 0) return set_error(N2V_EINVAL, "n2v_autotune: bad argument");
    uint32_t A_ret, A_out;
    if (walk_multipliers(p, q, &A_ret, &A_out)) return set_error(N2V_EINVAL, "n2v_autotune: bad p or q");
    TuneLayout T;
    const size_t need = tune_layout(n_walks, L, ws, ws_bytes, &T);
    if (need > ws_bytes) return set_error(N2V_ENOMEM, "n2v_autotune: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_sample_starts, dim3((n_walks + 255) / 256), dim3(256), 0, st, T.starts, n_walks, g->dg.n,
                       0x5eedu);
    N2V_HIP(hipGetLastError());

    JobCtx c;
    c.out = T.out;
    c.cnt = nullptr;
    c.checksum = nullptr;
    c.wbase = 0;
    c.L = L;
    c.k0 = 0x1234567u;
    c.k1 = 0;
    c.A_ret = A_ret;
    c.A_out = A_out;
    c.approx_t = 0;

    // events released on every return path
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events()
        {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    N2V_HIP(hipEventCreate(&ev.a));
    N2V_HIP(hipEventCreate(&ev.b));
    // Each candidate is timed from cold pair sketches, as a fresh pass over a
    // graph meets them: the sketches are cleared before its warm-up launch and
    // again before its timed launch, so no candidate reuses merges that the
    // warm-up or an earlier candidate made on the same sample.
    auto run = [&](const n2v_exec_opts &o, double *ms) -> int {
        Exec E;
        make_exec(g, o, &E);
        int rc = n2v_graph_memo_clear(g, st);
        if (!rc) rc = launch_one(g, E, c, T.starts, n_walks, o, st);  // warm-up
        if (!rc) rc = n2v_graph_memo_clear(g, st);
        if (rc) return rc;
        N2V_HIP(hipEventRecord(ev.a, st));
        rc = launch_one(g, E, c, T.starts, n_walks, o, st);
        if (rc) return rc;
        N2V_HIP(hipEventRecord(ev.b, st));
        N2V_HIP(hipEventSynchronize(ev.b));
        float f = 0;
        N2V_HIP(hipEventElapsedTime(&f, ev.a, ev.b));
        *ms = f;
        return N2V_OK;
    };

    n2v_exec_opts cur;
    g->has_tuned = false;
    n2v_exec_opts_default(g, &cur);
    cur.mode = N2V_MODE_PERSISTENT;
    double cur_ms = 0;
    int rc = run(cur, &cur_ms);
    if (rc) return rc;
    const uint32_t t_wave_c[] = {0, 8, 32, 64, 128, 256, 1024};
    // sparse_ratio 2^20 keeps every hub move on the dense path
    const uint32_t ratio_c[] = {1, 2, 4, 8, 16, 32, 1u << 20};
    const uint32_t waves_c[] = {0, 8, 12, 16};
    const uint32_t search_c[] = {0, 2, 4, 8, 16, 64, 0xFFFFFFFFu};
    for (int pass = 0; pass < 4; ++pass) {
        const uint32_t *vals = pass == 0 ? t_wave_c : pass == 1 ? ratio_c : pass == 2 ? waves_c : search_c;
        const int nv = pass == 0 ? 7 : pass == 1 ? 7 : pass == 2 ? 4 : 7;
        for (int i = 0; i < nv; ++i) {
            n2v_exec_opts o = cur;
            if (pass == 0) o.t_wave = vals[i];
            if (pass == 1) o.sparse_ratio = vals[i];
            if (pass == 2) o.waves_per_cu = vals[i];
            if (pass == 3) o.search_ratio = vals[i];
            double ms = 0;
            rc = run(o, &ms);
            if (rc) return rc;
            if (ms < cur_ms) {
                cur = o;
                cur_ms = ms;
            }
        }
    }
    // leave the sketches cold for the caller's next pass
    rc = n2v_graph_memo_clear(g, st);
    if (rc) return rc;
    cur.mode = N2V_MODE_AUTO;
    g->tuned = cur;
    g->has_tuned = true;
    if (best) *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return N2V_OK;
}
