#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
/* Drives the CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
 * R-MAT CSR, exact and FN-Approx walks with counts and checksum, the cost
 * model, and the FN-Approx gap decision at extreme degrees and weights. */
typedef struct or_graph or_graph;
int or_rmat_csr(uint32_t, uint32_t, double, double, double, uint64_t, uint64_t *, uint32_t *, uint16_t *, uint64_t,
                uint64_t *, int);
or_graph *or_graph_new(const uint64_t *, const uint32_t *, const uint16_t *, uint32_t);
void or_graph_free(or_graph *);
int or_walk(const or_graph *, const uint32_t *, const uint64_t *, uint64_t, uint64_t, uint32_t, double, double,
            uint64_t, uint32_t, uint32_t, uint32_t, uint32_t *, uint32_t *, uint64_t *, uint64_t *, int);
int or_walk_cost(const or_graph *, const uint32_t *, const uint64_t *, uint64_t, uint32_t, double, double, uint64_t,
                 uint32_t, uint32_t, uint32_t, uint64_t *, uint64_t *, uint64_t *, int);
int or_approx_gap_below(uint64_t, uint64_t, const uint32_t *, uint32_t, uint32_t, uint32_t);
int main(void)
{
    for (int weighted = 0; weighted < 2; ++weighted) {
        const uint32_t scale = 11, ef = 16, n = 1u << scale;
        const uint64_t cap = 2ull * ef * n;
        uint64_t *off = malloc((n + 1) * sizeof(uint64_t)), m = 0;
        uint32_t *adj = malloc(cap * sizeof(uint32_t));
        uint16_t *wt = weighted ? malloc(cap * sizeof(uint16_t)) : NULL;
        if (or_rmat_csr(scale, ef, 0.65, 0.15, 0.15, 11, off, adj, wt, cap, &m, 4)) return 1;
        or_graph *g = or_graph_new(off, adj, wt, n);
        const uint32_t W = 3 * n, L = 30;
        uint32_t *st = malloc(W * sizeof(uint32_t)), *out = malloc((uint64_t)W * (L + 1) * sizeof(uint32_t));
        uint32_t *cnt = calloc(n, sizeof(uint32_t));
        uint64_t *wid = malloc(64 * sizeof(uint64_t));
        for (uint32_t i = 0; i < W; ++i) st[i] = i % n;
        for (int i = 0; i < 64; ++i) wid[i] = (uint64_t)i * 977u;
        const double pq[3][2] = {{0.25, 4.0}, {2.0, 0.5}, {1.0, 1.0}};
        for (int k = 0; k < 3; ++k)
            for (uint32_t T = 0; T <= 100; T += 100) {
                uint64_t cs = 0, tr = 0, b = 0, s = 0, h = 0;
                if (or_walk(g, st, NULL, 0, W, L, pq[k][0], pq[k][1], 7, 64, 1024, T, out, cnt, &cs, &tr, 4)) return 2;
                if (or_walk_cost(g, st, wid, 64, L, pq[k][0], pq[k][1], 7, 64, 1024, T, &b, &s, &h, 4)) return 3;
                printf("weighted=%d p=%g q=%g T=%u moves=%llu checksum=%016llx cost=%llu\n", weighted, pq[k][0],
                       pq[k][1], T, (unsigned long long)tr, (unsigned long long)cs, (unsigned long long)b);
            }
        const uint32_t A[3] = {16, 4, 1};
        int acc = 0;
        for (uint64_t dv = 1025; dv < (1ull << 32); dv = dv * 7 + 3)
            acc += or_approx_gap_below(1024, dv, A, 1, 65535, 0xFFFFFFFFu);
        printf("gap decisions at extreme sizes: %d\n", acc);
        or_graph_free(g);
        free(off); free(adj); free(wt); free(st); free(out); free(cnt); free(wid);
    }
    return 0;
}
