/*
 * oracle.c -- plain CPU reference for node2vec biased second-order random
 * walks whose transition probabilities are computed on the fly.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark, and by nothing
 * else.  It shares no source, header, table or generator with the GPU
 * library: every function below is written directly from the definitions it
 * cites, in the simplest form that is still fast enough to be useful.
 *
 * What it follows (Zhou, Niu, Chen, "Efficient Graph Computation for
 * Node2Vec"):
 *   - Section 2.1 (node2vec random walk): the unnormalised probability of
 *     moving from the current vertex v to a neighbour x is w_vx * alpha(t,x),
 *     where alpha depends on the distance between x and the previous vertex
 *     t: 1/p when x is t, 1 when x is a common neighbour, 1/q otherwise.  The
 *     three cases are the ones Section 3.2 tests for; the values 1/p, 1, 1/q
 *     follow from the bound derivation of the FN-Approx paragraph in Section
 *     3.4 (minimal alpha 1 when x is not t, maximal 1/q when 1/p <= 1 <= 1/q).
 *   - Algorithm 1 (FN-Base): the first move of a walk is drawn from the
 *     static edge weights only; every later move is second-order; each
 *     vertex starts r walks; the walk length counts moves.
 *   - Section 4.1 (data sets): R-MAT picks one of the four quadrants with
 *     probabilities a, b, c, d recursively down to single cells.
 *   - Section 3.4 (FN-Approx, Eqs. 2 and 3): at a popular vertex reached
 *     from an unpopular one, a move whose probability bounds differ by less
 *     than a threshold is drawn from the static weights; the readings are
 *     listed where the rule is defined below.
 *
 * Readings of points the paper leaves open (the integer draw rule):
 *   - multipliers are integers: A_ret = 4/p, A_com = 4, A_out = 4/q, with
 *     p, q in {1/4, 1/2, 1, 2, 4}; 4*alpha is then exact, so the law below is
 *     exactly node2vec's law;
 *   - randomness is Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *     key = (seed mod 2^32, seed >> 32), counter = (walk mod 2^32, step,
 *     attempt, 0); R1 = r0*2^32 + r1, R2 = r2*2^32 + r3;
 *     hi64(x, y) = floor(x*y / 2^64);
 *   - vertices of degree d <= d_rule: rejection.  E = wmax(v) at step 0,
 *     A_max*wmax(v) later; attempt k draws j = hi64(R1, d), u = hi64(R2, E)
 *     and accepts neighbour j iff u < pi_j; after a_cap failed attempts the
 *     inverse-CDF rule runs with attempt index a_cap;
 *   - vertices of degree d > d_rule: inverse CDF with attempt index 0:
 *     S = sum pi_j, r = hi64(R1, S), answer = first i (CSR order) whose
 *     prefix sum P_i exceeds r;
 *   - a vertex with no neighbours ends the walk; the remaining entries of
 *     its row are 0xFFFFFFFF.
 *
 * Parity pins: see the test suite (Philox known-answer vectors, exact laws
 * on tiny graphs by enumeration, closed forms on cycles, cliques, complete
 * bipartite graphs and stars, R-MAT quadrant statistics).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_SENT 0xFFFFFFFFu

typedef unsigned __int128 or_u128;

/* ---------------------------------------------------------------------- */
/* Philox4x32-10, Salmon et al. SC'11: ten rounds of two 32x32->64 bit     */
/* multiplications with the Weyl key schedule.                             */
/* ---------------------------------------------------------------------- */
void or_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void ph(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t r[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    or_philox((uint32_t)seed, (uint32_t)(seed >> 32), ctr, r);
}

static uint64_t hi64(uint64_t x, uint64_t y)
{
    return (uint64_t)(((or_u128)x * (or_u128)y) >> 64);
}

uint64_t or_hi64(uint64_t x, uint64_t y) { return hi64(x, y); }

/* ---------------------------------------------------------------------- */
/* Small thread pool helper: run fn(arg, tid, nthreads) on nthreads.       */
/* ---------------------------------------------------------------------- */
typedef void (*or_task_fn)(void *arg, int tid, int nthreads);
typedef struct { or_task_fn fn; void *arg; int tid, nth; } or_task;

static void *or_task_main(void *p)
{
    or_task *t = (or_task *)p;
    t->fn(t->arg, t->tid, t->nth);
    return NULL;
}

static void or_parallel(or_task_fn fn, void *arg, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads == 1) { fn(arg, 0, 1); return; }
    pthread_t th[256];
    or_task tk[256];
    for (int i = 0; i < nthreads; ++i) {
        tk[i].fn = fn; tk[i].arg = arg; tk[i].tid = i; tk[i].nth = nthreads;
        pthread_create(&th[i], NULL, or_task_main, &tk[i]);
    }
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
}

/* ---------------------------------------------------------------------- */
/* R-MAT (Section 4.1).  Edge e picks `scale` quadrants, top level first;  */
/* level l uses word (l mod 4) of Philox(key=g; ctr=(e lo, e hi, l/4, 1)). */
/* Quadrant = [w>=T1]+[w>=T2]+[w>=T3] in the order top-left, top-right,    */
/* bottom-left, bottom-right; its high bit is the row (source) bit and its */
/* low bit the column (target) bit of position scale-1-l.                  */
/* ---------------------------------------------------------------------- */
void or_rmat_thresholds(double a, double b, double c, uint64_t T[3])
{
    double x[3] = {a, a + b, a + b + c};
    for (int i = 0; i < 3; ++i) {
        double y = x[i] * 4294967296.0;
        if (y < 0.0) y = 0.0;
        if (y > 4294967296.0) y = 4294967296.0;
        T[i] = (uint64_t)llround(y);
    }
}

void or_rmat_edge(uint32_t scale, const uint64_t T[3], uint64_t gseed, uint64_t e,
                  uint32_t *u_out, uint32_t *v_out)
{
    uint32_t u = 0, v = 0, r[4] = {0, 0, 0, 0};
    for (uint32_t l = 0; l < scale; ++l) {
        if (l % 4 == 0) ph(gseed, (uint32_t)e, (uint32_t)(e >> 32), l / 4, 1, r);
        uint64_t word = r[l % 4];
        uint32_t quad = (uint32_t)(word >= T[0]) + (uint32_t)(word >= T[1]) + (uint32_t)(word >= T[2]);
        u |= (quad >> 1) << (scale - 1 - l);
        v |= (quad & 1u) << (scale - 1 - l);
    }
    *u_out = u;
    *v_out = v;
}

/* Raw edge list (for generator statistics): u[e], v[e] for e < count. */
typedef struct {
    uint32_t scale; uint64_t T[3]; uint64_t gseed; uint64_t e0, count;
    uint32_t *u, *v;
} or_raw_job;

static void or_raw_task(void *p, int tid, int nth)
{
    or_raw_job *j = (or_raw_job *)p;
    uint64_t lo = j->count * (uint64_t)tid / (uint64_t)nth;
    uint64_t hi = j->count * (uint64_t)(tid + 1) / (uint64_t)nth;
    for (uint64_t i = lo; i < hi; ++i)
        or_rmat_edge(j->scale, j->T, j->gseed, j->e0 + i, &j->u[i], &j->v[i]);
}

void or_rmat_raw(uint32_t scale, double a, double b, double c, uint64_t gseed,
                 uint64_t e0, uint64_t count, uint32_t *u, uint32_t *v, int nthreads)
{
    or_raw_job j;
    j.scale = scale; j.gseed = gseed; j.e0 = e0; j.count = count; j.u = u; j.v = v;
    or_rmat_thresholds(a, b, c, j.T);
    or_parallel(or_raw_task, &j, nthreads);
}

/* Symmetric weight of the unordered pair {x, y}: 1 + floor(r0*1000/2^32),  */
/* r0 = word 0 of Philox(key=g; ctr=(min, max, 0, 2)).                      */
uint16_t or_pair_weight(uint64_t gseed, uint32_t x, uint32_t y)
{
    uint32_t lo = x < y ? x : y, hi = x < y ? y : x, r[4];
    ph(gseed, lo, hi, 0, 2, r);
    return (uint16_t)(1u + (uint32_t)(((uint64_t)r[0] * 1000u) >> 32));
}

/* CSR of the symmetrised, de-duplicated, loop-free R-MAT edge set.        */
/* Construction: count both directions of every non-loop edge per source,  */
/* scatter, sort each row, drop repeats.                                   */
typedef struct {
    uint32_t scale; uint64_t T[3]; uint64_t gseed; uint64_t M; uint32_t n;
    uint64_t *cnt;      /* n: directed entries per source (with repeats) */
    uint64_t *cursor;   /* n: scatter cursors */
    uint32_t *raw;      /* sum cnt */
    uint64_t *rowstart; /* n+1 */
    uint64_t *ucnt;     /* n: entries per row after de-dup */
    uint64_t *off;      /* n+1 output */
    uint32_t *adj;      /* output */
    uint16_t *wt;       /* output or NULL */
    int phase;
    uint64_t next_row;  /* dynamic row scheduling */
} or_csr_job;

static int or_cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

static void or_csr_task(void *p, int tid, int nth)
{
    or_csr_job *j = (or_csr_job *)p;
    if (j->phase == 0 || j->phase == 1) {
        uint64_t lo = j->M * (uint64_t)tid / (uint64_t)nth;
        uint64_t hi = j->M * (uint64_t)(tid + 1) / (uint64_t)nth;
        for (uint64_t e = lo; e < hi; ++e) {
            uint32_t u, v;
            or_rmat_edge(j->scale, j->T, j->gseed, e, &u, &v);
            if (u == v) continue;
            if (j->phase == 0) {
                __atomic_fetch_add(&j->cnt[u], 1, __ATOMIC_RELAXED);
                __atomic_fetch_add(&j->cnt[v], 1, __ATOMIC_RELAXED);
            } else {
                uint64_t pu = __atomic_fetch_add(&j->cursor[u], 1, __ATOMIC_RELAXED);
                uint64_t pv = __atomic_fetch_add(&j->cursor[v], 1, __ATOMIC_RELAXED);
                j->raw[pu] = v;
                j->raw[pv] = u;
            }
        }
        return;
    }
    /* phases 2 and 3: rows handed out in blocks of 1024 */
    for (;;) {
        uint64_t r0 = __atomic_fetch_add(&j->next_row, 1024, __ATOMIC_RELAXED);
        if (r0 >= j->n) break;
        uint64_t r1 = r0 + 1024 < j->n ? r0 + 1024 : j->n;
        for (uint64_t r = r0; r < r1; ++r) {
            uint32_t *row = j->raw + j->rowstart[r];
            uint64_t len = j->rowstart[r + 1] - j->rowstart[r];
            if (j->phase == 2) {
                qsort(row, len, sizeof(uint32_t), or_cmp_u32);
                uint64_t k = 0;
                for (uint64_t i = 0; i < len; ++i)
                    if (i == 0 || row[i] != row[i - 1]) row[k++] = row[i];
                j->ucnt[r] = k;
            } else {
                uint64_t o = j->off[r];
                for (uint64_t i = 0; i < j->ucnt[r]; ++i) {
                    j->adj[o + i] = row[i];
                    if (j->wt) j->wt[o + i] = or_pair_weight(j->gseed, (uint32_t)r, row[i]);
                }
            }
        }
    }
}

/* Returns 0 on success, -1 if cap is too small (m_out then holds m), -2 on */
/* bad parameters or allocation failure.  off has n+1 entries, adj and wt   */
/* have room for cap entries; wt may be NULL for an unweighted graph.       */
int or_rmat_csr(uint32_t scale, uint32_t edge_factor, double a, double b, double c,
                uint64_t gseed, uint64_t *off, uint32_t *adj, uint16_t *wt,
                uint64_t cap, uint64_t *m_out, int nthreads)
{
    if (scale < 1 || scale > 31 || edge_factor < 1) return -2;
    or_csr_job j;
    memset(&j, 0, sizeof j);
    j.scale = scale; j.gseed = gseed; j.n = 1u << scale;
    j.M = (uint64_t)edge_factor << scale;
    or_rmat_thresholds(a, b, c, j.T);
    uint64_t n = j.n;
    j.cnt = (uint64_t *)calloc(n, sizeof(uint64_t));
    j.cursor = (uint64_t *)malloc(n * sizeof(uint64_t));
    j.rowstart = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
    j.ucnt = (uint64_t *)malloc(n * sizeof(uint64_t));
    if (!j.cnt || !j.cursor || !j.rowstart || !j.ucnt) goto fail;
    j.phase = 0;
    or_parallel(or_csr_task, &j, nthreads);
    j.rowstart[0] = 0;
    for (uint64_t r = 0; r < n; ++r) j.rowstart[r + 1] = j.rowstart[r] + j.cnt[r];
    memcpy(j.cursor, j.rowstart, n * sizeof(uint64_t));
    j.raw = (uint32_t *)malloc((j.rowstart[n] ? j.rowstart[n] : 1) * sizeof(uint32_t));
    if (!j.raw) goto fail;
    j.phase = 1;
    or_parallel(or_csr_task, &j, nthreads);
    j.phase = 2; j.next_row = 0;
    or_parallel(or_csr_task, &j, nthreads);
    off[0] = 0;
    for (uint64_t r = 0; r < n; ++r) off[r + 1] = off[r] + j.ucnt[r];
    *m_out = off[n];
    if (off[n] > cap) { free(j.raw); j.raw = NULL; goto toosmall; }
    j.off = off; j.adj = adj; j.wt = wt;
    j.phase = 3; j.next_row = 0;
    or_parallel(or_csr_task, &j, nthreads);
    free(j.raw); free(j.cnt); free(j.cursor); free(j.rowstart); free(j.ucnt);
    return 0;
toosmall:
    free(j.cnt); free(j.cursor); free(j.rowstart); free(j.ucnt);
    return -1;
fail:
    free(j.raw); free(j.cnt); free(j.cursor); free(j.rowstart); free(j.ucnt);
    return -2;
}

/* ---------------------------------------------------------------------- */
/* Graph view and the node2vec transition rule.                           */
/* ---------------------------------------------------------------------- */
typedef struct {
    const uint64_t *off;   /* n+1 */
    const uint32_t *adj;   /* m, each row strictly ascending */
    const uint16_t *wt;    /* m or NULL (all weights 1) */
    uint32_t n;
    uint16_t *wmax;        /* n, derived: largest weight in the row (0 if empty) */
    uint16_t wlo, whi;     /* derived: smallest and largest weight of the graph (1, 1 unweighted) */
} or_graph;

or_graph *or_graph_new(const uint64_t *off, const uint32_t *adj, const uint16_t *wt, uint32_t n)
{
    or_graph *g = (or_graph *)calloc(1, sizeof(or_graph));
    if (!g) return NULL;
    g->off = off; g->adj = adj; g->wt = wt; g->n = n;
    g->wmax = (uint16_t *)malloc((n ? n : 1) * sizeof(uint16_t));
    if (!g->wmax) { free(g); return NULL; }
    for (uint32_t v = 0; v < n; ++v) {
        uint16_t m = 0;
        for (uint64_t e = off[v]; e < off[v + 1]; ++e) {
            uint16_t w = wt ? wt[e] : 1;
            if (w > m) m = w;
        }
        g->wmax[v] = m;
    }
    g->wlo = 1;
    g->whi = 1;
    if (wt && off[n] > 0) {
        g->wlo = wt[0];
        g->whi = wt[0];
        for (uint64_t e = 1; e < off[n]; ++e) {
            if (wt[e] < g->wlo) g->wlo = wt[e];
            if (wt[e] > g->whi) g->whi = wt[e];
        }
    }
    return g;
}

void or_graph_free(or_graph *g)
{
    if (!g) return;
    free(g->wmax);
    free(g);
}

/* Multipliers A_ret, A_com, A_out = 4/p, 4, 4/q.  Returns 0, or -1 when   */
/* p or q is outside {1/4, 1/2, 1, 2, 4}.                                   */
int or_multipliers(double p, double q, uint32_t A[3])
{
    static const double allowed[5] = {0.25, 0.5, 1.0, 2.0, 4.0};
    int okp = 0, okq = 0;
    for (int i = 0; i < 5; ++i) { okp |= (p == allowed[i]); okq |= (q == allowed[i]); }
    if (!okp || !okq) return -1;
    A[0] = (uint32_t)lround(4.0 / p);
    A[1] = 4;
    A[2] = (uint32_t)lround(4.0 / q);
    return 0;
}

/* x in N(t)?  Plain binary search over the sorted row of t. */
static int or_has_edge(const or_graph *g, uint32_t t, uint32_t x)
{
    uint64_t lo = g->off[t], hi = g->off[t + 1];
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (g->adj[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo < g->off[t + 1] && g->adj[lo] == x;
}

/* Unnormalised probability of the j-th neighbour of v (Section 2.1):      */
/* w at the first move; w * A(t, x) afterwards.                             */
static uint64_t or_pi(const or_graph *g, uint32_t s, uint32_t t, uint32_t v,
                      uint64_t j, const uint32_t A[3])
{
    uint64_t e = g->off[v] + j;
    uint64_t w = g->wt ? g->wt[e] : 1u;
    if (s == 0) return w;
    uint32_t x = g->adj[e];
    if (x == t) return w * A[0];
    if (or_has_edge(g, t, x)) return w * A[1];
    return w * A[2];
}

static uint32_t or_inverse_cdf(const or_graph *g, uint64_t seed, uint32_t wid, uint32_t s,
                               uint32_t k, uint32_t t, uint32_t v, const uint32_t A[3])
{
    uint64_t d = g->off[v + 1] - g->off[v];
    uint32_t r[4];
    ph(seed, wid, s, k, 0, r);
    uint64_t R1 = ((uint64_t)r[0] << 32) | r[1];
    uint64_t S = 0;
    for (uint64_t j = 0; j < d; ++j) S += or_pi(g, s, t, v, j, A);
    uint64_t target = hi64(R1, S);
    uint64_t P = 0;
    for (uint64_t j = 0; j < d; ++j) {
        P += or_pi(g, s, t, v, j, A);
        if (P > target) return g->adj[g->off[v] + j];
    }
    return OR_SENT; /* not reached: P_{d-1} = S > target */
}

/* ---------------------------------------------------------------------- */
/* FN-Approx (Section 3.4, Eqs. 2 and 3).  At a popular vertex v reached   */
/* from an unpopular vertex u, every neighbour x != u of v has a transition */
/* probability between a lower and an upper bound that depend only on      */
/* d_u, d_v, the multipliers and the range of edge weights; when the two    */
/* bounds differ by less than a threshold, the move is drawn from the       */
/* static edge weights alone (first order).  Readings:                      */
/*   - popular means degree > d_rule (the inverse-CDF class), unpopular     */
/*     degree <= d_rule;                                                    */
/*   - Weight_min and Weight_max are the graph's smallest and largest edge  */
/*     weights (1 and 1 when unweighted);                                   */
/*   - the numerator of a neighbour x != u lies between Weight_min times    */
/*     the smaller and Weight_max times the larger of A_com, A_out;         */
/*   - the denominator is A_ret w_vu + sum over the other d_v - 1           */
/*     neighbours of A_com w (c common neighbours of u and v) or A_out w   */
/*     (the rest); c ranges over 0 .. min(d_u - 1, d_v - 1), since u's      */
/*     neighbour v is not a neighbour of v itself (Eq. 3 writes d_u; its    */
/*     extreme case has d_u - 1 common neighbours); the smallest and the   */
/*     largest denominator take Weight_min and Weight_max for every weight  */
/*     and the c that minimises or maximises the multiplier sum;           */
/*   - LB = smallest numerator / largest denominator, UB = largest          */
/*     numerator / smallest denominator (Eqs. 2 and 3 when                  */
/*     1/p <= 1 <= 1/q); the threshold is 1/T for an integer T (the paper's */
/*     1e-3 is T = 1000) and UB - LB < 1/T is decided exactly by            */
/*     cross-multiplying in 128-bit integers;                               */
/*   - the first-order draw is the first-move rule at v with the move's     */
/*     own counter: inverse CDF over the weights, attempt index 0.          */
/* ---------------------------------------------------------------------- */
void or_approx_bounds(uint64_t du, uint64_t dv, const uint32_t A[3], uint32_t wlo, uint32_t whi,
                      uint64_t *lb_num, uint64_t *lb_den, uint64_t *ub_num, uint64_t *ub_den)
{
    uint64_t a_lo = A[1] < A[2] ? A[1] : A[2];
    uint64_t a_hi = A[1] > A[2] ? A[1] : A[2];
    uint64_t cmax = du - 1 < dv - 1 ? du - 1 : dv - 1;
    /* multiplier sum with c common neighbours: A_ret + c A_com + (d_v-1-c) A_out */
    uint64_t with_none = A[0] + (dv - 1) * A[2];
    uint64_t with_all = A[0] + cmax * A[1] + (dv - 1 - cmax) * A[2];
    uint64_t sum_lo = with_none < with_all ? with_none : with_all;
    uint64_t sum_hi = with_none > with_all ? with_none : with_all;
    *lb_num = wlo * a_lo;
    *lb_den = whi * sum_hi;
    *ub_num = whi * a_hi;
    *ub_den = wlo * sum_lo;
}

/* UB - LB < 1/T for degrees du, dv >= 1 (exact). */
int or_approx_gap_below(uint64_t du, uint64_t dv, const uint32_t A[3], uint32_t wlo, uint32_t whi, uint32_t T)
{
    uint64_t ln, ld, un, ud;
    or_approx_bounds(du, dv, A, wlo, whi, &ln, &ld, &un, &ud);
    /* un/ud - ln/ld < 1/T  <=>  T (un ld - ln ud) < ud ld */
    or_u128 diff = (or_u128)un * ld - (or_u128)ln * ud;
    return (or_u128)T * diff < (or_u128)ud * ld;
}

/* Whether FN-Approx draws the move at v (previous vertex t, s > 0) from   */
/* the static weights, for the threshold 1/T (T = 0: never).               */
int or_approx_applies(const or_graph *g, uint32_t t, uint32_t v, const uint32_t A[3],
                      uint32_t d_rule, uint32_t T)
{
    if (T == 0) return 0;
    uint64_t dv = g->off[v + 1] - g->off[v], du = g->off[t + 1] - g->off[t];
    if (dv <= d_rule || du > d_rule || du == 0) return 0;
    return or_approx_gap_below(du, dv, A, g->wlo, g->whi, T);
}

/* First-order draw at v with counter (walk, s, 0): the first move's rule   */
/* for a vertex of the inverse-CDF class.                                   */
static uint32_t or_static_draw(const or_graph *g, uint64_t seed, uint32_t wid, uint32_t s, uint32_t v)
{
    uint64_t ov = g->off[v], d = g->off[v + 1] - ov;
    uint32_t r[4];
    ph(seed, wid, s, 0, 0, r);
    uint64_t R1 = ((uint64_t)r[0] << 32) | r[1];
    uint64_t S = 0;
    for (uint64_t j = 0; j < d; ++j) S += g->wt ? g->wt[ov + j] : 1u;
    uint64_t target = hi64(R1, S), P = 0;
    for (uint64_t j = 0; j < d; ++j) {
        P += g->wt ? g->wt[ov + j] : 1u;
        if (P > target) return g->adj[ov + j];
    }
    return OR_SENT; /* not reached */
}

/* One move of walk `wid` at step s from v (previous vertex t, ignored at  */
/* s = 0).  Returns the next vertex, or OR_SENT when v has no neighbours.  */
/* approx_t > 0 applies FN-Approx with threshold 1/approx_t.               */
uint32_t or_step(const or_graph *g, uint64_t seed, uint32_t wid, uint32_t s,
                 uint32_t t, uint32_t v, const uint32_t A[3], uint32_t d_rule, uint32_t a_cap,
                 uint32_t approx_t)
{
    uint64_t d = g->off[v + 1] - g->off[v];
    if (d == 0) return OR_SENT;
    if (s > 0 && or_approx_applies(g, t, v, A, d_rule, approx_t)) return or_static_draw(g, seed, wid, s, v);
    uint32_t k = 0;
    if (d <= d_rule) {
        uint32_t amax = A[0] > A[1] ? A[0] : A[1];
        if (A[2] > amax) amax = A[2];
        uint64_t E = (uint64_t)g->wmax[v] * (s == 0 ? 1u : amax);
        for (k = 0; k < a_cap; ++k) {
            uint32_t r[4];
            ph(seed, wid, s, k, 0, r);
            uint64_t R1 = ((uint64_t)r[0] << 32) | r[1];
            uint64_t R2 = ((uint64_t)r[2] << 32) | r[3];
            uint64_t j = hi64(R1, d);
            uint64_t u = hi64(R2, E);
            if (u < or_pi(g, s, t, v, j, A)) return g->adj[g->off[v] + j];
        }
    }
    return or_inverse_cdf(g, seed, wid, s, k, t, v, A);
}

/* ---------------------------------------------------------------------- */
/* Walks, visit counts and checksum.                                       */
/* ---------------------------------------------------------------------- */
/* Checksum term of entry (walk, column, vertex): r0*2^32 + r1 of           */
/* Philox(key=seed; ctr=(walk mod 2^32, column, vertex, 3)).               */
uint64_t or_entry_hash(uint64_t seed, uint32_t wid, uint32_t col, uint32_t x)
{
    uint32_t r[4];
    ph(seed, wid, col, x, 3, r);
    return ((uint64_t)r[0] << 32) | r[1];
}

typedef struct {
    const or_graph *g;
    const uint32_t *starts;
    const uint64_t *wids;   /* NULL: walk i has id walk_base + i */
    uint64_t walk_base, count;
    uint32_t L;
    uint32_t A[3];
    uint64_t seed;
    uint32_t d_rule, a_cap, approx_t;
    uint32_t *out;          /* count x (L+1) or NULL */
    uint32_t *cnt;          /* n or NULL */
    uint64_t checksum;      /* accumulated under a lock-free add */
    uint64_t transitions;
    uint64_t next;          /* dynamic scheduling cursor */
} or_walk_job;

static void or_walk_task(void *p, int tid, int nth)
{
    (void)tid; (void)nth;
    or_walk_job *j = (or_walk_job *)p;
    uint64_t local_sum = 0, local_steps = 0;
    uint32_t L = j->L;
    for (;;) {
        uint64_t i0 = __atomic_fetch_add(&j->next, 256, __ATOMIC_RELAXED);
        if (i0 >= j->count) break;
        uint64_t i1 = i0 + 256 < j->count ? i0 + 256 : j->count;
        for (uint64_t i = i0; i < i1; ++i) {
            uint64_t wg = j->wids ? j->wids[i] : j->walk_base + i;
            uint32_t wid = (uint32_t)wg;
            uint32_t v = j->starts[i], t = OR_SENT;
            uint32_t *row = j->out ? j->out + i * (uint64_t)(L + 1) : NULL;
            if (row) row[0] = v;
            if (j->cnt) __atomic_fetch_add(&j->cnt[v], 1u, __ATOMIC_RELAXED);
            local_sum += or_entry_hash(j->seed, wid, 0, v);
            uint32_t s = 0;
            for (; s < L; ++s) {
                uint32_t x = or_step(j->g, j->seed, wid, s, t, v, j->A, j->d_rule, j->a_cap, j->approx_t);
                if (x == OR_SENT) break;
                if (row) row[s + 1] = x;
                if (j->cnt) __atomic_fetch_add(&j->cnt[x], 1u, __ATOMIC_RELAXED);
                local_sum += or_entry_hash(j->seed, wid, s + 1, x);
                ++local_steps;
                t = v;
                v = x;
            }
            if (row) for (uint32_t c = s + 1; c <= L; ++c) row[c] = OR_SENT;
        }
    }
    __atomic_fetch_add(&j->checksum, local_sum, __ATOMIC_RELAXED);
    __atomic_fetch_add(&j->transitions, local_steps, __ATOMIC_RELAXED);
}

/* Runs `count` walks of L moves.  Walk i starts at starts[i] and has id    */
/* wids[i] (or walk_base + i when wids is NULL).  out (count x (L+1), row   */
/* major) and cnt (n, accumulated, caller zeroes it) may each be NULL.      */
/* approx_t > 0 applies FN-Approx with threshold 1/approx_t.               */
/* Returns 0, or -1 on bad p/q or a start id >= n.                          */
int or_walk(const or_graph *g, const uint32_t *starts, const uint64_t *wids, uint64_t walk_base,
            uint64_t count, uint32_t L, double p, double q, uint64_t seed,
            uint32_t d_rule, uint32_t a_cap, uint32_t approx_t, uint32_t *out, uint32_t *cnt,
            uint64_t *checksum, uint64_t *transitions, int nthreads)
{
    or_walk_job j;
    memset(&j, 0, sizeof j);
    if (or_multipliers(p, q, j.A) != 0) return -1;
    for (uint64_t i = 0; i < count; ++i) if (starts[i] >= g->n) return -1;
    j.g = g; j.starts = starts; j.wids = wids; j.walk_base = walk_base; j.count = count;
    j.L = L; j.seed = seed; j.d_rule = d_rule; j.a_cap = a_cap; j.approx_t = approx_t; j.out = out; j.cnt = cnt;
    or_parallel(or_walk_task, &j, nthreads);
    if (checksum) *checksum = j.checksum;
    if (transitions) *transitions = j.transitions;
    return 0;
}

/* Histogram of single moves at a fixed (t, v, s): for walk ids wid0 ..     */
/* wid0+draws-1, hist[j] counts how often neighbour j of v was chosen.       */
int or_step_hist(const or_graph *g, uint32_t t, uint32_t v, uint32_t s, uint32_t wid0,
                 uint64_t draws, double p, double q, uint64_t seed, uint32_t d_rule,
                 uint32_t a_cap, uint32_t approx_t, uint64_t *hist)
{
    uint32_t A[3];
    if (or_multipliers(p, q, A) != 0) return -1;
    uint64_t base = g->off[v], d = g->off[v + 1] - base;
    if (d == 0) return -1;
    for (uint64_t i = 0; i < draws; ++i) {
        uint32_t x = or_step(g, seed, wid0 + (uint32_t)i, s, t, v, A, d_rule, a_cap, approx_t);
        uint64_t lo = base, hi = base + d;
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (g->adj[mid] < x) lo = mid + 1; else hi = mid;
        }
        hist[lo - base] += 1;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Algorithmic-bytes model: the distinct 64-byte segments of the CSR       */
/* arrays (off u64, adj u32, wt u16, wmax u16) that the cheapest exact     */
/* evaluation of one move must read, plus 4 bytes of output.  State that   */
/* an evaluation carries from the previous move (the previous vertex's     */
/* row bounds and the position of the previous vertex in the current row) */
/* is not charged again.  Segments are counted within one move only.      */
/* ---------------------------------------------------------------------- */
typedef struct { uint64_t *v; uint64_t n, cap; } or_segset;

static void seg_add(or_segset *s, uint32_t array, uint64_t byte_off)
{
    if (s->n == s->cap) {
        uint64_t nc = s->cap ? s->cap * 2 : 256;
        uint64_t *nv = (uint64_t *)realloc(s->v, nc * sizeof(uint64_t));
        if (!nv) return;
        s->v = nv; s->cap = nc;
    }
    s->v[s->n++] = ((uint64_t)array << 58) | (byte_off >> 6);
}

static void seg_add_range(or_segset *s, uint32_t array, uint64_t b0, uint64_t b1)
{
    if (b1 <= b0) return;
    for (uint64_t x = b0 >> 6; x <= (b1 - 1) >> 6; ++x) seg_add(s, array, x << 6);
}

static int or_cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

static uint64_t seg_count(or_segset *s)
{
    if (s->n == 0) return 0;
    qsort(s->v, s->n, sizeof(uint64_t), or_cmp_u64);
    uint64_t k = 1;
    for (uint64_t i = 1; i < s->n; ++i) k += s->v[i] != s->v[i - 1];
    return k;
}

enum { SEG_OFF = 1, SEG_ADJ = 2, SEG_WT = 3, SEG_WMAX = 4, SEG_WTOT = 5 };

/* Lower-bound search of x in adj[lo, hi), recording probed segments.      */
static uint64_t seg_search(or_segset *s, const uint32_t *adj, uint64_t lo, uint64_t hi, uint32_t x)
{
    uint64_t end = hi;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        seg_add(s, SEG_ADJ, mid * 4);
        if (adj[mid] < x) lo = mid + 1; else hi = mid;
    }
    if (lo < end) seg_add(s, SEG_ADJ, lo * 4);
    return lo;
}

/* Bytes of one move (returns 0 for a walk that has ended). */
uint64_t or_step_cost(const or_graph *g, uint64_t seed, uint32_t wid, uint32_t s,
                      uint32_t t, uint32_t v, const uint32_t A[3], uint32_t d_rule, uint32_t a_cap,
                      uint32_t approx_t, uint32_t *next)
{
    or_segset S = {NULL, 0, 0};
    uint64_t ov = g->off[v], d = g->off[v + 1] - ov;
    seg_add(&S, SEG_OFF, (uint64_t)v * 8);
    seg_add(&S, SEG_OFF, (uint64_t)v * 8 + 8);
    uint32_t x = or_step(g, seed, wid, s, t, v, A, d_rule, a_cap, approx_t);
    *next = x;
    if (d == 0) { free(S.v); return 0; }
    if (s > 0 && or_approx_applies(g, t, v, A, d_rule, approx_t)) {
        /* first-order draw: the chosen entry, and for weights the row total */
        /* and the weights up to it (d_t is carried state)                   */
        uint64_t lo = ov, hi = ov + d;
        while (lo < hi) { uint64_t mid = lo + (hi - lo) / 2; if (g->adj[mid] < x) lo = mid + 1; else hi = mid; }
        seg_add(&S, SEG_ADJ, lo * 4);
        if (g->wt) {
            seg_add(&S, SEG_WTOT, (uint64_t)v * 8);
            seg_add_range(&S, SEG_WT, ov * 2, (lo + 1) * 2);
        }
        uint64_t c = seg_count(&S);
        free(S.v);
        return c * 64 + 4;
    }
    uint32_t amax = A[0] > A[1] ? A[0] : A[1];
    if (A[2] > amax) amax = A[2];
    uint32_t acmin = A[1] < A[2] ? A[1] : A[2], acmax = A[1] > A[2] ? A[1] : A[2];
    int hub = d > d_rule;
    uint64_t ot = 0, dt = 0;
    if (s > 0) { ot = g->off[t]; dt = g->off[t + 1] - ot; }
    /* position of t in N(v) is carried state (d when absent) */
    uint64_t pos_t = d;
    if (s > 0) {
        uint64_t lo = ov, hi = ov + d;
        while (lo < hi) { uint64_t mid = lo + (hi - lo) / 2; if (g->adj[mid] < t) lo = mid + 1; else hi = mid; }
        if (lo < ov + d && g->adj[lo] == t) pos_t = lo - ov;
    }
    uint32_t k_fallback = 0;
    if (!hub) {
        if (g->wt) seg_add(&S, SEG_WMAX, (uint64_t)v * 2);
        uint64_t E = (uint64_t)g->wmax[v] * (s == 0 ? 1u : amax);
        uint32_t k;
        for (k = 0; k < a_cap; ++k) {
            uint32_t r[4];
            ph(seed, wid, s, k, 0, r);
            uint64_t j = hi64(((uint64_t)r[0] << 32) | r[1], d);
            uint64_t u = hi64(((uint64_t)r[2] << 32) | r[3], E);
            uint64_t w = 1;
            if (g->wt) { seg_add(&S, SEG_WT, (ov + j) * 2); w = g->wt[ov + j]; }
            int acc;
            if (s == 0) {
                acc = u < w;
                if (acc) seg_add(&S, SEG_ADJ, (ov + j) * 4);
            } else if (j == pos_t) {
                acc = u < A[0] * w;              /* x is t: known without a read */
            } else if (u < acmin * w) {
                acc = 1;
                seg_add(&S, SEG_ADJ, (ov + j) * 4);
            } else if (u >= acmax * w) {
                acc = 0;
            } else {
                uint32_t xj = g->adj[ov + j];
                seg_add(&S, SEG_ADJ, (ov + j) * 4);
                uint64_t pos = seg_search(&S, g->adj, ot, ot + dt, xj);
                int com = pos < ot + dt && g->adj[pos] == xj;
                acc = u < (uint64_t)(com ? A[1] : A[2]) * w;
            }
            if (acc) break;
        }
        if (k < a_cap) {
            uint64_t c = seg_count(&S);
            free(S.v);
            return c * 64 + 4;
        }
        k_fallback = 1;
    }
    (void)k_fallback;
    /* inverse CDF: the cheaper of a streaming merge and a sparse correction */
    or_segset D = {NULL, 0, 0};
    for (uint64_t i = 0; i < S.n; ++i) seg_add(&D, (uint32_t)(S.v[i] >> 58), (S.v[i] & ((1ull << 58) - 1)) << 6);
    /* dense: all of N(v) (and its weights) and, after the first move, N(t) */
    seg_add_range(&D, SEG_ADJ, ov * 4, (ov + d) * 4);
    if (g->wt) seg_add_range(&D, SEG_WT, ov * 2, (ov + d) * 2);
    if (s > 0) seg_add_range(&D, SEG_ADJ, ot * 4, (ot + dt) * 4);
    uint64_t dense = seg_count(&D);
    free(D.v);
    uint64_t best = dense;
    if (s > 0) {
        /* sparse: every member of N(t) searched in N(v); the weighted case     */
        /* also reads the row total, the weights of the matches and the weights */
        /* of N(v) up to the chosen neighbour                                   */
        or_segset P = {NULL, 0, 0};
        for (uint64_t i = 0; i < S.n; ++i) seg_add(&P, (uint32_t)(S.v[i] >> 58), (S.v[i] & ((1ull << 58) - 1)) << 6);
        seg_add_range(&P, SEG_ADJ, ot * 4, (ot + dt) * 4);
        for (uint64_t i = 0; i < dt; ++i) {
            uint32_t y = g->adj[ot + i];
            uint64_t pos = seg_search(&P, g->adj, ov, ov + d, y);
            if (g->wt && pos < ov + d && g->adj[pos] == y) seg_add(&P, SEG_WT, pos * 2);
        }
        uint64_t lo = ov, hi = ov + d;
        while (lo < hi) { uint64_t mid = lo + (hi - lo) / 2; if (g->adj[mid] < x) lo = mid + 1; else hi = mid; }
        seg_add(&P, SEG_ADJ, lo * 4);
        if (g->wt) {
            seg_add(&P, SEG_WTOT, (uint64_t)v * 8);
            seg_add_range(&P, SEG_WT, ov * 2, (lo + 1) * 2);
        }
        uint64_t sparse = seg_count(&P);
        free(P.v);
        if (sparse < best) best = sparse;
    } else if (!g->wt) {
        /* unweighted first move: S = d and the answer is index hi64(R1, d), */
        /* so only the chosen entry of N(v) is read                           */
        or_segset F = {NULL, 0, 0};
        for (uint64_t i = 0; i < S.n; ++i) seg_add(&F, (uint32_t)(S.v[i] >> 58), (S.v[i] & ((1ull << 58) - 1)) << 6);
        uint64_t lo = ov, hi = ov + d;
        while (lo < hi) { uint64_t mid = lo + (hi - lo) / 2; if (g->adj[mid] < x) lo = mid + 1; else hi = mid; }
        seg_add(&F, SEG_ADJ, lo * 4);
        uint64_t first = seg_count(&F);
        free(F.v);
        if (first < best) best = first;
    }
    free(S.v);
    return best * 64 + 4;
}

typedef struct {
    const or_graph *g;
    const uint32_t *starts;
    const uint64_t *wids;
    uint64_t count;
    uint32_t L;
    uint32_t A[3];
    uint64_t seed;
    uint32_t d_rule, a_cap, approx_t;
    uint64_t bytes, steps, hub_steps, next;
    uint64_t hub2_bytes, hub2_steps;  /* second-order moves (s > 0) at vertices above d_rule */
} or_cost_job;

static void or_cost_task(void *p, int tid, int nth)
{
    (void)tid; (void)nth;
    or_cost_job *j = (or_cost_job *)p;
    uint64_t b = 0, st = 0, hs = 0, hb2 = 0, hs2 = 0;
    for (;;) {
        uint64_t i = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
        if (i >= j->count) break;
        uint32_t wid = (uint32_t)j->wids[i];
        uint32_t v = j->starts[i], t = OR_SENT;
        for (uint32_t s = 0; s < j->L; ++s) {
            uint32_t x;
            uint64_t c = or_step_cost(j->g, j->seed, wid, s, t, v, j->A, j->d_rule, j->a_cap, j->approx_t, &x);
            if (x == OR_SENT) break;
            b += c;
            ++st;
            int hub = (j->g->off[v + 1] - j->g->off[v]) > j->d_rule;
            hs += hub;
            if (hub && s > 0) { hb2 += c; ++hs2; }
            t = v;
            v = x;
        }
    }
    __atomic_fetch_add(&j->bytes, b, __ATOMIC_RELAXED);
    __atomic_fetch_add(&j->steps, st, __ATOMIC_RELAXED);
    __atomic_fetch_add(&j->hub_steps, hs, __ATOMIC_RELAXED);
    __atomic_fetch_add(&j->hub2_bytes, hb2, __ATOMIC_RELAXED);
    __atomic_fetch_add(&j->hub2_steps, hs2, __ATOMIC_RELAXED);
}

/* Sums the algorithmic bytes, the moves taken and the moves made at        */
/* vertices of degree > d_rule over the given walks.                        */
int or_walk_cost(const or_graph *g, const uint32_t *starts, const uint64_t *wids, uint64_t count,
                 uint32_t L, double p, double q, uint64_t seed, uint32_t d_rule, uint32_t a_cap,
                 uint32_t approx_t, uint64_t *bytes, uint64_t *steps, uint64_t *hub_steps, int nthreads)
{
    or_cost_job j;
    memset(&j, 0, sizeof j);
    if (or_multipliers(p, q, j.A) != 0) return -1;
    j.g = g; j.starts = starts; j.wids = wids; j.count = count; j.L = L; j.seed = seed;
    j.d_rule = d_rule; j.a_cap = a_cap; j.approx_t = approx_t;
    or_parallel(or_cost_task, &j, nthreads);
    *bytes = j.bytes; *steps = j.steps; *hub_steps = j.hub_steps;
    return 0;
}

/* As or_walk_cost, split into two classes: cls[0], cls[1] = bytes and      */
/* moves of second-order moves (s > 0) at vertices above d_rule (the        */
/* inverse-CDF class); cls[2], cls[3] = bytes and moves of all other moves. */
int or_walk_cost_classes(const or_graph *g, const uint32_t *starts, const uint64_t *wids, uint64_t count,
                         uint32_t L, double p, double q, uint64_t seed, uint32_t d_rule, uint32_t a_cap,
                         uint32_t approx_t, uint64_t cls[4], int nthreads)
{
    or_cost_job j;
    memset(&j, 0, sizeof j);
    if (or_multipliers(p, q, j.A) != 0) return -1;
    j.g = g; j.starts = starts; j.wids = wids; j.count = count; j.L = L; j.seed = seed;
    j.d_rule = d_rule; j.a_cap = a_cap; j.approx_t = approx_t;
    or_parallel(or_cost_task, &j, nthreads);
    cls[0] = j.hub2_bytes;
    cls[1] = j.hub2_steps;
    cls[2] = j.bytes - j.hub2_bytes;
    cls[3] = j.steps - j.hub2_steps;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Memo-aware algorithmic bytes of a whole pass (the FN-Cache paragraph of */
/* Section 3.4: work done for popular vertices is kept and reused within  */
/* a run).  A second-order move at a vertex v above d_rule needs, besides */
/* v's row bounds and its 4-byte output, either                            */
/*   - the intersection of N(v) with N(t), when no earlier move of the     */
/*     pass computed it ("cold"), or                                       */
/*   - a kept per-pair summary of it ("warm"): 64 segment counts and 64    */
/*     first-half counts of members of N(t) in equal segments of N(v), and */
/*     64 start positions in N(t) (192 two-byte words: 6 lines), plus the  */
/*     half segment of N(v) that holds the drawn prefix sum and the part of */
/*     N(t) whose values fall in it (its share of N(t) in proportion),     */
/* whichever is cheaper for the move (the directed cold cost below against */
/* the warm one).  The intersection behind a summary is charged once per   */
/* pass and pair whose moves read it: the cheaper of a                     */
/* streaming merge of both rows and a search of each member of the shorter */
/* row in the longer (one line per search level below a 16-entry line,    */
/* at least one), on top of reading the shorter row.  A summary serves     */
/* both directions of a pair when both endpoints keep summaries (degree in */
/* [memo_min, 4161536]); otherwise only moves at the endpoint that keeps   */
/* them.  Moves at vertices that keep none (and every move of a weighted   */
/* graph, or of a pass without summaries) pay the directed cold cost each  */
/* time.  The directed cold cost: the cheaper of merging N(v) with N(t) and */
/* searching N(t)'s                                                         */
/* members in N(v), plus the weights of N(v) for a weighted graph.  All    */
/* counts are 64-byte lines of arrays that start on a line.  The pass is   */
/* given by its walk matrix (count x (L+1), N2V sentinel after the end).   */
/* ---------------------------------------------------------------------- */
#define OR_MEMO_MAX_DEG 4161536ull

static uint64_t lines_of(uint64_t elem, uint64_t lo, uint64_t hi)
{
    if (hi <= lo) return 0;
    return ((hi * elem - 1) >> 6) - ((lo * elem) >> 6) + 1;
}

/* Lines holding off[v] and off[v+1]. */
uint64_t or_memo_off_lines(uint32_t v)
{
    return lines_of(8, v, (uint64_t)v + 2);
}

/* Search levels charged per member searched in a row of d entries:        */
/* ceil(log2(d / 16)), at least 1.                                          */
uint64_t or_memo_search_levels(uint64_t d)
{
    uint64_t k = 1;
    while ((16ull << k) < d) ++k;
    return k;
}

/* Lines of one intersection of the rows of a and b (unweighted). */
uint64_t or_memo_pair_lines(const uint64_t *off, uint32_t a, uint32_t b)
{
    uint64_t da = off[a + 1] - off[a], db = off[b + 1] - off[b];
    uint64_t dense = lines_of(4, off[a], off[a + 1]) + lines_of(4, off[b], off[b + 1]);
    uint32_t sh = da <= db ? a : b;
    uint64_t dsh = da <= db ? da : db, dlo = da <= db ? db : da;
    uint64_t search = lines_of(4, off[sh], off[sh + 1]) + dsh * or_memo_search_levels(dlo);
    return search < dense ? search : dense;
}

/* Lines of one move at v after t evaluated without a summary. */
uint64_t or_memo_cold_lines(const uint64_t *off, int weighted, uint32_t t, uint32_t v)
{
    uint64_t dv = off[v + 1] - off[v], dt = off[t + 1] - off[t];
    uint64_t rt = lines_of(4, off[t], off[t + 1]);
    uint64_t w = weighted ? lines_of(2, off[v], off[v + 1]) : 0;
    uint64_t dense = lines_of(4, off[v], off[v + 1]) + rt + w;
    uint64_t search = rt + dt * or_memo_search_levels(dv) + w;
    return search < dense ? search : dense;
}

/* Bytes of one summary row of a vertex of degree d: per segment a count,   */
/* a start hint and a first-half count (16 bits each) and, on a weighted    */
/* graph, four 32-bit weight sums, over the row's segments (whole 512-entry */
/* tiles, at most 64 segments) rounded up to an even number.                */
uint64_t or_memo_row_bytes(uint64_t d, int weighted)
{
    uint64_t tiles = (d + 511) / 512;
    uint64_t per = tiles ? (tiles + 63) / 64 : 1;
    uint64_t segs = (tiles + per - 1) / per;
    segs = (segs + 1) & ~1ull;
    return (weighted ? 22 : 6) * segs;
}

/* Lines of one move at v after t that reads a summary: the summary row,    */
/* the half segment holding the draw (and its weights on a weighted graph) */
/* and N(t)'s proportional share of it.                                     */
uint64_t or_memo_warm_lines(const uint64_t *off, int weighted, uint32_t t, uint32_t v)
{
    uint64_t dv = off[v + 1] - off[v], dt = off[t + 1] - off[t];
    uint64_t tiles = (dv + 511) / 512;
    uint64_t seglen = ((tiles + 63) / 64) * 512;
    uint64_t h = seglen / 2 < dv ? seglen / 2 : dv;
    uint64_t ht = (dt * h + dv - 1) / dv;
    uint64_t row = (or_memo_row_bytes(dv, weighted) + 63) / 64;
    if (weighted) return row + (4 * h + 63) / 64 + (2 * h + 63) / 64 + (4 * ht + 63) / 64;
    return row + (4 * h + 63) / 64 + (4 * ht + 63) / 64;
}

static int or_memo_keeps(uint64_t d, uint32_t memo_min)
{
    return d >= memo_min && d <= OR_MEMO_MAX_DEG;
}

/* Totals over a pass: res[0] = bytes of second-order moves at vertices     */
/* above d_rule (cold and warm, intersections included), res[1] = those     */
/* moves, res[2] = all other moves (first moves and moves at vertices of    */
/* degree <= d_rule), res[3] = intersections charged, res[4] = warm moves.  */
/* memo = 0: no summaries.  A weighted graph's summary of (t -> v) also     */
/* holds weight sums of N(v), so it serves that direction only and costs   */
/* the directed cold evaluation (weights of N(v) included) to build.       */
/* Returns -1 on allocation failure.                                        */
int or_memo_pass_bytes(const uint64_t *off, int weighted, const uint32_t *out, uint64_t count, uint32_t L,
                       uint32_t d_rule, uint32_t memo_min, int memo, uint64_t res[5])
{
    uint64_t cap = 1024, nk = 0;
    uint64_t *keys = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!keys) return -1;
    memset(res, 0, 5 * sizeof(uint64_t));
    int summaries = memo;
    for (uint64_t i = 0; i < count; ++i) {
        const uint32_t *row = out + i * (uint64_t)(L + 1);
        for (uint32_t s = 0; s < L; ++s) {
            if (row[s] == OR_SENT || row[s + 1] == OR_SENT) break;
            uint32_t v = row[s];
            uint64_t dv = off[v + 1] - off[v];
            if (s == 0 || dv <= d_rule) { res[2] += 1; continue; }
            uint32_t t = row[s - 1];
            res[1] += 1;
            uint64_t lines = or_memo_off_lines(v);
            uint64_t cold = or_memo_cold_lines(off, weighted, t, v);
            uint64_t warm = summaries && or_memo_keeps(dv, memo_min) ? or_memo_warm_lines(off, weighted, t, v) : cold;
            if (warm < cold) {
                lines += warm;
                res[4] += 1;
                uint64_t dt = off[t + 1] - off[t];
                uint64_t key;
                if (!weighted && or_memo_keeps(dt, memo_min))
                    key = t < v ? ((uint64_t)t << 32) | v : ((uint64_t)v << 32) | t;
                else
                    key = ((uint64_t)v << 32) | t;
                if (nk == cap) {
                    uint64_t *nkeys = (uint64_t *)realloc(keys, 2 * cap * sizeof(uint64_t));
                    if (!nkeys) { free(keys); return -1; }
                    keys = nkeys;
                    cap *= 2;
                }
                keys[nk++] = key;
            } else {
                lines += cold;
            }
            res[0] += lines * 64 + 4;
        }
    }
    if (nk) {
        qsort(keys, nk, sizeof(uint64_t), or_cmp_u64);
        for (uint64_t k = 0; k < nk; ++k) {
            if (k > 0 && keys[k] == keys[k - 1]) continue;
            uint32_t a = (uint32_t)(keys[k] >> 32), b = (uint32_t)keys[k];
            /* weighted keys are (v, t) */
            res[0] += (weighted ? or_memo_cold_lines(off, 1, b, a) : or_memo_pair_lines(off, a, b)) * 64;
            res[3] += 1;
        }
    }
    free(keys);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Skip-gram negatives (the stage that consumes the walks, Sections 1 and */
/* 2.1): negative k of walk w at training step `step` is the vertex x with */
/* cum[x] <= r < cum[x+1], r = hi64(R1, cum[n]), R1 = r0*2^32 + r1 of      */
/* Philox(key = seed; ctr = (w mod 2^32, k, step, 6)).  cum is the         */
/* cumulative noise weight table (cum[0] = 0, cum[n] > 0).                 */
/* ---------------------------------------------------------------------- */
void or_sgns_negatives(const uint64_t *cum, uint32_t n, uint64_t seed, uint64_t walk_base, uint32_t step,
                       uint32_t n_walks, uint32_t nneg, uint32_t *out)
{
    for (uint64_t i = 0; i < n_walks; ++i) {
        for (uint32_t k = 0; k < nneg; ++k) {
            uint32_t r[4];
            ph(seed, (uint32_t)(walk_base + i), k, step, 6, r);
            uint64_t target = hi64(((uint64_t)r[0] << 32) | r[1], cum[n]);
            uint32_t x = 0;
            while (!(cum[x] <= target && target < cum[x + 1])) ++x; /* linear scan: plain */
            out[i * nneg + k] = x;
        }
    }
}
