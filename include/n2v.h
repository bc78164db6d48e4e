/*
 * n2v.h -- C ABI of the MI355X node2vec walk engine.
 *
 * The engine generates node2vec biased second-order random walks whose
 * transition probabilities are computed on the fly at every move (Zhou, Niu,
 * Chen, "Efficient Graph Computation for Node2Vec": model of Section 2.1,
 * on-demand probabilities of Section 3.2 and Algorithm 1, multi-round walks
 * of the FN-Multi paragraph of Section 3.4, R-MAT graphs of Section 4.1).
 *
 * Conventions
 *   - Every call returns an int status: N2V_OK (0), N2V_PENDING (1) or a
 *     negative error code.  n2v_last_error() returns a message for the last
 *     failing call on the calling thread.  Nothing throws across the ABI.
 *   - Device buffers are owned by the caller and passed as plain device
 *     pointers.  The engine never allocates device memory on its own: extra
 *     memory it needs comes from caller-provided workspaces whose sizes are
 *     returned by the *_workspace queries.  Workspaces must be 256-byte
 *     aligned.
 *   - Streams are HIP streams (hipStream_t) passed as void*; NULL is the
 *     legacy default stream.  Unless stated otherwise a call only enqueues
 *     work on the stream and returns.
 *   - Vertex ids are uint32; 0xFFFFFFFF (N2V_SENT) is reserved.  Row offsets
 *     are uint64.  Edge weights are uint16 in [1, 65535].
 *
 * The draw rule (one correct output for every input)
 *   - K = 4; multipliers A_ret = 4/p (x is the previous vertex t), A_com = 4
 *     (x is a neighbour of t), A_out = 4/q (otherwise); p, q must be one of
 *     0.25, 0.5, 1, 2, 4, so each multiplier is an integer in {1,2,4,8,16}
 *     and the integer law equals node2vec's law exactly.
 *   - pi_j = w_j at the first move, w_j * A(t, x_j) afterwards.
 *   - Randomness: Philox4x32-10 with key (seed mod 2^32, seed >> 32) and
 *     counter (walk mod 2^32, move, attempt, 0); R1 = r0*2^32 + r1,
 *     R2 = r2*2^32 + r3; hi64(x, y) = floor(x*y / 2^64).
 *   - d <= d_rule: rejection with envelope E = wmax(v) (first move) or
 *     A_max*wmax(v); attempt k takes j = hi64(R1, d), u = hi64(R2, E) and
 *     accepts neighbour j iff u < pi_j; after a_cap attempts the inverse CDF
 *     runs with attempt index a_cap.
 *   - d > d_rule: inverse CDF with attempt index 0: S = sum pi_j,
 *     r = hi64(R1, S), result = first j in row order whose prefix sum
 *     exceeds r.
 *   - a vertex without neighbours ends the walk; the rest of its output row
 *     is N2V_SENT.
 */
#ifndef N2V_H
#define N2V_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define N2V_SENT 0xFFFFFFFFu
#define N2V_ABI_VERSION 7

enum {
    N2V_OK = 0,
    N2V_PENDING = 1,
    N2V_EINVAL = -1,    /* bad argument */
    N2V_ENOMEM = -2,    /* workspace or pool too small */
    N2V_EGRAPH = -3,    /* CSR violates the graph contract */
    N2V_EDEVICE = -4,   /* HIP runtime error */
    N2V_EAGAIN = -5,    /* queue full; retry later */
    N2V_ETOOBIG = -6,   /* request can never fit the server's pool */
    N2V_ENOTFOUND = -7  /* unknown ticket */
};

typedef struct n2v_graph n2v_graph;
typedef struct n2v_server n2v_server;

/* Message of the last failing call on this thread (never NULL). */
const char *n2v_last_error(void);
/* N2V_ABI_VERSION of the loaded library. */
int n2v_abi_version(void);

/* ------------------------------------------------------------------------
 * R-MAT generator (Section 4.1: each edge picks one of the four quadrants of
 * the adjacency matrix with probabilities a, b, c, d = 1-a-b-c, recursively,
 * top level first).
 *
 * Edge e < edge_factor * 2^scale takes `scale` quadrant choices; level l uses
 * word (l mod 4) of Philox(key = seed; ctr = (e mod 2^32, e >> 32, l/4, 1))
 * compared with T1 = round(a*2^32), T2 = round((a+b)*2^32),
 * T3 = round((a+b+c)*2^32); quadrant q = [w>=T1]+[w>=T2]+[w>=T3] sets bit
 * scale-1-l of the source to q>>1 and of the target to q&1.  Self-loops are
 * dropped, both directions are kept, duplicates are removed, rows are sorted.
 * Weighted graphs get w{x,y} = 1 + floor(r0*1000/2^32) with r0 = word 0 of
 * Philox(key = seed; ctr = (min(x,y), max(x,y), 0, 2)).
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t scale;        /* n = 2^scale vertices, 1 <= scale <= 31 */
    uint32_t edge_factor;  /* edges generated = edge_factor * 2^scale */
    double a, b, c;        /* quadrant probabilities, a+b+c <= 1 */
    uint64_t seed;
    int weighted;          /* nonzero: fill weights */
} n2v_rmat_params;

/* Workspace bytes and an upper bound m_max on the directed entries (the
 * capacity `adj` and `wt` must have). */
int n2v_rmat_workspace(const n2v_rmat_params *prm, size_t *ws_bytes, uint64_t *m_max);

/* Generates the CSR into caller buffers: off (device, n+1 entries), adj
 * (device, m_max entries), wt (device, m_max entries; NULL unless weighted).
 * Writes the entry count to *m_out (host).  Synchronises the stream once to
 * read the count.  Errors: N2V_EINVAL (bad parameters), N2V_ENOMEM (workspace
 * smaller than the query), N2V_EDEVICE. */
int n2v_rmat_generate(const n2v_rmat_params *prm, void *ws, size_t ws_bytes, uint64_t *off,
                      uint32_t *adj, uint16_t *wt, uint64_t *m_out, void *stream);

/* ------------------------------------------------------------------------
 * Graph: borrows a CSR (off, adj, optional wt; all device) until destroyed
 * and derives per-vertex records, reverse-edge positions and (weighted)
 * per-vertex weight sums and maxima into the caller's workspace.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t d_rule;   /* rule threshold: rejection iff degree <= d_rule (default 1024) */
    uint32_t a_cap;    /* rejection attempts before the inverse-CDF fallback (default 1024, >= 1) */
    int validate;      /* 0: trust the CSR; 1: check it (default); 2: also check symmetry */
} n2v_graph_opts;

/* Fills the defaults above. */
void n2v_graph_opts_default(n2v_graph_opts *o);

/* Workspace bytes for a graph with n vertices and m entries. */
int n2v_graph_workspace(uint32_t n, uint64_t m, int weighted, size_t *ws_bytes);

/* Contract: off[0] = 0, off[n] = m, off non-decreasing; each row strictly
 * ascending; no self-loops; ids < n; n <= 2^32 - 2; weights >= 1.  With
 * validate >= 1 a violation returns N2V_EGRAPH (this synchronises the
 * stream).  On success *out is a handle valid until n2v_graph_destroy. */
int n2v_graph_create(const uint64_t *off, const uint32_t *adj, const uint16_t *wt, uint32_t n,
                     uint64_t m, const n2v_graph_opts *opts, void *ws, size_t ws_bytes,
                     void *stream, n2v_graph **out);

/* Frees the handle (the caller's arrays and workspace stay the caller's),
 * after waiting for replays of its recorded plain-form graphs still in
 * flight.  N2V_EINVAL while a server created on the graph has not been
 * destroyed. */
int n2v_graph_destroy(n2v_graph *g);

/* Number of vertices / entries and the rule parameters of a graph. */
int n2v_graph_info(const n2v_graph *g, uint32_t *n, uint64_t *m, uint32_t *d_rule,
                   uint32_t *a_cap, int *weighted);

/* ------------------------------------------------------------------------
 * Walks.  Walk i starts at starts[i] and uses walk id walk_base + i in the
 * random counter (walk_base + n_starts <= 2^32).  L >= 1 moves.
 * ---------------------------------------------------------------------- */
enum { N2V_MODE_AUTO = 0, N2V_MODE_PLAIN = 1, N2V_MODE_PERSISTENT = 2 };
enum { N2V_OUT_WALKS = 1, N2V_OUT_COUNTS = 2 };

typedef struct {
    int mode;            /* N2V_MODE_*; AUTO = PERSISTENT */
    uint32_t t_wave;     /* persistent: rejection moves at degree > t_wave run wave-cooperatively */
    uint32_t t_sparse;   /* hub moves use the sparse intersection when deg(t) <= t_sparse (default
                            1023, the most the sparse path holds) ... */
    uint32_t sparse_ratio; /* ... and deg(t) * sparse_ratio * log2(deg v) < deg(v) + deg(t) */
    uint32_t waves_per_cu; /* persistent grid size (0: occupancy-derived) */
    uint32_t block;      /* workgroup size (256) */
    uint32_t memo;       /* 1: use the graph's pair sketches when attached (default 1) */
    uint32_t t_wg;       /* plain: dense hub moves at degree > max(t_wg, d_rule) are evaluated by
                            a whole workgroup (its wavefronts split the merge), the others by one
                            wavefront each (default 65536) */
    uint32_t search_ratio; /* dense hub moves look N(v)'s entries up in N(t) (pivots in LDS, then
                            a search in one bucket) instead of streaming N(t) when the part of
                            N(t) to stream is more than search_ratio times longer (default 24;
                            0: always look up) */
} n2v_exec_opts;

/* Fills execution defaults (tuned values when an autotune result was stored
 * in the graph; see n2v_autotune).  Execution options never change outputs. */
void n2v_exec_opts_default(const n2v_graph *g, n2v_exec_opts *o);

/* Walks of L moves; out (device) is n_starts x (L+1) uint32, row-major, with
 * out[i][0] = starts[i].  Uses the persistent kernel and needs no workspace.
 * Start ids >= n produce an all-N2V_SENT tail and set the graph's device
 * error flag (read with n2v_graph_check).  Calls on one graph may overlap:
 * each persistent launch takes one of the graph's 64 walk counters that no
 * launch still in flight holds, and N2V_EAGAIN is returned (nothing
 * enqueued) while all 64 are held. */
int n2v_walk(const n2v_graph *g, const uint32_t *starts, uint32_t n_starts, uint32_t L, float p,
             float q, uint64_t seed, uint32_t *out, void *stream);

/* Workspace bytes n2v_walk_ex needs for these options (0 for persistent). */
int n2v_walk_workspace(const n2v_graph *g, uint32_t n_starts, uint32_t L,
                       const n2v_exec_opts *opts, size_t *ws_bytes);

/* General form.  outputs is a mask of N2V_OUT_*: WALKS writes `out` as in
 * n2v_walk; COUNTS adds, for every entry out[i][c] != N2V_SENT, one to
 * cnt[x] (device, n uint32) and H(walk id, c, x) to *checksum (device u64,
 * modulo 2^64), H = r0*2^32 + r1 of Philox(key = seed; ctr = (walk id mod
 * 2^32, c, x, 3)).  Counts accumulate: zero them before the first chunk.
 * `opts` may be NULL (defaults); `ws` may be NULL when the query says 0.
 * The plain form (N2V_MODE_PLAIN) is one superstep of two kernels per move
 * (Algorithm 1).  A plain call whose every argument (pointers, sizes, options,
 * seed) equals that of one of the graph's last 8 distinct plain calls is
 * recorded into a HIP graph on its second occurrence and replayed from then
 * on: one graph launch instead of 2L+2 kernel launches, same results, and the
 * buffers' contents may change between calls.  Recording allocates the
 * graph's host and device memory; calls enqueued on a stream that is being
 * captured launch their kernels directly. */
int n2v_walk_ex(const n2v_graph *g, const uint32_t *starts, uint32_t n_starts, uint64_t walk_base,
                uint32_t L, float p, float q, uint64_t seed, const n2v_exec_opts *opts,
                int outputs, uint32_t *out, uint32_t *cnt, uint64_t *checksum, void *ws,
                size_t ws_bytes, void *stream);

/* FN-Approx (Section 3.4, Eqs. 2 and 3): as n2v_walk_ex, except that a move
 * at a vertex v of degree > d_rule whose previous vertex t has degree <=
 * d_rule is drawn from the static edge weights (the rule of a first move:
 * inverse CDF over w_vx with attempt index 0 and the move's own counter) when
 * the bounds of Eqs. 2 and 3 on the probability of a neighbour x != t differ
 * by less than 1/approx_t.  The bounds hold for every (p, q): the numerator
 * lies between wlo min(A_com, A_out) and whi max(A_com, A_out), the
 * denominator between wlo and whi times the extremes of A_ret + c A_com +
 * (d_v - 1 - c) A_out over c = 0 .. min(d_t, d_v) - 1 common neighbours,
 * with wlo and whi the graph's smallest and largest edge weights; the
 * comparison is exact (128-bit cross-multiplication).  approx_t = 0 is the
 * exact rule (identical to n2v_walk_ex); the paper's threshold 1e-3 is
 * approx_t = 1000.  Errors as n2v_walk_ex. */
int n2v_walk_approx(const n2v_graph *g, const uint32_t *starts, uint32_t n_starts, uint64_t walk_base,
                    uint32_t L, float p, float q, uint64_t seed, uint32_t approx_t,
                    const n2v_exec_opts *opts, int outputs, uint32_t *out, uint32_t *cnt,
                    uint64_t *checksum, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the plain
 * form of n2v_walk_approx (approx_t = 0: n2v_walk_ex) with the mode forced to
 * N2V_MODE_PLAIN and its workspace replaced by a fixed scratch array that the
 * library holds on each GPU it runs on (about 40 MiB, kept until the process
 * ends).  Results are identical to n2v_walk_ex / n2v_walk_approx.  At most
 * 2^21 walks of at most 1023 moves per call, else N2V_ENOMEM with nothing
 * enqueued.  It calls no allocating routine.  Every call on one GPU shares
 * that GPU's scratch: calls that overlap on one GPU (other streams, other
 * threads) race and give wrong results; calls ordered on one stream do not.
 * The per-superstep counters are cleared by a kernel at the start of each
 * call. */
int n2v_walk_static(const n2v_graph *g, const uint32_t *starts, uint32_t n_starts, uint64_t walk_base,
                    uint32_t L, float p, float q, uint64_t seed, uint32_t approx_t,
                    const n2v_exec_opts *opts, int outputs, uint32_t *out, uint32_t *cnt,
                    uint64_t *checksum, void *stream);

/* Visit profile (the frequency-versus-degree study of Section 3.3): for
 * visit counts cnt (device, n uint32, as written by the COUNTS output),
 * vertices[k] and visits[k] (device, nbuckets uint64 each, overwritten)
 * receive the number of vertices and their summed visits in degree bucket k:
 * bucket 0 holds degree 0, bucket k >= 1 degrees in ((k-1) width, k width],
 * and bucket nbuckets-1 also every larger degree.  width >= 1, 2 <= nbuckets
 * <= 2048, else N2V_EINVAL.  Asynchronous on `stream`. */
int n2v_visit_profile(const n2v_graph *g, const uint32_t *cnt, uint32_t width, uint32_t nbuckets,
                      uint64_t *vertices, uint64_t *visits, void *stream);

/* Pair sketches (the FN-Cache paragraph of Section 3.4 keeps work done for
 * popular vertices for reuse): memory in which walk calls memoise, for every
 * traversed move (t -> v) at a vertex v of degree > d_rule, the exact number
 * of members of N(t) in each of nsup segments of N(v) (whole 512-entry tiles,
 * at most 64 segments of equal tile counts) and in each segment's first half
 * (as count + 1; 0 = unknown), and for each segment a
 * hint where its merge may start in N(t); on weighted graphs also, per
 * segment and per first half, the weight sum of those members (+ 1) and of
 * all entries (u32 words after the u16 ones).  A later move
 * along the same pair then recomputes half a segment instead of the whole
 * intersection.  Rows of degree above 4,161,536 (127 x 512 x 64) keep no
 * sketches.  On unweighted graphs a merge for (t -> v) also fills the sketch
 * of (v -> t) when t has degree > d_rule.  Results never depend on the sketches: unknown
 * entries are recomputed, and every known entry is exact (hints never point
 * past the segment's first candidate).
 * Sketches describe the graph only (not p, q, seed or the walks), so they
 * persist across calls: every call, and every server on the graph, reads
 * and fills the same memory, and overlapping calls only ever write equal
 * values into an entry.  Attaching clears the memory; n2v_graph_memo_clear
 * makes later calls start from unknown entries again (a cold pass).
 * Each row is sized for its vertex: with nsp = nsup rounded up to even, a row
 * of a vertex of degree d is 6 nsp bytes (22 nsp on weighted graphs), so a
 * hub of degree d keeps d such rows (at most 384, or 1408, bytes each).
 * n2v_graph_memo_bytes returns the size over every row of degree > d_rule;
 * n2v_graph_set_memo attaches caller device memory
 * (NULL detaches).  Attaching synchronises the device, and returns N2V_EINVAL,
 * changing nothing, while a server created on the graph is alive. */
int n2v_graph_memo_bytes(const n2v_graph *g, size_t *bytes);
int n2v_graph_set_memo(n2v_graph *g, void *mem, size_t bytes);

/* Enqueues on `stream` the clearing of the attached sketch memory (N2V_OK
 * with nothing to do when none is attached).  Walks still in flight on other
 * streams may fill entries again; their results are unaffected. */
int n2v_graph_memo_clear(n2v_graph *g, void *stream);

/* Sketches for part of the hub rows, when all of them do not fit: only moves
 * at vertices of degree >= min_degree (> d_rule) keep sketches; the other hub
 * moves take the full pass every time.  n2v_graph_memo_plan returns the
 * smallest such threshold whose rows fit in `budget` bytes, and those rows'
 * bytes (*min_degree = 0xFFFFFFFF and *bytes = 0 when none fit).  It
 * allocates nothing (its degree statistics use the
 * graph's workspace) and synchronises the device, so plans on one graph must
 * not run concurrently.
 * n2v_graph_set_memo_min attaches `bytes` of device memory (256-byte aligned)
 * for rows of degree >= min_degree; it re-indexes the rows on the default
 * stream and synchronises, so no walk on this graph may be in flight.
 * N2V_ENOMEM if `bytes` is too small, N2V_EINVAL while a server is alive:
 * both leave the graph as it was.  NULL detaches. */
int n2v_graph_memo_plan(const n2v_graph *g, size_t budget, uint32_t *min_degree, size_t *bytes);
int n2v_graph_set_memo_min(n2v_graph *g, void *mem, size_t bytes, uint32_t min_degree);

/* Synchronises the stream and returns N2V_EINVAL if any walk since the last
 * check had a start id >= n, N2V_EDEVICE if a kernel detected an internal
 * inconsistency (never expected), else N2V_OK.  Clears the flags. */
int n2v_graph_check(const n2v_graph *g, void *stream);

/* ------------------------------------------------------------------------
 * Skip-gram with negative sampling over walks (Section 1 and Section 2.1:
 * node2vec learns vertex embeddings by running Skip-gram over its walks).
 * One step over a batch of walks (rows of row_len entries, N2V_SENT after a
 * walk's end) against embedding tables win and wout (device, n x dim fp32,
 * row-major):
 *   - each position i < len of a walk (len = entries before the first
 *     sentinel, row_len <= 96) is a center v = win[x_i]; its contexts are the
 *     positions j < len with 1 <= |i - j| <= window, u = wout[x_j]; the walk's
 *     `negatives` (<= 64) vertices n_k, drawn from the noise distribution, are
 *     negatives of every center of the walk, u = wout[n_k];
 *   - z = v . u; loss = sum over (center, context) of softplus(-z) + neg_weight
 *     x sum over (center, negative) of softplus(z), accumulated into *loss
 *     (device f64);
 *   - gradients: (sigmoid(z) - 1) u and neg_weight sigmoid(z) u into the
 *     center's row, (sigmoid(z) - 1) v and neg_weight sigmoid(z) v into the
 *     target's, summed over the batch;
 *   - then win -= lr x its gradient and wout -= lr x its gradient (every walk
 *     of the batch sees the tables as they were before the step).
 * Products run in bf16 with fp32 accumulation; gradients accumulate in fp32
 * (atomically, so their summation order varies).
 * Negative k of the walk with id w (= walk_base + index in the batch):
 * r = hi64(R1, cum[n]) with R1 = r0*2^32 + r1 of Philox(key = seed;
 * ctr = (w mod 2^32, k, step, 6)), and the vertex x with cum[x] <= r <
 * cum[x+1]; cum (device, n+1 u64) is the caller's cumulative noise weight
 * table (cum[0] = 0, non-decreasing, cum[n] > 0).
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t dim;        /* embedding dimension: 128 */
    uint32_t window;     /* context positions j with 1 <= |i - j| <= window */
    uint32_t negatives;  /* shared negatives per walk, <= 64 */
    float neg_weight;    /* weight of each (center, negative) term */
    float lr;            /* SGD step size */
    uint64_t seed;       /* negative-sampling key */
    uint32_t step;       /* step index in the negative-sampling counter */
} n2v_sgns_params;

/* Workspace bytes of n2v_sgns_step: two n x dim fp32 gradient tables, which
 * must be zero before the first step (every step leaves them zero), and the
 * batch's negatives. */
int n2v_sgns_workspace(uint32_t n, uint32_t dim, uint32_t n_walks, uint32_t negatives, size_t *ws_bytes);

/* The negatives of walks walk_base .. walk_base + n_walks - 1 into out
 * (device, n_walks x negatives u32), as n2v_sgns_step draws them. */
int n2v_sgns_negatives(const uint64_t *cum, uint32_t n, uint64_t seed, uint64_t walk_base, uint32_t step,
                       uint32_t n_walks, uint32_t negatives, uint32_t *out, void *stream);

/* One training step (above).  Errors: N2V_EINVAL (dim != 128, row_len not in
 * 1..96, negatives > 64, misaligned workspace or tables), N2V_ENOMEM
 * (workspace smaller than the query).  Asynchronous on `stream`. */
int n2v_sgns_step(const n2v_sgns_params *prm, const uint32_t *walks, uint32_t n_walks, uint32_t row_len,
                  uint64_t walk_base, const uint64_t *cum, uint32_t n, float *win, float *wout, void *ws,
                  size_t ws_bytes, double *loss, void *stream);

/* ------------------------------------------------------------------------
 * Autotuner: times the persistent kernel on a seeded sample of walks from
 * the graph under a set of candidate execution options and stores the best
 * in the graph (n2v_exec_opts_default then returns it).  Outputs are
 * unchanged by construction.  Needs a workspace of at least
 * n2v_autotune_workspace bytes.  Synchronises the stream.
 * ---------------------------------------------------------------------- */
int n2v_autotune_workspace(const n2v_graph *g, uint32_t n_walks, uint32_t L, size_t *ws_bytes);
int n2v_autotune(n2v_graph *g, uint32_t n_walks, uint32_t L, float p, float q, void *ws,
                 size_t ws_bytes, void *stream, n2v_exec_opts *best, double *best_ms);

/* ------------------------------------------------------------------------
 * Serving (FN-Multi paragraph of Section 3.4: walks are independent, so work
 * can be cut into rounds and admitted as memory allows).  A server keeps the
 * graph resident and runs a scheduler thread that admits submitted requests
 * into a caller-provided device pool as space frees up, cuts them into walk
 * chunks, and launches chunks of several requests together on its stream, one
 * captured graph replay (table copy plus persistent kernel) per tick.
 * Results are identical to n2v_walk_approx (n2v_walk_ex when approx_t = 0)
 * with walk_base = 0 on the same request, alone or in any mix.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t max_queue;     /* pending requests accepted before N2V_EAGAIN (default 4096) */
    uint32_t chunk_walks;   /* walks per chunk (default 65536) */
    uint32_t max_inflight;  /* chunks per tick (default 64, at most 256) */
    uint32_t tick_walks;    /* walks per tick (default 2^19); ticks take chunks of the
                               requests with the least remaining work first */
} n2v_server_opts;

typedef struct {
    const uint32_t *host_starts;  /* host array, copied at submit */
    uint32_t n_starts;
    uint32_t L;
    float p, q;
    uint64_t seed;
    uint32_t approx_t;  /* FN-Approx threshold 1/approx_t as in n2v_walk_approx (0: exact) */
} n2v_request;

typedef struct {
    const uint32_t *d_out;  /* device, n_starts x (L+1); valid until n2v_release */
    uint32_t n_starts, L;
    uint64_t submit_ns, start_ns, done_ns;  /* CLOCK_MONOTONIC stamps */
} n2v_result;

void n2v_server_opts_default(n2v_server_opts *o);

/* pool: device memory of pool_bytes owned by the caller for the server's
 * lifetime.  The server launches on `stream` only. */
int n2v_server_create(const n2v_graph *g, void *pool, size_t pool_bytes, const n2v_server_opts *o,
                      void *stream, n2v_server **out);
/* Waits for in-flight work, then frees host state. */
int n2v_server_destroy(n2v_server *s);

/* Thread-safe, non-blocking.  Returns N2V_ETOOBIG when the request can never
 * fit the pool, N2V_EAGAIN when the queue is full, N2V_EINVAL on bad
 * arguments (including start ids >= n). */
int n2v_submit(n2v_server *s, const n2v_request *r, uint64_t *ticket);

/* N2V_PENDING until the request is complete, then N2V_OK with *res filled,
 * or the request's error.  N2V_ENOTFOUND for unknown tickets. */
int n2v_poll(n2v_server *s, uint64_t ticket, n2v_result *res);

/* Frees the request's pool space; its d_out becomes invalid. */
int n2v_release(n2v_server *s, uint64_t ticket);

/* Requests queued, admitted but not complete, and complete but unreleased. */
int n2v_server_stats(n2v_server *s, uint32_t *queued, uint32_t *running, uint32_t *done);

#ifdef __cplusplus
}
#endif

#endif /* N2V_H */
