// skipgram.hip -- Skip-gram with negative sampling over node2vec walks.
//
// The walks feed a Skip-gram model (Section 1 and Section 2.1 of the paper:
// node2vec learns embeddings by running Skip-gram over its random walks).
// One training step over a batch of walks, every walk with its own set of
// shared negatives:
//   - centers: the walk's vertices x_0 .. x_{len-1} (len = entries before the
//     first sentinel); context of position i: positions j with
//     1 <= |i - j| <= window; negatives: the walk's `negatives` vertices drawn
//     from the noise distribution;
//   - z = v(center) . u(context or negative), v rows of `win`, u rows of `wout`;
//   - loss: softplus(-z) per (center, context) pair plus neg_weight *
//     softplus(z) per (center, negative) pair;
//   - gradient coefficients g = sigmoid(z) - 1 (context) and
//     neg_weight * sigmoid(z) (negative); dv = sum g u, du = sum g v;
//   - after every walk of the batch is evaluated against the same tables, both
//     tables take one SGD step in which each row moves by its mean gradient
//     per occurrence in the batch: w -= lr * gradient / occurrences.
// Per walk the contractions (logits, center gradients, target gradients)
// are dense products of at most 96 centers by 160 targets by 128
// dimensions; one workgroup evaluates them with bf16 MFMA (fp32 accumulate)
// from LDS tiles, and adds the gradient rows into fp32 gradient tables.
#include <math.h>

#include <algorithm>

#include "prims.hpp"

namespace n2v {

namespace {

constexpr int SG_DIM = 128;               // embedding dimension
constexpr int SG_MAXC = 96;               // walk positions per walk (L + 1 <= 96)
constexpr int SG_MAXNEG = 64;             // shared negatives per walk
constexpr int SG_T = SG_MAXC + SG_MAXNEG; // targets: walk positions, then negatives
constexpr int SG_BLOCK = 512;             // eight wavefronts, one product unit each
constexpr int LD_V = SG_DIM + 8;          // LDS row stride (bf16) of V[c][d] and T[t][d], padded against bank conflicts

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct SgArgs {
    const uint32_t *walks;   // n_walks x row_len
    const uint32_t *negs;    // n_walks x nneg
    const float *win, *wout; // n x SG_DIM
    float *gin, *gout;       // n x SG_DIM gradient accumulators
    float *cin, *cout;       // n occurrence counts of each row in the batch
    double *loss;
    uint32_t n_walks, row_len, nneg, window;
    float neg_weight;
};

// The rows of one walk in LDS, row-major bf16 (69 KB, so that two workgroups
// share a CU): center rows V (win) and target rows T (wout: the walk's
// positions, then its negatives).  The gradient products read the tables
// across rows (see lds_rows8) instead of keeping transposed copies, and take
// the coefficients straight from the logits' accumulators.
struct alignas(16) SgLds {
    __bf16 V[SG_MAXC * LD_V];
    __bf16 T[SG_T * LD_V];
    uint32_t ids[SG_T];
    float wloss[SG_BLOCK / WAVE];
};

__device__ __forceinline__ bf16x8 lds8(const __bf16 *p) { return *(const bf16x8 *)p; }

// One 32x32 output tile: sum over k < K of A[ra + i][k] * B[cb + j][k], with A
// and B row-major in LDS (row strides lda, ldb).  Lane l supplies row l % 32 of
// A and of B, k-slices 8 (l / 32) .. +8 of each 16-wide step.
template <int K>
__device__ __forceinline__ f32x16 tile_dot(const __bf16 *A, int lda, int ra, const __bf16 *B, int ldb, int cb)
{
    const int l = lane_id();
    const __bf16 *a = A + (ra + (l & 31)) * lda + 8 * (l >> 5);
    const __bf16 *b = B + (cb + (l & 31)) * ldb + 8 * (l >> 5);
    f32x16 acc = {};
#pragma unroll
    for (int k = 0; k < K; k += 16) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lds8(a + k), lds8(b + k), acc, 0, 0, 0);
    return acc;
}

// Row of accumulator register r of lane l within a 32x32 tile (its column is l % 32).
__device__ __forceinline__ int tile_row(int r) { return 8 * (r >> 2) + 4 * (lane_id() >> 5) + (r & 3); }

// A tile's accumulator registers 8s .. 8s+7 of lane l hold rows 16s + 4 (l /
// 32) + {0, 1, 2, 3, 8, 9, 10, 11} of column l % 32.  Used as the A operand
// of a 16-deep k-step (lane l: row l % 32, k = 8 (l / 32) + j), they contract
// over those rows in that order; this is the matching B operand from a
// row-major LDS table M: lane l supplies M[r][d0 + l % 32] for the same eight
// rows r, from r0 = tile base + 16s.
__device__ __forceinline__ bf16x8 lds_rows8(const __bf16 *M, int r0, int d0)
{
    const int l = lane_id();
    const __bf16 *p = M + (r0 + 4 * (l >> 5)) * LD_V + d0 + (l & 31);
    bf16x8 b;
    b[0] = p[0];
    b[1] = p[LD_V];
    b[2] = p[2 * LD_V];
    b[3] = p[3 * LD_V];
    b[4] = p[8 * LD_V];
    b[5] = p[9 * LD_V];
    b[6] = p[10 * LD_V];
    b[7] = p[11 * LD_V];
    return b;
}

// Gradient coefficient of the logit z of (center c, target t), adding its
// loss term to `loss`: context pairs (a walk position within the window)
// sigmoid(z) - 1, negatives neg_weight * sigmoid(z), anything else 0.  All
// come from e = exp(-|z|) and r = 1 / (1 + e) without cancellation:
// sigmoid(z) is r for z >= 0 and e r below, sigmoid(z) - 1 is -e r and -r,
// and softplus(-z) = max(-z, 0) + log(1 + e), softplus(z) = max(z, 0) +
// log(1 + e).  The hardware exponential and reciprocal leave a relative error
// of about (|z| + 4) 2^-24, far below the bf16 rounding of the logits and of
// the coefficients themselves.
__device__ __forceinline__ float sg_coef(const SgArgs &A, uint32_t len, uint32_t c, uint32_t t, float z, float &loss)
{
    if (c >= len) return 0.f;
    bool ctx = false;
    if (t < (uint32_t)SG_MAXC) {
        const uint32_t dist = c > t ? c - t : t - c;
        if (!(t < len && dist >= 1 && dist <= A.window)) return 0.f;
        ctx = true;
    } else if (t - SG_MAXC >= A.nneg) {
        return 0.f;
    }
    const float e = __expf(-fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.f + e);
    const float er = e * r;
    // log(1 + e): the series where 1 + e would round away most of e
    const float l1 = e < 0x1p-12f ? e * (1.f - 0.5f * e) : __logf(1.f + e);
    if (ctx) {
        loss += fmaxf(-z, 0.f) + l1;
        return z >= 0.f ? -er : -r;
    }
    loss += A.neg_weight * (fmaxf(z, 0.f) + l1);
    return A.neg_weight * (z >= 0.f ? r : er);
}

// Whether center block cb (centers 32 cb ..) and target block tb (walk
// positions 32 tb .. for tb < 3, negatives 32 (tb - 3) .. above) hold a pair
// with a nonzero coefficient; the products skip blocks without one.
__device__ __forceinline__ bool sg_block_live(const SgArgs &A, uint32_t len, uint32_t cb, uint32_t tb)
{
    if (32 * cb >= len) return false;
    if (tb < (uint32_t)(SG_MAXC / 32)) {
        if (32 * tb >= len) return false;
        return 32 * tb <= 32 * cb + 31 + A.window && 32 * tb + 31 + A.window >= 32 * cb;
    }
    return 32 * (tb - SG_MAXC / 32) < A.nneg;
}

__global__ __launch_bounds__(SG_BLOCK, 2) void k_sg_walks(SgArgs A)
{
    __shared__ SgLds S;
    const int tid = threadIdx.x, l = lane_id(), wv = tid / WAVE;
    const uint32_t walk = blockIdx.x;
    const uint32_t *row = A.walks + (uint64_t)walk * A.row_len;
    // positions before the first sentinel
    if (tid < SG_T) {
        uint32_t id = SENT;
        if (tid < SG_MAXC) id = (uint32_t)tid < A.row_len ? row[tid] : SENT;
        else if ((uint32_t)(tid - SG_MAXC) < A.nneg) id = A.negs[(uint64_t)walk * A.nneg + (tid - SG_MAXC)];
        S.ids[tid] = id;
    }
    __syncthreads();
    uint32_t len = 0;
    while (len < A.row_len && S.ids[len] != SENT) ++len;
    // occurrences: every valid center row and target row once per walk
    if (tid < SG_T) {
        if ((uint32_t)tid < len) atomicAdd(A.cin + S.ids[tid], 1.f);
        const bool tv = tid < SG_MAXC ? (uint32_t)tid < len : (uint32_t)(tid - SG_MAXC) < A.nneg;
        if (tv) atomicAdd(A.cout + S.ids[tid], 1.f);
    }
    // rows to bf16 tiles: 32 lanes per row, 4 floats each; a thread's GATHER
    // rows are loaded together, so their latencies overlap instead of adding up
    constexpr int NROWS = SG_MAXC + SG_T;                // 256 rows
    constexpr int RSTEP = SG_BLOCK / 32;                 // rows per pass of the block
    constexpr int GATHER = 16;                           // loads in flight per thread (one batch)
    static_assert(NROWS % (RSTEP * GATHER) == 0, "rows split evenly into gather batches");
    const int q = tid & 31;
    for (int r0 = tid / 32; r0 < NROWS; r0 += RSTEP * GATHER) {
        float4 x[GATHER];
#pragma unroll
        for (int k = 0; k < GATHER; ++k) {
            const int r = r0 + k * RSTEP;
            const bool center = r < SG_MAXC;
            const int t = center ? r : r - SG_MAXC;
            const uint32_t id = S.ids[t];
            const bool valid =
                center ? (uint32_t)r < len : (t < SG_MAXC ? (uint32_t)t < len : (uint32_t)(t - SG_MAXC) < A.nneg);
            x[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (valid) x[k] = *(const float4 *)((center ? A.win : A.wout) + (uint64_t)id * SG_DIM + 4 * q);
        }
#pragma unroll
        for (int k = 0; k < GATHER; ++k) {
            const int r = r0 + k * RSTEP;
            const bool center = r < SG_MAXC;
            const int t = center ? r : r - SG_MAXC;
            bf16x4 b;
            b[0] = (__bf16)x[k].x;
            b[1] = (__bf16)x[k].y;
            b[2] = (__bf16)x[k].z;
            b[3] = (__bf16)x[k].w;
            *(bf16x4 *)((center ? S.V : S.T) + t * LD_V + 4 * q) = b;
        }
    }
    __syncthreads();
    // Eight units, one per wavefront (unit wv), each for all four 32-wide
    // column blocks of the 128 dimensions:
    //   units 0..2: center gradients dV = G T of center block ci = u: the
    //     logits of the block, transposed (Z^T = T V^T, lanes hold centers),
    //     give the A operands directly, T rows the B operands;
    //   units 3..7: target gradients dT = G^T V of target block tj = u - 3:
    //     the logits Z = V T^T (lanes hold targets) give the A operands, V
    //     rows the B operands; these units also add up the loss.
    float loss = 0.f;
    static_assert(SG_BLOCK / WAVE == 8, "one product unit per wavefront");
    {
        const int u = wv;
        const bool centers = u < 3;
        const int blk = centers ? u : u - 3;
        f32x16 acc[4];
#pragma unroll
        for (int dj = 0; dj < 4; ++dj) acc[dj] = f32x16{};
        const int nk = centers ? SG_T / 32 : SG_MAXC / 32;  // 32-row blocks of the contraction
        for (int kb = 0; kb < nk; ++kb) {
            if (!(centers ? sg_block_live(A, len, blk, kb) : sg_block_live(A, len, kb, blk))) continue;
            // logits tile: rows kb-block of the other side, columns (lanes) this unit's block
            const f32x16 z = centers ? tile_dot<SG_DIM>(S.T, LD_V, 32 * kb, S.V, LD_V, 32 * blk)
                                     : tile_dot<SG_DIM>(S.V, LD_V, 32 * kb, S.T, LD_V, 32 * blk);
            bf16x8 a0, a1;
            float dummy = 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t rr = 32 * kb + tile_row(r), ll = 32 * blk + (l & 31);
                const float g = centers ? sg_coef(A, len, ll, rr, z[r], dummy) : sg_coef(A, len, rr, ll, z[r], loss);
                if (r < 8) a0[r] = (__bf16)g;
                else a1[r - 8] = (__bf16)g;
            }
            const __bf16 *M = centers ? S.T : S.V;
#pragma unroll
            for (int dj = 0; dj < 4; ++dj) {
                acc[dj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, lds_rows8(M, 32 * kb, 32 * dj), acc[dj], 0, 0, 0);
                acc[dj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, lds_rows8(M, 32 * kb + 16, 32 * dj), acc[dj], 0, 0,
                                                                  0);
            }
        }
        // rows of acc: this unit's block (centers or targets), columns d
#pragma unroll
        for (int dj = 0; dj < 4; ++dj) {
            const int d = 32 * dj + (l & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t i = 32 * blk + tile_row(r);
                if (centers) {
                    if (i < len) atomicAdd(A.gin + (uint64_t)S.ids[i] * SG_DIM + d, acc[dj][r]);
                } else {
                    const bool valid = i < (uint32_t)SG_MAXC ? i < len : i - SG_MAXC < A.nneg;
                    if (valid) atomicAdd(A.gout + (uint64_t)S.ids[i] * SG_DIM + d, acc[dj][r]);
                }
            }
        }
    }
    // loss of the workgroup
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) loss += __shfl_xor(loss, m, WAVE);
    if (l == 0) S.wloss[wv] = loss;
    __syncthreads();
    if (tid == 0) {
        float s = 0.f;
        for (int w = 0; w < SG_BLOCK / WAVE; ++w) s += S.wloss[w];
        if (s != 0.f) atomicAdd(A.loss, (double)s);
    }
}

// w -= lr * g / max(1, c) and g = 0, c = 0 over a table of rows of SG_DIM
// floats.  The 32 float4 of a row sit in one half of a wavefront (the stride
// is a multiple of 64 threads), so every lane of the row reads c before its
// first lane clears it.
__global__ __launch_bounds__(256) void k_sg_apply(float *__restrict__ w, float *__restrict__ g, float *__restrict__ c,
                                                  uint64_t count4, float lr)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count4; i += stride) {
        const uint64_t row = i / (SG_DIM / 4);
        const float occ = c[row];
        const float s = lr / (occ > 1.f ? occ : 1.f);
        float4 a = ((float4 *)w)[i];
        const float4 b = ((float4 *)g)[i];
        a.x -= s * b.x;
        a.y -= s * b.y;
        a.z -= s * b.z;
        a.w -= s * b.w;
        ((float4 *)w)[i] = a;
        ((float4 *)g)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        __builtin_amdgcn_wave_barrier();
        if ((i & (SG_DIM / 4 - 1)) == 0 && occ != 0.f) c[row] = 0.f;
    }
}

// Negative k of walk i: r = hi64(R1, total) with R1 from Philox(seed; (walk
// id, k, step, 6)); the vertex x with cum[x] <= r < cum[x+1].
__global__ __launch_bounds__(256) void k_sg_negatives(const uint64_t *__restrict__ cum, uint32_t n, uint32_t k0,
                                                      uint32_t k1, uint32_t wbase, uint32_t step, uint32_t n_walks,
                                                      uint32_t nneg, uint32_t *__restrict__ out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)n_walks * nneg) return;
    const uint32_t w = (uint32_t)(i / nneg), k = (uint32_t)(i % nneg);
    const R4 r = philox(k0, k1, wbase + w, k, step, 6u);
    const uint64_t target = hi64(join64(r.x, r.y), cum[n]);
    uint32_t lo = 0, hi = n;  // first x with cum[x + 1] > target
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (cum[mid + 1] > target) hi = mid;
        else lo = mid + 1;
    }
    out[i] = lo;
}

struct SgLayout {
    float *gin, *gout;
    float *cin, *cout;
    uint32_t *negs;
};

size_t sg_layout(uint32_t n, uint32_t n_walks, uint32_t nneg, void *ws, size_t ws_bytes, SgLayout *L)
{
    Carver c(ws, ws_bytes);
    L->gin = c.take<float>((uint64_t)n * SG_DIM);
    L->gout = c.take<float>((uint64_t)n * SG_DIM);
    L->cin = c.take<float>(n);
    L->cout = c.take<float>(n);
    L->negs = c.take<uint32_t>((uint64_t)(n_walks ? n_walks : 1) * (nneg ? nneg : 1));
    return c.total();
}

}  // namespace

}  // namespace n2v

using namespace n2v;

extern "C" int n2v_sgns_workspace(uint32_t n, uint32_t dim, uint32_t n_walks, uint32_t negatives, size_t *ws_bytes)
{
    if (!ws_bytes || n == 0) return set_error(N2V_EINVAL, "n2v_sgns_workspace: bad argument");
    if (dim != SG_DIM) return set_error(N2V_EINVAL, "n2v_sgns_workspace: dim must be %d", SG_DIM);
    SgLayout L;
    *ws_bytes = sg_layout(n, n_walks, negatives, nullptr, 0, &L);
    return N2V_OK;
}

extern "C" int n2v_sgns_negatives(const uint64_t *cum, uint32_t n, uint64_t seed, uint64_t walk_base, uint32_t step,
                                  uint32_t n_walks, uint32_t negatives, uint32_t *out, void *stream)
{
    if (!cum || !out || n == 0) return set_error(N2V_EINVAL, "n2v_sgns_negatives: bad argument");
    if (walk_base + (uint64_t)n_walks > (1ull << 32)) return set_error(N2V_EINVAL, "n2v_sgns_negatives: walk ids exceed 2^32");
    const uint64_t count = (uint64_t)n_walks * negatives;
    if (count == 0) return N2V_OK;
    if (count > 0xFFFFFFFFull * 256) return set_error(N2V_EINVAL, "n2v_sgns_negatives: too many draws");
    hipLaunchKernelGGL(k_sg_negatives, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream, cum,
                       n, (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)walk_base, step, n_walks, negatives, out);
    N2V_HIP(hipGetLastError());
    return N2V_OK;
}

extern "C" int n2v_sgns_step(const n2v_sgns_params *prm, const uint32_t *walks, uint32_t n_walks, uint32_t row_len,
                             uint64_t walk_base, const uint64_t *cum, uint32_t n, float *win, float *wout, void *ws,
                             size_t ws_bytes, double *loss, void *stream)
{
    if (!prm || !walks || !cum || !win || !wout || !ws || !loss || n == 0)
        return set_error(N2V_EINVAL, "n2v_sgns_step: null argument");
    if (prm->dim != SG_DIM) return set_error(N2V_EINVAL, "n2v_sgns_step: dim must be %d", SG_DIM);
    if (row_len < 1 || row_len > (uint32_t)SG_MAXC)
        return set_error(N2V_EINVAL, "n2v_sgns_step: rows of 1 .. %d entries (walks of at most %d moves)", SG_MAXC,
                         SG_MAXC - 1);
    if (prm->negatives > (uint32_t)SG_MAXNEG)
        return set_error(N2V_EINVAL, "n2v_sgns_step: at most %d negatives per walk", SG_MAXNEG);
    if (n_walks >= 0x80000000u) return set_error(N2V_EINVAL, "n2v_sgns_step: at most 2^31-1 walks per step");
    if (((uintptr_t)ws & 255) != 0 || ((uintptr_t)win & 15) != 0 || ((uintptr_t)wout & 15) != 0)
        return set_error(N2V_EINVAL, "n2v_sgns_step: workspace must be 256-byte and tables 16-byte aligned");
    SgLayout L;
    const size_t need = sg_layout(n, n_walks, prm->negatives, ws, ws_bytes, &L);
    if (need > ws_bytes) return set_error(N2V_ENOMEM, "n2v_sgns_step: workspace %zu < %zu bytes", ws_bytes, need);
    if (n_walks == 0) return N2V_OK;
    hipStream_t st = (hipStream_t)stream;
    int rc = n2v_sgns_negatives(cum, n, prm->seed, walk_base, prm->step, n_walks, prm->negatives, L.negs, stream);
    if (rc) return rc;
    SgArgs A;
    A.walks = walks;
    A.negs = L.negs;
    A.win = win;
    A.wout = wout;
    A.gin = L.gin;
    A.gout = L.gout;
    A.cin = L.cin;
    A.cout = L.cout;
    A.loss = loss;
    A.n_walks = n_walks;
    A.row_len = row_len;
    A.nneg = prm->negatives;
    A.window = prm->window;
    A.neg_weight = prm->neg_weight;
    hipLaunchKernelGGL(k_sg_walks, dim3(n_walks), dim3(SG_BLOCK), 0, st, A);
    N2V_HIP(hipGetLastError());
    const uint64_t count4 = (uint64_t)n * SG_DIM / 4;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((count4 + 255) / 256, 8192);
    hipLaunchKernelGGL(k_sg_apply, dim3(blocks), dim3(256), 0, st, win, L.gin, L.cin, count4, prm->lr);
    hipLaunchKernelGGL(k_sg_apply, dim3(blocks), dim3(256), 0, st, wout, L.gout, L.cout, count4, prm->lr);
    N2V_HIP(hipGetLastError());
    return N2V_OK;
}
