// prims.hip -- device-wide exclusive prefix sum (reduce, scan of block sums,
// scan-and-add), used for CSR row offsets and radix-sort digit offsets.
#include "prims.hpp"

namespace n2v {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr uint64_t SCAN_TILE = (uint64_t)SCAN_THREADS * SCAN_ITEMS;

__device__ uint64_t block_excl_scan(uint64_t v, uint64_t *total)
{
    __shared__ uint64_t wsum[SCAN_THREADS / WAVE];
    const int w = threadIdx.x / WAVE, l = lane_id();
    uint64_t inc = wave_incl_scan(v);
    if (l == WAVE - 1) wsum[w] = inc;
    __syncthreads();
    uint64_t before = 0, all = 0;
    for (int i = 0; i < SCAN_THREADS / WAVE; ++i) {
        if (i < w) before += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const uint64_t *__restrict__ in, uint64_t n,
                                                              uint64_t *__restrict__ bsum)
{
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) s += in[base + i];
    uint64_t total;
    block_excl_scan(s, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(uint64_t *__restrict__ data, uint64_t n,
                                                             const uint64_t *__restrict__ boff)
{
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint64_t v[SCAN_ITEMS];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = base + i < n ? data[base + i] : 0;
        s += v[i];
    }
    uint64_t total;
    uint64_t run = block_excl_scan(s, &total) + (boff ? boff[blockIdx.x] : 0);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) data[base + i] = run;
        run += v[i];
    }
}

}  // namespace

size_t scan_scratch_bytes(uint64_t n)
{
    size_t bytes = 0;
    while (n > SCAN_TILE) {
        n = (n + SCAN_TILE - 1) / SCAN_TILE;
        bytes += ((n * sizeof(uint64_t)) + 255) & ~(size_t)255;
    }
    return bytes + 256;
}

int exclusive_scan_u64(uint64_t *data, uint64_t n, void *scratch, hipStream_t st)
{
    if (n == 0) return N2V_OK;
    const uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(SCAN_THREADS), 0, st, data, n, (const uint64_t *)nullptr);
        N2V_HIP(hipGetLastError());
        return N2V_OK;
    }
    uint64_t *bsum = (uint64_t *)scratch;
    void *rest = (char *)scratch + (((nb * sizeof(uint64_t)) + 255) & ~(size_t)255);
    hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)nb), dim3(SCAN_THREADS), 0, st, data, n, bsum);
    N2V_HIP(hipGetLastError());
    int rc = exclusive_scan_u64(bsum, nb, rest, st);
    if (rc != N2V_OK) return rc;
    hipLaunchKernelGGL(k_scan_apply, dim3((uint32_t)nb), dim3(SCAN_THREADS), 0, st, data, n,
                       (const uint64_t *)bsum);
    N2V_HIP(hipGetLastError());
    return N2V_OK;
}

}  // namespace n2v
