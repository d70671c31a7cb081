// Device-wide exclusive prefix sum (used by the symbolic phase).
//
// Three-kernel scheme per level: per-tile reduction, recursive scan of the
// tile sums, then per-tile scan with wavefront shuffles plus a carry.
#include "internal.h"

namespace feasm {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int64_t kScanTile = (int64_t)kScanBlock * kScanItems;
constexpr int kWaves = kScanBlock / 64;

__device__ inline int64_t block_sum(int64_t v, int64_t* wsum) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wsum[w] = v;
    __syncthreads();
    int64_t total = 0;
    for (int i = 0; i < kWaves; ++i) total += wsum[i];
    __syncthreads();
    return total;
}

// Inclusive scan of one value per thread over the block; `total` gets the block sum.
__device__ inline int64_t block_incl_scan(int64_t v, int64_t* wsum, int64_t& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        int64_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    int64_t pre = 0;
    total = 0;
    for (int i = 0; i < kWaves; ++i) {
        if (i < w) pre += wsum[i];
        total += wsum[i];
    }
    __syncthreads();
    return v + pre;
}

template <typename T>
__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(const T* __restrict__ in, int64_t n,
                                                           int64_t* __restrict__ sums) {
    __shared__ int64_t wsum[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t acc = 0;
    for (int i = threadIdx.x; i < kScanTile; i += kScanBlock) {
        const int64_t idx = base + i;
        if (idx < n) acc += (int64_t)in[idx];
    }
    acc = block_sum(acc, wsum);
    if (threadIdx.x == 0) sums[blockIdx.x] = acc;
}

// offs may be null (single tile).  The last block writes out[n].
template <typename T>
__global__ void __launch_bounds__(kScanBlock) k_scan_apply(const T* __restrict__ in, int64_t n,
                                                          const int64_t* __restrict__ offs,
                                                          int64_t* __restrict__ out) {
    __shared__ int64_t wsum[kWaves];
    int64_t carry = offs ? offs[blockIdx.x] : 0;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t idx = base + (int64_t)r * kScanBlock + threadIdx.x;
        const int64_t v = idx < n ? (int64_t)in[idx] : 0;
        int64_t total;
        const int64_t incl = block_incl_scan(v, wsum, total);
        if (idx < n) out[idx] = carry + incl - v;
        carry += total;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = carry;
}

}  // namespace

int64_t scan_scratch_elems(int64_t n) {
    if (n <= kScanTile) return 1;
    const int64_t nb = ceil_div(n, kScanTile);
    return nb + (nb + 1) + scan_scratch_elems(nb);
}

template <typename T>
int exclusive_scan(const T* in, int64_t n, int64_t* out, int64_t* scratch, hipStream_t s) {
    if (n <= kScanTile) {
        k_scan_apply<T><<<1, kScanBlock, 0, s>>>(in, n, nullptr, out);
        FEASM_HIP(hipGetLastError());
        return FEASM_OK;
    }
    const int64_t nb = ceil_div(n, kScanTile);
    int64_t* sums = scratch;
    int64_t* offs = scratch + nb;
    int64_t* rest = offs + nb + 1;
    k_scan_reduce<T><<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, sums);
    FEASM_HIP(hipGetLastError());
    int rc = exclusive_scan<int64_t>(sums, nb, offs, rest, s);
    if (rc != FEASM_OK) return rc;
    k_scan_apply<T><<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, offs, out);
    FEASM_HIP(hipGetLastError());
    return FEASM_OK;
}

template int exclusive_scan<int32_t>(const int32_t*, int64_t, int64_t*, int64_t*, hipStream_t);
template int exclusive_scan<int64_t>(const int64_t*, int64_t, int64_t*, int64_t*, hipStream_t);

}  // namespace feasm
