// Element-matrix generator for benchmarks and serving: counter-based
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and two recipes whose
// arithmetic is exact or a fixed sequence of correctly rounded IEEE
// operations (no fused multiply-add), so the matrices are reproducible bit
// for bit by any implementation of the same definition.
//
//   laplacian  K_rs = 2u - 1 (r < s, mirrored), K_rr = -sum_{s != r} K_rs
//   spd        B_ij = (((u0+u1)+u2)+u3 - 2) * sqrt(3);  K = B B^T / n + I
//
// u = x * 2^-32 for a 32-bit Philox output x; element e uses counters
// (entry, (e+e0) low, (e+e0) high, recipe) under key (seed low, seed high).
// This is workload generation, not part of the assembly method.
#include <algorithm>

#include "internal.h"

namespace feasm {
namespace {

__device__ inline void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

constexpr double kTwoM32 = 2.3283064365386963e-10;  // 2^-32
constexpr double kSqrt3 = 1.7320508075688772;

// One block per element; K staged in LDS.
__global__ void __launch_bounds__(256)
    k_gen(int kind, int64_t n_elem, int32_t n, uint32_t k0, uint32_t k1, int64_t e0,
          double* __restrict__ ke) {
    extern __shared__ double sm[];
    double* B = sm;  // [n][n]
    const int32_t n2 = n * n;
    for (int64_t e = blockIdx.x; e < n_elem; e += gridDim.x) {
        const uint64_t ge = (uint64_t)(e + e0);
        double* K = ke + e * (int64_t)n2;
        if (kind == 0) {
            for (int32_t i = threadIdx.x; i < n2; i += blockDim.x) {
                uint32_t c0 = (uint32_t)i, c1 = (uint32_t)ge, c2 = (uint32_t)(ge >> 32), c3 = 0;
                philox4x32_10(c0, c1, c2, c3, k0, k1);
                B[i] = __dsub_rn(__dmul_rn(2.0, __dmul_rn((double)c0, kTwoM32)), 1.0);
            }
            __syncthreads();
            for (int32_t i = threadIdx.x; i < n2; i += blockDim.x) {
                const int32_t r = i / n, s = i - r * n;
                if (r < s) {
                    K[i] = B[i];
                } else if (r > s) {
                    K[i] = B[s * n + r];
                } else {
                    double acc = 0.0;
                    for (int32_t t = 0; t < n; ++t)
                        if (t != r) acc = __dadd_rn(acc, r < t ? B[r * n + t] : B[t * n + r]);
                    K[i] = -acc;
                }
            }
        } else {
            for (int32_t i = threadIdx.x; i < n2; i += blockDim.x) {
                uint32_t c0 = (uint32_t)i, c1 = (uint32_t)ge, c2 = (uint32_t)(ge >> 32), c3 = 1;
                philox4x32_10(c0, c1, c2, c3, k0, k1);
                double u = __dadd_rn(__dmul_rn((double)c0, kTwoM32), __dmul_rn((double)c1, kTwoM32));
                u = __dadd_rn(u, __dmul_rn((double)c2, kTwoM32));
                u = __dadd_rn(u, __dmul_rn((double)c3, kTwoM32));
                B[i] = __dmul_rn(__dsub_rn(u, 2.0), kSqrt3);
            }
            __syncthreads();
            for (int32_t i = threadIdx.x; i < n2; i += blockDim.x) {
                const int32_t r = i / n, s = i - r * n;
                double acc = 0.0;
                for (int32_t t = 0; t < n; ++t)
                    acc = __dadd_rn(acc, __dmul_rn(B[r * n + t], B[s * n + t]));
                double v = __ddiv_rn(acc, (double)n);
                if (r == s) v = __dadd_rn(v, 1.0);
                K[i] = v;
            }
        }
        __syncthreads();
    }
}

}  // namespace
}  // namespace feasm

extern "C" int generate_ke(int recipe, int64_t n_elem, int32_t n, uint64_t seed, int64_t elem_offset,
                           double* ke, hipStream_t stream) {
    using namespace feasm;
    if (!ke) FEASM_FAIL(FEASM_EINVAL, "generate_ke: ke is NULL");
    if (recipe != 0 && recipe != 1) FEASM_FAIL(FEASM_EINVAL, "generate_ke: unknown recipe");
    if (n_elem < 0 || n <= 0 || elem_offset < 0) FEASM_FAIL(FEASM_EINVAL, "generate_ke: bad size");
    if ((int64_t)n * n * 8 > 64 * 1024) FEASM_FAIL(FEASM_ELIMIT, "generate_ke: n too large");
    if (n_elem == 0) return FEASM_OK;
    const unsigned grid = (unsigned)std::min<int64_t>(n_elem, 65536);
    k_gen<<<grid, 256, (size_t)n * n * 8, stream>>>(recipe, n_elem, n, (uint32_t)seed,
                                                    (uint32_t)(seed >> 32), elem_offset, ke);
    FEASM_HIP(hipGetLastError());
    return FEASM_OK;
}
