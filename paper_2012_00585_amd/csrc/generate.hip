// Element-matrix generator for benchmarks and serving: counter-based
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and two recipes whose
// arithmetic is exact or a fixed sequence of correctly rounded IEEE
// operations (the library is built without FMA contraction), so the
// matrices are reproducible bit for bit by any implementation of the same
// definition.  Entry i = r*n + s of element e takes 32-bit word i mod 4 of
// Philox(counter (i div 4, (e+e0) low, (e+e0) high, recipe), key (seed low,
// seed high)), u = word * 2^-32.
//
//   laplacian  K_rs = 2u - 1 for r < s (mirrored); K_rr = -sum_{s != r} K_rs
//              in increasing s
//   spd        B_rs = (u - 1/2) * sqrt(12) (unit variance);
//              K_rs = (sum_t B_rt B_st, t increasing) / n + [r == s]
//
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
constexpr double kSqrt12 = 3.4641016151377544;

// One 64-lane block per element; the uniforms in LDS (recipe 1: rows
// padded by one value, so that lanes reading different rows hit different
// banks), then the matrix.  Recipe 1 computes every entry, both triangles,
// in 3x3 register blocks: K_sr sums the same products (B_st B_rt equals
// B_rt B_st exactly) in the same order as K_rs, so the matrix is exactly
// symmetric, and all 64 lanes have work (8 x 8 blocks for n = 24).
__global__ void __launch_bounds__(64)
    k_gen(int recipe, int64_t n_elem, int32_t n, uint32_t k0, uint32_t k1, int64_t e0,
          double* __restrict__ ke) {
    extern __shared__ double B[];  // [n][ldb]
    const int32_t n2 = n * n;
    const int32_t ldb = recipe == 0 ? n : n + 1;
    const int32_t nb = (n + 2) / 3;
    for (int64_t e = blockIdx.x; e < n_elem; e += gridDim.x) {
        const uint64_t ge = (uint64_t)(e + e0);
        double* K = ke + e * (int64_t)n2;
        for (int32_t c = threadIdx.x; c * 4 < n2; c += 64) {
            uint32_t w[4] = {(uint32_t)c, (uint32_t)ge, (uint32_t)(ge >> 32), (uint32_t)recipe};
            philox4x32_10(w[0], w[1], w[2], w[3], k0, k1);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t i = c * 4 + q;
                if (i < n2) {
                    const double u = (double)w[q] * kTwoM32;
                    const int32_t r = i / n, s = i - r * n;
                    B[r * ldb + s] = recipe == 0 ? 2.0 * u - 1.0 : (u - 0.5) * kSqrt12;
                }
            }
        }
        __syncthreads();
        if (recipe == 0) {
            for (int32_t i = threadIdx.x; i < n2; i += 64) {
                const int32_t r = i / n, s = i - r * n;
                if (r != s) {
                    K[i] = r < s ? B[i] : B[s * n + r];
                } else {
                    double acc = 0.0;
                    for (int32_t t = 0; t < n; ++t)
                        if (t != r) acc = acc + (r < t ? B[r * n + t] : B[t * n + r]);
                    K[i] = -acc;
                }
            }
        } else {
            const double dn = (double)n;
            for (int32_t bi = threadIdx.x; bi < nb * nb; bi += 64) {
                const int32_t R = bi / nb, S = bi - R * nb;
                double acc[3][3] = {};
                for (int32_t t = 0; t < n; ++t) {
                    double br[3], bs[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const int32_t r = 3 * R + q, s = 3 * S + q;
                        br[q] = r < n ? B[r * ldb + t] : 0.0;
                        bs[q] = s < n ? B[s * ldb + t] : 0.0;
                    }
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) acc[a][b] = acc[a][b] + br[a] * bs[b];
                }
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const int32_t r = 3 * R + a, s = 3 * S + b;
                        if (r < n && s < n) {
                            double v = acc[a][b] / dn;
                            if (r == s) v = v + 1.0;
                            K[r * n + s] = v;
                        }
                    }
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
    if ((int64_t)n * (n + 1) * 8 > 64 * 1024) FEASM_FAIL(FEASM_ELIMIT, "generate_ke: n too large");
    if (n_elem == 0) return FEASM_OK;
    const unsigned grid = (unsigned)std::min<int64_t>(n_elem, 1 << 20);
    const size_t lds = (size_t)n * (recipe == 0 ? n : n + 1) * 8;
    k_gen<<<grid, 64, lds, stream>>>(recipe, n_elem, n, (uint32_t)seed, (uint32_t)(seed >> 32),
                                     elem_offset, ke);
    FEASM_HIP(hipGetLastError());
    return FEASM_OK;
}
