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

// The four words of entries 4c .. 4c+3 of global element ge.
__device__ inline void philox_block(int32_t c, uint64_t ge, int recipe, uint32_t k0, uint32_t k1,
                                    uint32_t (&w)[4]) {
    w[0] = (uint32_t)c;
    w[1] = (uint32_t)ge;
    w[2] = (uint32_t)(ge >> 32);
    w[3] = (uint32_t)recipe;
    philox4x32_10(w[0], w[1], w[2], w[3], k0, k1);
}

// Uniform u of entry i of global element ge (word i mod 4 of its block).
__device__ inline double entry_uniform(int32_t i, uint64_t ge, int recipe, uint32_t k0, uint32_t k1) {
    uint32_t w[4];
    philox_block(i >> 2, ge, recipe, k0, k1, w);
    const int q = i & 3;
    const uint32_t word = q == 0 ? w[0] : q == 1 ? w[1] : q == 2 ? w[2] : w[3];
    return (double)word * kTwoM32;
}

// Diagonal entry r of the zero-row-sum recipe from its strict upper
// triangle U (row-major, n columns): minus the sum of row r's off-diagonal
// entries, in increasing column.
__device__ inline double laplacian_diagonal(const double* U, int32_t n, int32_t r) {
    double acc = 0.0;
    for (int32_t t = 0; t < n; ++t)
        if (t != r) acc = acc + (r < t ? U[r * n + t] : U[t * n + r]);
    return -acc;
}

// 3x3 block (R, S) of B B^T: acc[a][b] = sum over t, increasing, of
// B[3R+a][t] B[3S+b][t] (rows past n count as zero).
__device__ inline void spd_block(const double* B, int32_t ldb, int32_t n, int32_t R, int32_t S,
                                 double (&acc)[3][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[a][b] = 0.0;
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
}

// The sizes the kernels below are not compiled for (zero-row-sum with
// n*n > 64, SPD with n not in {8, 16, 24, 32, 40}): one 64-lane block per
// element; the uniforms in LDS (recipe 1: rows padded by one value, so that
// lanes reading different rows hit different banks), then the matrix.
// Recipe 1 computes every entry, both triangles, in 3x3 register blocks:
// K_sr sums the same products (B_st B_rt equals B_rt B_st exactly) in the
// same order as K_rs, so the matrix is exactly symmetric.  Where
// the blocks fit one pass of the lanes (n <= 24) the matrix is staged in
// LDS and stored by consecutive lanes, so that every store instruction
// covers whole lines; the element matrices are written with non-temporal
// stores (they are read once, by a later kernel).
// MODE: 0 zero-row-sum, 1 SPD staged (n <= 24), 2 SPD with direct stores.
template <int MODE>
__global__ void __launch_bounds__(64)
    k_gen(int64_t n_elem, int32_t n, uint32_t k0, uint32_t k1, int64_t e0, double* __restrict__ ke) {
    constexpr int recipe = MODE == 0 ? 0 : 1;
    extern __shared__ double B[];  // [n][ldb]
    const int32_t n2 = n * n;
    const int32_t ldb = recipe == 0 ? n : n + 1;
    const int32_t nb = (n + 2) / 3;
    const double dn = (double)n;
    for (int64_t e = blockIdx.x; e < n_elem; e += gridDim.x) {
        const uint64_t ge = (uint64_t)(e + e0);
        double* K = ke + e * (int64_t)n2;
        for (int32_t c = threadIdx.x; c * 4 < n2; c += 64) {
            uint32_t w[4];
            philox_block(c, ge, recipe, k0, k1, w);
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
        if (MODE == 0) {
            for (int32_t i = threadIdx.x; i < n2; i += 64) {
                const int32_t r = i / n, s = i - r * n;
                const double v = r == s ? laplacian_diagonal(B, n, r) : r < s ? B[i] : B[s * n + r];
                __builtin_nontemporal_store(v, K + i);
            }
        } else if (MODE == 1) {
            const int32_t bi = threadIdx.x, R = bi / nb, S = bi - R * nb;
            double acc[3][3];
            if (bi < nb * nb) spd_block(B, ldb, n, R, S, acc);
            __syncthreads();  // every lane has read B; it now holds K
            if (bi < nb * nb) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const int32_t r = 3 * R + a, s = 3 * S + b;
                        if (r < n && s < n) {
                            double v = acc[a][b] / dn;
                            if (r == s) v = v + 1.0;
                            B[r * n + s] = v;
                        }
                    }
            }
            __syncthreads();
            for (int32_t i = threadIdx.x; i < n2; i += 64) __builtin_nontemporal_store(B[i], K + i);
        } else {
            for (int32_t bi = threadIdx.x; bi < nb * nb; bi += 64) {
                const int32_t R = bi / nb, S = bi - R * nb;
                double acc[3][3];
                spd_block(B, ldb, n, R, S, acc);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const int32_t r = 3 * R + a, s = 3 * S + b;
                        if (r < n && s < n) {
                            double v = acc[a][b] / dn;
                            if (r == s) v = v + 1.0;
                            __builtin_nontemporal_store(v, K + r * n + s);
                        }
                    }
            }
        }
        __syncthreads();
    }
}

// Zero-row-sum recipe for the other n with n*n <= 64: 64/L elements per
// 64-lane block, L = 2^lpe_log2 >= n*n lanes per element; lane (g, i) draws
// entry i of element g into LDS, then writes entry i of the matrix.
__global__ void __launch_bounds__(64)
    k_gen_laplacian_small(int64_t n_elem, int32_t n, int32_t lpe_log2, uint32_t k0, uint32_t k1,
                          int64_t e0, double* __restrict__ ke) {
    __shared__ double U[64];
    const int32_t n2 = n * n, G = 64 >> lpe_log2;
    const int l = threadIdx.x, g = l >> lpe_log2, i = l & ((1 << lpe_log2) - 1);
    const double* Ug = U + (g << lpe_log2);
    for (int64_t eb = (int64_t)blockIdx.x * G; eb < n_elem; eb += (int64_t)gridDim.x * G) {
        const int64_t e = eb + g;
        const bool valid = e < n_elem && i < n2;
        if (valid) U[l] = 2.0 * entry_uniform(i, (uint64_t)(e + e0), 0, k0, k1) - 1.0;
        __syncthreads();
        if (valid) {
            const int32_t r = i / n, s = i - r * n;
            const double v = r == s ? laplacian_diagonal(Ug, n, r) : r < s ? Ug[i] : Ug[s * n + r];
            __builtin_nontemporal_store(v, ke + e * (int64_t)n2 + i);
        }
        __syncthreads();
    }
}

// Zero-row-sum recipe for N = 2, 4, 8: lane (j, c) draws Philox block c of
// element j (G = 64 / (N*N/4) elements per 64-lane block, each block drawn
// once), then the lanes write the G matrices' entries in order, consecutive
// lanes to consecutive addresses.
template <int N>
__global__ void __launch_bounds__(64)
    k_gen_laplacian_blocks(int64_t n_elem, uint32_t k0, uint32_t k1, int64_t e0,
                           double* __restrict__ ke) {
    constexpr int N2 = N * N, CH = N2 / 4, G = 64 / CH;
    __shared__ double U[G * N2];
    const int l = threadIdx.x, j0 = l / CH, c0 = l - j0 * CH;
    for (int64_t eb = (int64_t)blockIdx.x * G; eb < n_elem; eb += (int64_t)gridDim.x * G) {
        const int32_t here = (int32_t)(n_elem - eb < G ? n_elem - eb : G);
        if (j0 < here) {
            uint32_t w[4];
            philox_block(c0, (uint64_t)(eb + j0 + e0), 0, k0, k1, w);
#pragma unroll
            for (int q = 0; q < 4; ++q) U[j0 * N2 + 4 * c0 + q] = 2.0 * ((double)w[q] * kTwoM32) - 1.0;
        }
        __syncthreads();
        double* out = ke + eb * (int64_t)N2;
        for (int32_t i = l; i < here * N2; i += 64) {
            const int32_t j = i / N2, x = i - j * N2, r = x / N, s = x - r * N;
            const double* Uj = U + j * N2;
            const double v = r == s ? laplacian_diagonal(Uj, N, r) : r < s ? Uj[x] : Uj[s * N + r];
            __builtin_nontemporal_store(v, out + i);
        }
        __syncthreads();
    }
}

template <int N>
int launch_laplacian_blocks(int64_t n_elem, uint64_t seed, int64_t elem_offset, double* ke,
                            hipStream_t stream) {
    constexpr int G = 64 / (N * N / 4);
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n_elem, G), 1 << 20);
    k_gen_laplacian_blocks<N><<<grid, 64, 0, stream>>>(n_elem, (uint32_t)seed, (uint32_t)(seed >> 32),
                                                       elem_offset, ke);
    FEASM_HIP(hipGetLastError());
    return FEASM_OK;
}

// SPD recipe for n = N = 4m <= 40: only the m(m+1)/2 upper-triangle 4x4
// blocks of B B^T are summed, and each is written to both triangles (K_sr
// sums the same products, in the same order, as K_rs).  G = 64 / (m(m+1)/2)
// elements per 64-lane block (3 for N = 24, 63 of 64 lanes busy).  LDS holds
// each element's B transposed (column t of B contiguous, so that a lane
// reads its four rows' entries of column t as two 16-byte words), later the
// element's K, which consecutive lanes store as whole lines.  Rows of both
// are N + 2 values apart, so that the lanes writing one column of B, or one
// column of a K block, fall on different banks.
template <int N>
__global__ void __launch_bounds__(64)
    k_gen_spd_upper(int64_t n_elem, uint32_t k0, uint32_t k1, int64_t e0, double* __restrict__ ke) {
    constexpr int M = N / 4, U = M * (M + 1) / 2, G = 64 / U, N2 = N * N, CH = N2 / 4;
    constexpr int LD = N + 2, P = N * LD;  // row stride and element stride in LDS
    extern __shared__ double L[];           // [G][N][LD]
    const double dn = (double)N;
    const int l = threadIdx.x, g = l / U;
    int32_t blk = l - g * U, R = 0;
    while (R < M - 1 && blk >= M - R) {
        blk -= M - R;
        ++R;
    }
    const int32_t S = R + blk;
    for (int64_t eb = (int64_t)blockIdx.x * G; eb < n_elem; eb += (int64_t)gridDim.x * G) {
        const int32_t here = (int32_t)(n_elem - eb < G ? n_elem - eb : G);
        for (int32_t x = l; x < here * CH; x += 64) {
            const int32_t j = x / CH, c = x - j * CH;
            uint32_t w[4];
            philox_block(c, (uint64_t)(eb + j + e0), 1, k0, k1, w);
            double* Bt = L + j * P;
            const int32_t r = (4 * c) / N, s = 4 * c - r * N;  // four entries of row r
#pragma unroll
            for (int q = 0; q < 4; ++q) Bt[(s + q) * LD + r] = ((double)w[q] * kTwoM32 - 0.5) * kSqrt12;
        }
        __syncthreads();
        const bool work = g < here;
        double acc[4][4];
        if (work) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
            const double* Bt = L + g * P;
            for (int32_t t = 0; t < N; ++t) {
                const double2* pr = reinterpret_cast<const double2*>(Bt + t * LD + 4 * R);
                const double2* ps = reinterpret_cast<const double2*>(Bt + t * LD + 4 * S);
                const double2 r01 = pr[0], r23 = pr[1], s01 = ps[0], s23 = ps[1];
                const double br[4] = {r01.x, r01.y, r23.x, r23.y};
                const double bs[4] = {s01.x, s01.y, s23.x, s23.y};
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] = acc[a][b] + br[a] * bs[b];
            }
        }
        __syncthreads();  // every lane has read B; LDS now takes K
        if (work) {
            double* Kl = L + g * P;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int32_t r = 4 * R + a, s = 4 * S + b;
                    double v = acc[a][b] / dn;
                    if (r == s) v = v + 1.0;
                    Kl[r * LD + s] = v;
                    if (R != S) Kl[s * LD + r] = v;
                }
        }
        __syncthreads();
        double* out = ke + eb * (int64_t)N2;
        for (int32_t i = l; i < here * N2; i += 64) {
            const int32_t j = i / N2, w = i - j * N2, r = w / N, s = w - r * N;
            __builtin_nontemporal_store(L[j * P + r * LD + s], out + i);
        }
        __syncthreads();
    }
}

template <int N>
int launch_spd_upper(int64_t n_elem, uint64_t seed, int64_t elem_offset, double* ke, hipStream_t stream) {
    constexpr int M = N / 4, G = 64 / (M * (M + 1) / 2);
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n_elem, G), 1 << 20);
    const size_t lds = (size_t)G * N * (N + 2) * 8;
    k_gen_spd_upper<N><<<grid, 64, lds, stream>>>(n_elem, (uint32_t)seed, (uint32_t)(seed >> 32),
                                                  elem_offset, ke);
    FEASM_HIP(hipGetLastError());
    return FEASM_OK;
}

}  // namespace
}  // namespace feasm

extern "C" int generate_ke(int recipe, int64_t n_elem, int32_t n, uint64_t seed, int64_t elem_offset,
                           double* ke, hipStream_t stream) {
    return feasm::guarded("generate_ke", [&]() -> int {
        using namespace feasm;
        if (!ke) FEASM_FAIL(FEASM_EINVAL, "generate_ke: ke is NULL");
        if (recipe != 0 && recipe != 1) FEASM_FAIL(FEASM_EINVAL, "generate_ke: unknown recipe");
        if (n_elem < 0 || n <= 0 || elem_offset < 0) FEASM_FAIL(FEASM_EINVAL, "generate_ke: bad size");
        if ((int64_t)n * (n + 1) * 8 > 64 * 1024) FEASM_FAIL(FEASM_ELIMIT, "generate_ke: n too large");
        if (n_elem == 0) return FEASM_OK;
        if (recipe == 0) {
            switch (n) {
                case 2: return launch_laplacian_blocks<2>(n_elem, seed, elem_offset, ke, stream);
                case 4: return launch_laplacian_blocks<4>(n_elem, seed, elem_offset, ke, stream);
                case 8: return launch_laplacian_blocks<8>(n_elem, seed, elem_offset, ke, stream);
                default: break;
            }
        }
        if (recipe == 0 && n * n <= 64) {
            int32_t lg = 0;
            while ((1 << lg) < n * n) ++lg;
            const int64_t per_block = 64 >> lg;
            const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n_elem, per_block), 1 << 20);
            k_gen_laplacian_small<<<grid, 64, 0, stream>>>(n_elem, n, lg, (uint32_t)seed,
                                                           (uint32_t)(seed >> 32), elem_offset, ke);
            FEASM_HIP(hipGetLastError());
            return FEASM_OK;
        }
        if (recipe == 1) {
            switch (n) {
                case 8: return launch_spd_upper<8>(n_elem, seed, elem_offset, ke, stream);
                case 16: return launch_spd_upper<16>(n_elem, seed, elem_offset, ke, stream);
                case 24: return launch_spd_upper<24>(n_elem, seed, elem_offset, ke, stream);
                case 32: return launch_spd_upper<32>(n_elem, seed, elem_offset, ke, stream);
                case 40: return launch_spd_upper<40>(n_elem, seed, elem_offset, ke, stream);
                default: break;
            }
        }
        const unsigned grid = (unsigned)std::min<int64_t>(n_elem, 1 << 20);
        const size_t lds = (size_t)n * (recipe == 0 ? n : n + 1) * 8;
        const int32_t nb = (n + 2) / 3;
        auto kern = recipe == 0 ? k_gen<0> : nb * nb <= 64 ? k_gen<1> : k_gen<2>;
        kern<<<grid, 64, lds, stream>>>(n_elem, n, (uint32_t)seed, (uint32_t)(seed >> 32), elem_offset, ke);
        FEASM_HIP(hipGetLastError());
        return FEASM_OK;
    });
}
