// Sparse matrix-vector product y = G x with the assembled matrix, through
// CSR or through the CRAC runs -- the use of the runs named in the paper's
// conclusions and outlook.
//
// One 64-lane wavefront takes R consecutive rows, whose values are one
// contiguous range.  The range is processed in chunks of kChunk values:
// column indices come from col_idx (CSR) or are expanded from the CRAC
// pairs into LDS (value-parallel, whatever the run lengths), every lane
// forms products values[i] * x[col] for its values
// (coalesced loads of values and col_idx, gathers of x, all issued before
// any is used) into an LDS buffer,
// and lane r then adds row r's products in increasing column order.  Every
// product and every sum is rounded on its own (no fused multiply-add), so
// each y[i] equals a sequential loop over the row bit for bit.
#include <algorithm>

#include "internal.h"

namespace feasm {
namespace {


struct SpmvArgs {
    const int32_t* row_ptr;       // CSR [n_rows+1]
    const int32_t* col_idx;       // CSR [nnz]
    const int32_t* crac_row_ptr;  // CRAC [n_rows+1]
    const int32_t* ca;            // CRAC [n_ca]
    const double* values;
    const double* x;
    double* y;
    int64_t n_rows;
    int32_t rows_per_wave;  // <= 63
};

template <int FMT, int kChunk>
__global__ void __launch_bounds__(64) k_spmv(SpmvArgs A) {
    // slot j of a chunk: first the CRAC column of position j, then (written
    // by the lane that read the column) its product
    union Slot {
        double prod;
        int32_t col;
    };
    __shared__ Slot slot[kChunk];
    auto colb = [&](int32_t j) -> int32_t& { return slot[j].col; };
    const int l = threadIdx.x;
    const int64_t r0 = xcd_block(blockIdx.x, gridDim.x) * A.rows_per_wave;
    const int nr = (int)(A.n_rows - r0 < A.rows_per_wave ? A.n_rows - r0 : A.rows_per_wave);
    // The value range [vs, ve) of the rows comes from scalar loads, so the
    // value loads need not wait for the per-lane row bounds; lane l <= nr
    // holds the start of row r0 + l, needed only for the row sums.
    int32_t vs, ve, rb = 0, pb = 0, pe = 0;
    if (FMT == 0) {
        vs = A.row_ptr[r0];
        ve = A.row_ptr[r0 + nr];
        if (l <= nr) rb = A.row_ptr[r0 + l];
    } else {
        // pb, pe: the rows' pairs, as integer offsets into ca
        pb = A.crac_row_ptr[r0];
        pe = A.crac_row_ptr[r0 + nr];
        vs = A.ca[pb + 1];
        ve = A.ca[pe + 1];
        if (l <= nr) rb = A.crac_row_ptr[r0 + l];
    }
    if (FMT == 1 && l <= nr) rb = A.ca[rb + 1];
    const int32_t re = __shfl_down(rb, 1, 64);
    double s = 0.0;
    for (int32_t c0 = vs; c0 < ve; c0 += kChunk) {
        const int32_t c1 = std::min(c0 + kChunk, ve);
        // CRAC: expand the runs of the chunk into column indices.  Short runs
        // (the wavefront's values per pair at most 16) are written by one
        // lane per pair, longer ones by all lanes, one run at a time.
        const bool short_runs = FMT == 1 && (int64_t)(ve - vs) * 2 <= (int64_t)16 * (pe - pb);
        if (FMT == 1 && short_runs) {
            constexpr int PU = kChunk >= 512 ? kChunk / 256 : 1;
            for (int32_t g = pb; g < pe; g += 128 * PU) {
                int32_t first[PU], ps[PU], pn[PU];
#pragma unroll
                for (int u = 0; u < PU; ++u) {
                    const int32_t q = g + 2 * (l + 64 * u);
                    first[u] = ps[u] = pn[u] = 0;
                    if (q < pe) {
                        first[u] = A.ca[q];
                        ps[u] = A.ca[q + 1];
                        pn[u] = A.ca[q + 3];  // a run ends where the next pair's values begin
                    }
                }
#pragma unroll
                for (int u = 0; u < PU; ++u) {
                    const int32_t a = std::max(ps[u], c0), b = std::min(pn[u], c1);
                    for (int32_t i = a; i < b; ++i) colb(i - c0) = first[u] + (i - ps[u]);
                }
            }
            __syncthreads();
        } else if (FMT == 1) {
            // Long runs: the lanes fill one run at a time, 64 positions per
            // instruction; each group of 64 pairs is loaded one per lane and
            // read back with readlane.
            for (int32_t g = pb; g < pe; g += 128) {
                const int32_t q = g + 2 * l;
                int32_t first = 0, ps = 0, pn = 0;
                if (q < pe) {
                    first = A.ca[q];
                    ps = A.ca[q + 1];
                    pn = A.ca[q + 3];  // a run ends where the next pair's values begin
                }
                const int cnt = std::min(64, (pe - g) >> 1);
                for (int k = 0; k < cnt; ++k) {
                    const int32_t ks = __builtin_amdgcn_readlane(ps, k);
                    const int32_t ke = __builtin_amdgcn_readlane(pn, k);
                    const int32_t kd = __builtin_amdgcn_readlane(first, k) - ks;
                    const int32_t lo = std::max(ks, c0), hi = std::min(ke, c1);
                    for (int32_t i = lo + l; i < hi; i += 64) colb(i - c0) = i + kd;
                }
            }
            __syncthreads();
        }
        // all of a lane's loads of the chunk are issued before any is used:
        // column indices and values, then the x gathers
        constexpr int U = kChunk / 64;
        int32_t cu[U];
        double vu[U], xu[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t i = c0 + l + 64 * u;
            cu[u] = 0;
            vu[u] = 0.0;
            if (i < c1) {
                cu[u] = FMT == 0 ? __builtin_nontemporal_load(A.col_idx + i) : colb(i - c0);
                vu[u] = __builtin_nontemporal_load(A.values + i);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xu[u] = c0 + l + 64 * u < c1 ? A.x[cu[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c0 + l + 64 * u < c1) slot[l + 64 * u].prod = vu[u] * xu[u];
        __syncthreads();
        if (l < nr) {
            const int32_t a = std::max(rb, c0), b = std::min(re, c1);
#pragma unroll 8
            for (int32_t i = a; i < b; ++i) s = s + slot[i - c0].prod;
        }
        __syncthreads();
    }
    if (l < nr) A.y[r0 + l] = s;
}

int spmv_impl(const feasm_pattern* p, int fmt, const double* values, const double* x, double* y,
              hipStream_t s, const char* who) {
    const std::string w(who);
    if (!p) FEASM_FAIL(FEASM_EINVAL, w + ": null handle");
    if (fmt == 0 && !(p->flags & FEASM_BUILD_CSR))
        FEASM_FAIL(FEASM_EINVAL, w + ": handle was built without CSR");
    if (fmt == 1 && !(p->flags & FEASM_BUILD_CRAC))
        FEASM_FAIL(FEASM_EINVAL, w + ": handle was built without CRAC");
    if (p->n_rows == 0) return FEASM_OK;
    if (!values || !x || !y) FEASM_FAIL(FEASM_EINVAL, w + ": null values, x or y");
    const uintptr_t xa = (uintptr_t)x, ya = (uintptr_t)y, nb = (uintptr_t)p->n_rows * 8;
    if (xa < ya + nb && ya < xa + nb) FEASM_FAIL(FEASM_EINVAL, w + ": x and y overlap");
    SpmvArgs A{};
    A.row_ptr = p->row_ptr;
    A.col_idx = p->col_idx;
    A.crac_row_ptr = p->crac_row_ptr;
    A.ca = p->ca;
    A.values = values;
    A.x = x;
    A.y = y;
    A.n_rows = p->n_rows;
    // values per LDS chunk, and as many rows per wavefront as fill one
    const int64_t avg = std::max<int64_t>(1, p->nnz / p->n_rows);
    const int chunk = p->tune_spmv_chunk > 0 ? p->tune_spmv_chunk
                      : fmt == 0 || avg > 96  ? 1024
                                              : 512;
    A.rows_per_wave = (int32_t)std::min<int64_t>(63, std::max<int64_t>(1, chunk / avg));
    const unsigned blocks = (unsigned)ceil_div(p->n_rows, A.rows_per_wave);
#define FEASM_SPMV(CH)                                          \
    if (chunk == CH) {                                          \
        if (fmt == 0)                                           \
            k_spmv<0, CH><<<blocks, 64, 0, s>>>(A);             \
        else                                                    \
            k_spmv<1, CH><<<blocks, 64, 0, s>>>(A);             \
    }
    FEASM_SPMV(256) FEASM_SPMV(512) FEASM_SPMV(1024) FEASM_SPMV(2048)
#undef FEASM_SPMV
    FEASM_HIP(hipGetLastError());
    return FEASM_OK;
}

}  // namespace
}  // namespace feasm

extern "C" int spmv_csr(const feasm_pattern* p, const double* values, const double* x, double* y,
                        hipStream_t stream) {
    return feasm::guarded("spmv_csr", [&]() -> int {
        return feasm::spmv_impl(p, 0, values, x, y, stream, "spmv_csr");
    });
}

extern "C" int spmv_crac(const feasm_pattern* p, const double* values, const double* x, double* y,
                         hipStream_t stream) {
    return feasm::guarded("spmv_crac", [&]() -> int {
        return feasm::spmv_impl(p, 1, values, x, y, stream, "spmv_crac");
    });
}
