// Numeric phase: scatter-add of dense element matrices into CSR / CRAC values.
//
// Section 3 of the paper gives the loop G(D(r), D(c)) += K(r, c) over
// elements, rows and columns, made race-free either with atomic adds or by
// colouring, and vectorised over contiguous runs of the element's DOF array
// (Section 3.3).  Here a group of TPE threads handles one element:
//
//   1. start streaming K_e from HBM (non-temporal loads, U values per thread)
//   2. stage the element's node ids in LDS and split its local DOF order into
//      runs of consecutive global DOFs (the run-length form of Section 2.1)
//   3. one lookup per (row node, run) -- binary search of col_idx (CSR) or the
//      linear block search over column-alignment pairs (CRAC, Section 2.2) --
//      giving the run's offset inside the row; every DOF row of a node has the
//      same columns, so the offset is shared by its d rows
//   4. add every K_e(r, s) at rowstart(r) + offset(row node, run of s) + the
//      position of s inside its run: a hardware FP64 atomic add, or a plain
//      read-modify-write when the launch covers one colour.
#include <algorithm>
#include <climits>
#include <new>

#include "internal.h"

namespace feasm {

struct OffsetCache {
    int fmt = -1;
    int32_t* base = nullptr;  // dev [n_elem][k][k]: run offsets inside each row node's row
};

namespace {

enum { kCSR = 0, kCRAC = 1 };
constexpr int kBlock = 256;

struct AsmArgs {
    const int32_t* conn;
    int32_t k, d, n;
    const int32_t* row_ptr;       // CSR
    const int32_t* col_idx;       // CSR
    const int32_t* crac_row_ptr;  // CRAC
    const int32_t* ca;            // CRAC
    const double* ke;
    double* values;
    const int32_t* elem_list;  // optional: element ids to process
    int64_t count;             // number of elements to process
    int32_t lds_ints;          // LDS ints per element
    const int32_t* cache;      // optional cached offsets [n_elem][k][k]
    int32_t* cache_out;        // optional: write offsets here
};

// Offset of column c inside row R (CSR), or -1.
__device__ inline int32_t csr_offset(const int32_t* __restrict__ row_ptr,
                                     const int32_t* __restrict__ col_idx, int32_t R, int32_t c) {
    const int32_t rb = row_ptr[R];
    int32_t lo = rb, hi = row_ptr[R + 1];
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (col_idx[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < row_ptr[R + 1] && col_idx[lo] == c) ? lo - rb : -1;
}

// Linear block search (Section 2.2 listing): step over the row's pairs while
// the next run starts at or before c; the last run of the row is the
// default.  Returns the offset of c inside row R, or -1.
__device__ inline int32_t crac_offset(const int32_t* __restrict__ crp, const int32_t* __restrict__ ca,
                                      int32_t R, int32_t c) {
    const int32_t b = crp[R], e = crp[R + 1];
    if (b == e) return -1;
    int32_t q = b;
    while (q + 2 < e && ca[q + 2] <= c) q += 2;
    const int32_t first = ca[q], vpos = ca[q + 1], vend = ca[q + 3];
    if (c < first || c >= first + (vend - vpos)) return -1;
    return vpos + (c - first) - ca[b + 1];
}

template <int FMT, bool ATOMIC, int TPE, int U>
__global__ void __launch_bounds__(kBlock) k_assemble(AsmArgs A) {
    extern __shared__ int32_t lds[];
    constexpr int EPB = kBlock / TPE;
    const int g = threadIdx.x / TPE, t = threadIdx.x % TPE;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t slot = blk * EPB + g;
    const bool active = slot < A.count;
    const int64_t e = active ? (A.elem_list ? (int64_t)A.elem_list[slot] : slot) : 0;
    const int32_t k = A.k, d = A.d, n = A.n;
    const int32_t n2 = n * n;

    // LDS: node[k] | noderun[k] | first[k] | rowstart[n] | rowk[n] | colpack[n] | base[k*k]
    int32_t* s_node = lds + g * A.lds_ints;
    int32_t* s_noderun = s_node + k;
    int32_t* s_first = s_noderun + k;
    int32_t* s_rowstart = s_first + k;
    int32_t* s_rowk = s_rowstart + n;
    int32_t* s_colpack = s_rowk + n;
    int32_t* s_base = s_colpack + n;

    // 1. start the element matrix stream
    const double* __restrict__ K = A.ke + e * (int64_t)n2;
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int idx = t + u * TPE;
        v[u] = (active && idx < n2) ? __builtin_nontemporal_load(K + idx) : 0.0;
    }

    // 2. node ids; runs of consecutive node ids in local order (a DOF run is
    //    the d DOFs of each node of a node run)
    if (active)
        for (int a = t; a < k; a += TPE) s_node[a] = A.conn[e * k + a];
    __syncthreads();
    int32_t nruns = 1;
    if (active) {
        for (int a = t; a < k; a += TPE) {
            int32_t run = 0;
            for (int b = 1; b <= a; ++b) run += (s_node[b] != s_node[b - 1] + 1);
            s_noderun[a] = run;
            if (a == 0 || s_node[a] != s_node[a - 1] + 1) s_first[run] = a;
        }
        for (int b = 1; b < k; ++b) nruns += (s_node[b] != s_node[b - 1] + 1);
    }
    __syncthreads();
    if (active) {
        // per local DOF x = a*d + c: start of global row D(x), the row node's
        // slot in the offset table, and (run, position inside the run) of x
        // as a column
        for (int x = t; x < n; x += TPE) {
            const int a = x / d, c = x - a * d;
            const int32_t R = d * s_node[a] + c;
            s_rowstart[x] = (FMT == kCSR) ? A.row_ptr[R] : A.ca[A.crac_row_ptr[R] + 1];
            s_rowk[x] = a * k;
            const int32_t run = s_noderun[a];
            s_colpack[x] = (run << 16) | (x - d * s_first[run]);
        }
        // 3. one lookup per (row node, run)
        if (A.cache) {
            const int32_t* cb = A.cache + e * (int64_t)k * k;
            for (int w = t; w < k * nruns; w += TPE) {
                const int a = w / nruns, j = w - a * nruns;
                s_base[a * k + j] = cb[a * k + j];
            }
        } else {
            for (int w = t; w < k * nruns; w += TPE) {
                const int a = w / nruns, j = w - a * nruns;
                const int32_t R = d * s_node[a];
                const int32_t c = d * s_node[s_first[j]];
                const int32_t off = (FMT == kCSR) ? csr_offset(A.row_ptr, A.col_idx, R, c)
                                                  : crac_offset(A.crac_row_ptr, A.ca, R, c);
                s_base[a * k + j] = off;
                if (A.cache_out) A.cache_out[e * (int64_t)k * k + a * k + j] = off;
            }
        }
    }
    __syncthreads();
    if (!active) return;

    // 4. scatter-add
    int r = t / n, s = t - (t / n) * n;
    const int step_r = TPE / n, step_s = TPE - (TPE / n) * n;
    for (int base = 0; base < n2; base += U * TPE) {
        if (base > 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = base + t + u * TPE;
                v[u] = idx < n2 ? __builtin_nontemporal_load(K + idx) : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + t + u * TPE;
            if (idx < n2) {
                const int32_t cp = s_colpack[s];
                const int32_t off = s_base[s_rowk[r] + (cp >> 16)];
                if (off >= 0) {
                    double* dst = A.values + (s_rowstart[r] + off + (cp & 0xffff));
                    if (ATOMIC)
                        unsafeAtomicAdd(dst, v[u]);
                    else
                        *dst += v[u];
                }
            }
            r += step_r;
            s += step_s;
            if (s >= n) {
                s -= n;
                ++r;
            }
        }
    }
}

__global__ void k_zero(double* __restrict__ p, int64_t n) {
    // 16-byte stores from the first 16-byte aligned element on
    const int64_t head = ((reinterpret_cast<uintptr_t>(p) & 15) != 0 && n > 0) ? 1 : 0;
    const int64_t n2 = (n - head) / 2;
    double2* q = reinterpret_cast<double2*>(p + head);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
         i += (int64_t)gridDim.x * blockDim.x)
        q[i] = make_double2(0.0, 0.0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (head) p[0] = 0.0;
        if ((n - head) & 1) p[n - 1] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Row-owned assembly.  The paper's fastest CPU methods give each global row
// to one thread at a time (a spin lock held in the row pointer, Section 3.2)
// and add whole contiguous slices of K's rows into it (Section 3.3).  On the
// GPU the same exclusivity comes from static ownership instead of a lock: a
// group of G lanes owns node v, i.e. the d DOF rows d*v .. d*v+d-1, whose
// values are one contiguous block.  It walks the incident (element, local
// node a) entries in increasing element order, looks up where each of the
// element's nodes sits in row d*v (binary search of the CSR columns, or the
// linear block search over the CRAC pairs, both staged in LDS), and adds
// rows d*a .. d*a+d-1 of K_e into an LDS accumulator.  The block is written
// once with coalesced stores: no atomics, no reset pass, and every value is
// the sum of its contributions in increasing element order -- the order of
// the sequential listing.
struct OwnArgs {
    const int32_t* conn;
    int32_t k, d, n;
    const int64_t* inc_ptr;
    const int32_t* inc_q;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const int32_t* crac_row_ptr;
    const int32_t* ca;
    const double* ke;
    double* values;
    int64_t n_nodes;
    int32_t acc_doubles;  // per group: d*d*max_deg
    int32_t idx_ints;     // per group: CSR d*max_deg, CRAC 2*max_deg+2
    int32_t group_bytes;  // per group LDS bytes (8-byte multiple)
    int32_t accumulate;
};

template <int FMT>
__device__ inline int32_t row_lookup(const int32_t* sidx, int32_t ncols, int32_t npairs, int32_t rs,
                                     int32_t col) {
    if (FMT == kCSR) {
        int32_t lo = 0, hi = ncols;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (sidx[mid] < col)
                lo = mid + 1;
            else
                hi = mid;
        }
        return (lo < ncols && sidx[lo] == col) ? lo : -1;
    } else {
        if (npairs == 0) return -1;
        int32_t q = 0;
        while (q + 1 < npairs && sidx[2 * q + 2] <= col) ++q;
        const int32_t first = sidx[2 * q], vpos = sidx[2 * q + 1], vend = sidx[2 * q + 3];
        if (col < first || col >= first + (vend - vpos)) return -1;
        return vpos + (col - first) - rs;
    }
}

template <int FMT, int G, int J, int B, bool REPEATS>
__global__ void __launch_bounds__(64) k_owner(OwnArgs A) {
    extern __shared__ double lds_d[];
    __shared__ int32_t s_lmax;
    constexpr int NG = 64 / G;
    const int g = threadIdx.x / G, l = threadIdx.x % G;
    const int64_t v = xcd_block(blockIdx.x, gridDim.x) * NG + g;
    const bool active = v < A.n_nodes;
    const int32_t k = A.k, d = A.d, n = A.n, dn = d * n;
    double* acc = reinterpret_cast<double*>(reinterpret_cast<char*>(lds_d) + g * A.group_bytes);
    int32_t* sidx = reinterpret_cast<int32_t*>(acc + A.acc_doubles);
    int32_t* scol = sidx + A.idx_ints;

    if (threadIdx.x == 0) s_lmax = 0;
    int32_t rs = 0, ncols = 0, npairs = 0;
    int64_t ib = 0, L = 0;
    if (active) {
        const int32_t R = d * (int32_t)v;
        ib = A.inc_ptr[v];
        L = A.inc_ptr[v + 1] - ib;
        if (FMT == kCSR) {
            rs = A.row_ptr[R];
            ncols = A.row_ptr[R + 1] - rs;
            for (int x = l; x < ncols; x += G) sidx[x] = A.col_idx[rs + x];
        } else {
            const int32_t pb = A.crac_row_ptr[R], pe = A.crac_row_ptr[R + 1];
            npairs = (pe - pb) >> 1;
            if (npairs > 0) {
                for (int x = l; x < pe - pb + 2; x += G) sidx[x] = A.ca[pb + x];
                rs = A.ca[pb + 1];
                ncols = A.ca[pe + 1] - rs;
            }
        }
        for (int x = l; x < d * ncols; x += G) acc[x] = 0.0;
    }
    __syncthreads();
    if (active && l == 0) atomicMax(&s_lmax, (int32_t)L);
    // this lane's slab entries j = l + u*G: K row offset c1 and column s
    int jc1[J], jb[J], jc[J];
#pragma unroll
    for (int u = 0; u < J; ++u) {
        const int j = l + u * G;
        const int c1 = j / n, s = j - (j / n) * n;
        jc1[u] = c1;
        jb[u] = s / d;
        jc[u] = s - (s / d) * d;
    }
    __syncthreads();
    const int32_t lmax = s_lmax;
    for (int32_t t0 = 0; t0 < lmax; t0 += B) {
        double val[B][J];
        if (active) {
            // where each node of the batch's elements sits in row d*v
            for (int w = l; w < B * k; w += G) {
                const int tb = w / k, b = w - (w / k) * k;
                if (t0 + tb < L) {
                    const int32_t q = A.inc_q[ib + t0 + tb];
                    const int32_t col = d * A.conn[(int64_t)(q / k) * k + b];
                    scol[w] = row_lookup<FMT>(sidx, ncols, npairs, rs, col);
                }
            }
            // rows d*a .. d*a+d-1 of each element matrix (contiguous)
#pragma unroll
            for (int tb = 0; tb < B; ++tb) {
                if (t0 + tb < L) {
                    const int32_t q = A.inc_q[ib + t0 + tb];
                    const int64_t e = q / k, a = q - e * k;
                    const double* slab = A.ke + e * (int64_t)n * n + a * d * n;
#pragma unroll
                    for (int u = 0; u < J; ++u) {
                        const int j = l + u * G;
                        val[tb][u] = j < dn ? __builtin_nontemporal_load(slab + j) : 0.0;
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int tb = 0; tb < B; ++tb) {
            if (active && t0 + tb < L) {
#pragma unroll
                for (int u = 0; u < J; ++u) {
                    const int j = l + u * G;
                    if (j < dn) {
                        const int32_t off = scol[tb * k + jb[u]];
                        if (off >= 0) {
                            double* dst = acc + jc1[u] * ncols + off + jc[u];
                            if (REPEATS)
                                atomicAdd(dst, val[tb][u]);
                            else
                                *dst += val[tb][u];
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    if (active) {
        double* out = A.values + rs;
        if (A.accumulate)
            for (int x = l; x < d * ncols; x += G) out[x] += acc[x];
        else
            for (int x = l; x < d * ncols; x += G) out[x] = acc[x];
    }
}

struct OwnShape {
    int g, j, b;
    int32_t group_bytes;
};

// Lanes per node row G, slab values per lane J, incidences per batch B; G
// grows (fewer node rows per 64-lane block) until the per-row LDS fits.
// Returns g = 0 if even one row per block does not fit in 64 KiB.
OwnShape owner_shape(const feasm_pattern* p, int fmt) {
    const int dn = p->d * p->n;
    int g = 4;
    while (g < dn && g < 64) g <<= 1;
    for (;; g <<= 1) {
        if (g > 64) return {0, 0, 0, 0};
        const int j = (int)ceil_div(dn, g);
        const int jj = j <= 1 ? 1 : j <= 2 ? 2 : j <= 4 ? 4 : j <= 8 ? 8 : 16;
        const int b = jj <= 2 ? 8 : jj == 4 ? 4 : jj == 8 ? 2 : 1;
        const int64_t idx = (fmt == kCSR) ? (int64_t)p->d * p->max_deg : 2 * (int64_t)p->max_deg + 2;
        const int64_t bytes = (int64_t)p->d * p->d * p->max_deg * 8 + idx * 4 + (int64_t)b * p->k * 4;
        const int64_t gb = ceil_div(bytes, 8) * 8;
        if (gb * (64 / g) <= 64 * 1024) return {g, jj, b, (int32_t)gb};
    }
}

template <int FMT, int G, int J, int B>
int launch_owner_t(const feasm_pattern* p, OwnArgs& A, hipStream_t s) {
    constexpr int NG = 64 / G;
    const int64_t blocks = ceil_div(p->n_nodes, NG);
    const size_t lds = (size_t)A.group_bytes * NG;
    if (p->has_repeats)
        k_owner<FMT, G, J, B, true><<<(unsigned)blocks, 64, lds, s>>>(A);
    else
        k_owner<FMT, G, J, B, false><<<(unsigned)blocks, 64, lds, s>>>(A);
    FEASM_HIP(hipGetLastError());
    return FEASM_OK;
}

template <int FMT>
int launch_owner_f(const feasm_pattern* p, OwnArgs& A, hipStream_t s) {
    const OwnShape sh = owner_shape(p, FMT);
    if (sh.g == 0)
        FEASM_FAIL(FEASM_ELIMIT, "row-owned assembly: node rows too long for the LDS accumulator");
    A.idx_ints = (FMT == kCSR) ? p->d * p->max_deg : 2 * p->max_deg + 2;
    A.acc_doubles = p->d * p->d * p->max_deg;
    A.group_bytes = sh.group_bytes;
    switch (sh.g * 100 + sh.j) {
        case 401: return launch_owner_t<FMT, 4, 1, 8>(p, A, s);
        case 801: return launch_owner_t<FMT, 8, 1, 8>(p, A, s);
        case 1601: return launch_owner_t<FMT, 16, 1, 8>(p, A, s);
        case 3201: return launch_owner_t<FMT, 32, 1, 8>(p, A, s);
        case 6401: return launch_owner_t<FMT, 64, 1, 8>(p, A, s);
        case 6402: return launch_owner_t<FMT, 64, 2, 8>(p, A, s);
        case 6404: return launch_owner_t<FMT, 64, 4, 4>(p, A, s);
        case 6408: return launch_owner_t<FMT, 64, 8, 2>(p, A, s);
        default: return launch_owner_t<FMT, 64, 16, 1>(p, A, s);
    }
}

bool owner_fits(const feasm_pattern* p, int fmt) {
    return (int64_t)p->d * p->n <= 1024 && owner_shape(p, fmt).g != 0;
}

int launch_owner(const feasm_pattern* p, int fmt, const double* ke, double* values, bool accumulate,
                 hipStream_t s) {
    if ((int64_t)p->d * p->n > 1024)
        FEASM_FAIL(FEASM_ELIMIT, "row-owned assembly supports d * n <= 1024");
    OwnArgs A{};
    A.conn = p->conn;
    A.k = p->k;
    A.d = p->d;
    A.n = p->n;
    A.inc_ptr = p->inc_ptr;
    A.inc_q = p->inc_q;
    A.row_ptr = p->row_ptr;
    A.col_idx = p->col_idx;
    A.crac_row_ptr = p->crac_row_ptr;
    A.ca = p->ca;
    A.ke = ke;
    A.values = values;
    A.n_nodes = p->n_nodes;
    A.accumulate = accumulate ? 1 : 0;
    return fmt == kCSR ? launch_owner_f<kCSR>(p, A, s) : launch_owner_f<kCRAC>(p, A, s);
}

// Threads per element and values per thread, by element-matrix size.
struct Shape {
    int tpe, u;
};
Shape choose_shape(int32_t n) {
    const int64_t n2 = (int64_t)n * n;
    if (n2 <= 16) return {16, 1};
    if (n2 <= 64) return {32, 2};
    if (n2 <= 1024) return {64, 16};
    return {256, 16};
}

template <int FMT, bool ATOMIC, int TPE, int U>
int launch_t(const AsmArgs& A, hipStream_t s) {
    constexpr int EPB = kBlock / TPE;
    const int64_t blocks = ceil_div(A.count, EPB);
    if (blocks == 0) return FEASM_OK;
    const size_t lds = sizeof(int32_t) * (size_t)A.lds_ints * EPB;
    k_assemble<FMT, ATOMIC, TPE, U><<<(unsigned)blocks, kBlock, lds, s>>>(A);
    FEASM_HIP(hipGetLastError());
    return FEASM_OK;
}

template <int FMT, bool ATOMIC>
int launch_f(const AsmArgs& A, hipStream_t s) {
    const Shape sh = choose_shape(A.n);
    if (sh.tpe == 16) return launch_t<FMT, ATOMIC, 16, 1>(A, s);
    if (sh.tpe == 32) return launch_t<FMT, ATOMIC, 32, 2>(A, s);
    if (sh.tpe == 64) return launch_t<FMT, ATOMIC, 64, 16>(A, s);
    return launch_t<FMT, ATOMIC, 256, 16>(A, s);
}

int launch(int fmt, bool atomic, const AsmArgs& A, hipStream_t s) {
    if (fmt == kCSR) return atomic ? launch_f<kCSR, true>(A, s) : launch_f<kCSR, false>(A, s);
    return atomic ? launch_f<kCRAC, true>(A, s) : launch_f<kCRAC, false>(A, s);
}

int assemble_impl(const feasm_pattern* p, int fmt, const double* ke, double* values, int scatter,
                  const int32_t* cache, int32_t* cache_out, hipStream_t s, const char* who) {
    if (!p) FEASM_FAIL(FEASM_EINVAL, std::string(who) + ": null handle");
    if (!ke || !values) FEASM_FAIL(FEASM_EINVAL, std::string(who) + ": ke or values is NULL");
    if (fmt == kCSR && !(p->flags & FEASM_BUILD_CSR))
        FEASM_FAIL(FEASM_EINVAL, std::string(who) + ": handle was built without CSR");
    if (fmt == kCRAC && !(p->flags & FEASM_BUILD_CRAC))
        FEASM_FAIL(FEASM_EINVAL, std::string(who) + ": handle was built without CRAC");
    const bool accumulate = (scatter & FEASM_ACCUMULATE) != 0;
    scatter &= ~FEASM_ACCUMULATE;
    if (scatter == FEASM_SCATTER_AUTO)
        scatter = owner_fits(p, fmt) ? FEASM_SCATTER_OWNER : FEASM_SCATTER_ATOMIC;
    if (scatter != FEASM_SCATTER_ATOMIC && scatter != FEASM_SCATTER_COLOURED &&
        scatter != FEASM_SCATTER_OWNER)
        FEASM_FAIL(FEASM_EINVAL, std::string(who) + ": unknown scatter strategy");
    if (scatter == FEASM_SCATTER_OWNER) return launch_owner(p, fmt, ke, values, accumulate, s);
    if (scatter == FEASM_SCATTER_COLOURED && !(p->flags & FEASM_BUILD_COLOUR))
        FEASM_FAIL(FEASM_EINVAL,
                   std::string(who) + ": coloured scatter needs a handle built with colouring");

    AsmArgs A{};
    A.conn = p->conn;
    A.k = p->k;
    A.d = p->d;
    A.n = p->n;
    A.row_ptr = p->row_ptr;
    A.col_idx = p->col_idx;
    A.crac_row_ptr = p->crac_row_ptr;
    A.ca = p->ca;
    A.ke = ke;
    A.values = values;
    A.lds_ints = 3 * p->k + 3 * p->n + p->k * p->k;
    A.cache = cache;
    A.cache_out = cache_out;
    const Shape sh = choose_shape(p->n);
    if ((size_t)A.lds_ints * 4 * (kBlock / sh.tpe) > 64 * 1024)
        FEASM_FAIL(FEASM_ELIMIT, std::string(who) + ": element too large for the LDS layout");

    if (!accumulate) {
        k_zero<<<(unsigned)std::min<int64_t>(ceil_div(p->nnz / 2 + 1, 256), 16384), 256, 0, s>>>(
            values, p->nnz);
        FEASM_HIP(hipGetLastError());
    }
    if (scatter == FEASM_SCATTER_ATOMIC) {
        A.elem_list = nullptr;
        A.count = p->n_elem;
        return launch(fmt, true, A, s);
    }
    // Elements of one colour share no node, so no two of them touch the same
    // value; an element that lists a node twice touches some values twice
    // itself, and then the adds stay atomic.
    for (int32_t c = 0; c < p->n_colours; ++c) {
        A.elem_list = p->colour_elems + p->colour_ptr[c];
        A.count = p->colour_ptr[c + 1] - p->colour_ptr[c];
        const int rc = launch(fmt, p->has_repeats, A, s);
        if (rc != FEASM_OK) return rc;
    }
    return FEASM_OK;
}

}  // namespace

void release_cache(feasm_pattern* p) {
    if (p->cache) {
        if (p->cache->base) (void)hipFree(p->cache->base);
        delete p->cache;
        p->cache = nullptr;
    }
}

}  // namespace feasm

extern "C" int assemble_csr(const feasm_pattern* p, const double* ke, double* values, int scatter,
                            hipStream_t stream) {
    return feasm::assemble_impl(p, 0, ke, values, scatter, nullptr, nullptr, stream,
                                "assemble_csr");
}

extern "C" int assemble_crac(const feasm_pattern* p, const double* ke, double* values, int scatter,
                             hipStream_t stream) {
    return feasm::assemble_impl(p, 1, ke, values, scatter, nullptr, nullptr, stream,
                                "assemble_crac");
}

extern "C" int reassemble_values(feasm_pattern* p, int fmt, const double* ke, double* values,
                                 int scatter, hipStream_t stream) {
    using namespace feasm;
    if (!p) FEASM_FAIL(FEASM_EINVAL, "reassemble_values: null handle");
    if (fmt != FEASM_FMT_CSR && fmt != FEASM_FMT_CRAC)
        FEASM_FAIL(FEASM_EINVAL, "reassemble_values: fmt must be FEASM_FMT_CSR or FEASM_FMT_CRAC");
    // The first call on a format performs the lookups and records them; later
    // calls read the recorded offsets instead of searching.
    if (!p->cache || p->cache->fmt != fmt) {
        release_cache(p);
        p->cache = new (std::nothrow) OffsetCache();
        if (!p->cache) FEASM_FAIL(FEASM_ENOMEM, "reassemble_values: out of host memory");
        const size_t bytes = sizeof(int32_t) * (size_t)p->n_elem * p->k * p->k;
        hipError_t e = hipMalloc((void**)&p->cache->base, bytes);
        if (e != hipSuccess) {
            release_cache(p);
            FEASM_FAIL(FEASM_ENOMEM, "reassemble_values: cannot allocate lookup cache");
        }
        p->cache->fmt = fmt;
        return assemble_impl(p, fmt, ke, values, scatter, nullptr, p->cache->base, stream,
                             "reassemble_values");
    }
    return assemble_impl(p, fmt, ke, values, scatter, p->cache->base, nullptr, stream,
                         "reassemble_values");
}
