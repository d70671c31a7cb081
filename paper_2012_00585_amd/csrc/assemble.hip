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

// Runs of a row searched linearly up to this count, by bisection above it.
constexpr int32_t kLinearRuns = 8;

// Block search (Section 2.2 listing): the last run of row R whose first
// column is <= c, found by stepping over the row's pairs (linear, as in the
// listing) or, for rows with many runs, by bisection over the run starts.
// The last run of the row is the default.  Returns the offset of c inside
// row R, or -1.
__device__ inline int32_t crac_offset(const int32_t* __restrict__ crp, const int32_t* __restrict__ ca,
                                      int32_t R, int32_t c) {
    const int32_t b = crp[R], e = crp[R + 1];
    if (b == e) return -1;
    const int32_t npairs = (e - b) >> 1;
    int32_t q = b;
    if (npairs <= kLinearRuns) {
        while (q + 2 < e && ca[q + 2] <= c) q += 2;
    } else {
        int32_t lo = 0, hi = npairs - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (ca[b + 2 * mid] <= c)
                lo = mid;
            else
                hi = mid - 1;
        }
        q = b + 2 * lo;
    }
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
    const int32_t* inc_q;  // sorted entries e*k + a
    const int32_t* inc_elem;
    const int32_t* inc_local;
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
    int32_t persistent;   // 1: grid smaller than the tile count, blocks loop
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
        // block search over the row's (first column, value position) pairs:
        // the last run starting at or before col
        if (npairs == 0) return -1;
        int32_t q = 0;
        if (npairs <= kLinearRuns) {
            while (q + 1 < npairs && sidx[2 * q + 2] <= col) ++q;
        } else {
            int32_t lo = 0, hi = npairs - 1;  // answer in [lo, hi]
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (sidx[2 * mid] <= col)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            q = lo;
        }
        const int32_t first = sidx[2 * q], vpos = sidx[2 * q + 1], vend = sidx[2 * q + 3];
        if (col < first || col >= first + (vend - vpos)) return -1;
        return vpos + (col - first) - rs;
    }
}

__device__ inline int32_t wave_max(int32_t x) {
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t y = __shfl_xor(x, o, 64);
        x = x > y ? x : y;
    }
    return x;
}

// Lanes of a group add one batch of element rows into the accumulator with
// LDS FP64 atomic adds.  A wavefront's LDS operations execute in issue order,
// so the adds into one value happen in increasing element order, with no
// barrier between elements; atomicity also covers an element that lists a
// node twice.
template <int FMT, int G, int J, int B>
__global__ void __launch_bounds__(64) k_owner(OwnArgs A) {
    extern __shared__ double lds_d[];
    constexpr int NG = 64 / G;
    constexpr bool WAVE = (G == 64);  // one node row per wavefront: row values are uniform
    const int g = WAVE ? 0 : (int)threadIdx.x / G;
    const int l = WAVE ? (int)threadIdx.x : (int)threadIdx.x % G;
    const int32_t k = A.k, d = A.d, n = A.n, dn = d * n;
    double* acc = reinterpret_cast<double*>(reinterpret_cast<char*>(lds_d) + g * A.group_bytes);
    int32_t* sidx = reinterpret_cast<int32_t*>(acc + A.acc_doubles);
    int32_t* scol = sidx + A.idx_ints;

    // this lane's slab entries j = l + u*G: K row offset c1, column node b, component c
    int jc1[J], jb[J], jc[J];
#pragma unroll
    for (int u = 0; u < J; ++u) {
        const int j = l + u * G;
        const int c1 = j / n, s = j - (j / n) * n;
        jc1[u] = c1;
        jb[u] = s / d;
        jc[u] = s - (s / d) * d;
    }
    // this lane's first lookup slot w = l: batch entry tb0, element node b0
    const int tb0 = l / k, b0 = l - (l / k) * k;
    const int step_tb = G / k, step_b = G - (G / k) * k;

    const int64_t n_tiles = ceil_div(A.n_nodes, NG);
    int64_t first, last;
    if (A.persistent) {
        const int64_t per = ceil_div(n_tiles, gridDim.x);
        first = xcd_block(blockIdx.x, gridDim.x) * per;
        last = first + per < n_tiles ? first + per : n_tiles;
    } else {
        first = xcd_block(blockIdx.x, gridDim.x);
        last = first + 1;
    }
    for (int64_t tile = first; tile < last; ++tile) {
        const int64_t v = tile * NG + g;
        const bool active = v < A.n_nodes;
        int32_t rs = 0, ncols = 0, npairs = 0, L = 0;
        int64_t ib = 0;
        if (active) {
            const int32_t R = d * (int32_t)v;
            ib = A.inc_ptr[v];
            L = (int32_t)(A.inc_ptr[v + 1] - ib);
            if (FMT == kCSR) {
                rs = A.row_ptr[R];
                ncols = A.row_ptr[R + 1] - rs;
            } else {
                const int32_t pb = A.crac_row_ptr[R], pe = A.crac_row_ptr[R + 1];
                npairs = (pe - pb) >> 1;
                rs = npairs > 0 ? A.ca[pb + 1] : 0;
                ncols = npairs > 0 ? A.ca[pe + 1] - rs : 0;
            }
        }
        if (WAVE) {
            ib = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)ib) |
                 ((int64_t)__builtin_amdgcn_readfirstlane((int32_t)(ib >> 32)) << 32);
            L = __builtin_amdgcn_readfirstlane(L);
            rs = __builtin_amdgcn_readfirstlane(rs);
            ncols = __builtin_amdgcn_readfirstlane(ncols);
            npairs = __builtin_amdgcn_readfirstlane(npairs);
        }
        if (active) {
            const int32_t R = d * (int32_t)v;
            if (FMT == kCSR) {
                for (int x = l; x < ncols; x += G) sidx[x] = A.col_idx[rs + x];
            } else if (npairs > 0) {
                const int32_t pb = A.crac_row_ptr[R];
                for (int x = l; x < 2 * npairs + 2; x += G) sidx[x] = A.ca[pb + x];
            }
            for (int x = l; x < d * ncols; x += G) acc[x] = 0.0;
        }
        const int32_t lmax = WAVE ? L : wave_max(L);
        __syncthreads();
        for (int32_t t0 = 0; t0 < lmax; t0 += B) {
            double val[B][J];
            // rows d*a .. d*a+d-1 of each element matrix (contiguous)
#pragma unroll
            for (int tb = 0; tb < B; ++tb) {
                if (active && t0 + tb < L) {
                    const int64_t e = A.inc_elem[ib + t0 + tb];
                    const int64_t a = A.inc_local[ib + t0 + tb];
                    const double* slab = A.ke + e * (int64_t)n * n + a * d * n;
#pragma unroll
                    for (int u = 0; u < J; ++u) {
                        const int j = l + u * G;
                        val[tb][u] = j < dn ? __builtin_nontemporal_load(slab + j) : 0.0;
                    }
                }
            }
            // where each node of the batch's elements sits in row d*v
            if (active) {
                int tb = tb0, b = b0;
                for (int w = l; w < B * k; w += G) {
                    if (t0 + tb < L) {
                        const int64_t e = A.inc_elem[ib + t0 + tb];
                        const int32_t col = d * A.conn[e * k + b];
                        scol[w] = row_lookup<FMT>(sidx, ncols, npairs, rs, col);
                    }
                    tb += step_tb;
                    b += step_b;
                    if (b >= k) {
                        b -= k;
                        ++tb;
                    }
                }
            }
            __syncthreads();
            if (active) {
#pragma unroll
                for (int tb = 0; tb < B; ++tb) {
                    if (t0 + tb < L) {
#pragma unroll
                        for (int u = 0; u < J; ++u) {
                            const int j = l + u * G;
                            if (j < dn) {
                                const int32_t off = scol[tb * k + jb[u]];
                                if (off >= 0) atomicAdd(acc + jc1[u] * ncols + off + jc[u], val[tb][u]);
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (active) {
            double* out = A.values + rs;
            if (A.accumulate)
                for (int x = l; x < d * ncols; x += G) out[x] += acc[x];
            else
                for (int x = l; x < d * ncols; x += G) out[x] = acc[x];
        }
        __syncthreads();
    }
}

// One wavefront owns R consecutive node rows.  Their incidence entries are
// one contiguous range, so the wavefront loads the element rows of B entries
// at a time across row boundaries, which keeps more independent loads in
// flight per wavefront than one row at a time.  Adds into a row still run in
// its entries' (element) order.
template <int FMT, int R, int J, int B>
__global__ void __launch_bounds__(64) k_owner_rows(OwnArgs A) {
    extern __shared__ double lds_d[];
    const int l = threadIdx.x;
    const int32_t k = A.k, d = A.d, n = A.n, dn = d * n;
    int32_t* scol = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(lds_d) + R * A.group_bytes);

    int jc1[J], jb[J], jc[J];
#pragma unroll
    for (int u = 0; u < J; ++u) {
        const int j = l + u * 64;
        const int c1 = j / n, s = j - (j / n) * n;
        jc1[u] = c1;
        jb[u] = s / d;
        jc[u] = s - (s / d) * d;
    }
    const int tb0 = l / k, b0 = l - (l / k) * k;
    const int step_tb = 64 / k, step_b = 64 - (64 / k) * k;

    const int64_t v0 = xcd_block(blockIdx.x, gridDim.x) * R;
    const int nrows = (int)(A.n_nodes - v0 < R ? A.n_nodes - v0 : R);
    int32_t rs[R], ncols[R], npairs[R];
    int64_t bound[R + 1];  // entry range of row r: [bound[r], bound[r+1])
#pragma unroll
    for (int r = 0; r <= R; ++r) bound[r] = A.inc_ptr[v0 + (r < nrows ? r : nrows)];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        rs[r] = 0;
        ncols[r] = 0;
        npairs[r] = 0;
        if (r < nrows) {
            const int32_t Rw = d * (int32_t)(v0 + r);
            if (FMT == kCSR) {
                rs[r] = A.row_ptr[Rw];
                ncols[r] = A.row_ptr[Rw + 1] - rs[r];
            } else {
                const int32_t pb = A.crac_row_ptr[Rw], pe = A.crac_row_ptr[Rw + 1];
                npairs[r] = (pe - pb) >> 1;
                rs[r] = npairs[r] > 0 ? A.ca[pb + 1] : 0;
                ncols[r] = npairs[r] > 0 ? A.ca[pe + 1] - rs[r] : 0;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double* acc = reinterpret_cast<double*>(reinterpret_cast<char*>(lds_d) + r * A.group_bytes);
        int32_t* sidx = reinterpret_cast<int32_t*>(acc + A.acc_doubles);
        if (r < nrows) {
            if (FMT == kCSR) {
                for (int x = l; x < ncols[r]; x += 64) sidx[x] = A.col_idx[rs[r] + x];
            } else if (npairs[r] > 0) {
                const int32_t pb = A.crac_row_ptr[d * (int32_t)(v0 + r)];
                for (int x = l; x < 2 * npairs[r] + 2; x += 64) sidx[x] = A.ca[pb + x];
            }
            for (int x = l; x < d * ncols[r]; x += 64) acc[x] = 0.0;
        }
    }
    __syncthreads();
    const int64_t T = bound[R] - bound[0];
    for (int64_t t0 = 0; t0 < T; t0 += B) {
        double val[B][J];
#pragma unroll
        for (int tb = 0; tb < B; ++tb) {
            if (t0 + tb < T) {
                const int64_t q = A.inc_q[bound[0] + t0 + tb];
                const double* slab = A.ke + q * dn;  // e*n*n + a*d*n == (e*k + a)*d*n
#pragma unroll
                for (int u = 0; u < J; ++u) {
                    const int j = l + u * 64;
                    val[tb][u] = j < dn ? __builtin_nontemporal_load(slab + j) : 0.0;
                }
            }
        }
        {
            int tb = tb0, b = b0;
            for (int w = l; w < B * k; w += 64) {
                const int64_t t = bound[0] + t0 + tb;
                if (t0 + tb < T) {
                    int r = 0;
#pragma unroll
                    for (int rr = 1; rr < R; ++rr) r += (t >= bound[rr]);
                    const int32_t q = A.inc_q[t];
                    const int32_t col = d * A.conn[(int64_t)(q - q % k) + b];
                    const int32_t* sidx = reinterpret_cast<const int32_t*>(
                        reinterpret_cast<char*>(lds_d) + r * A.group_bytes + A.acc_doubles * 8);
                    int32_t nc = 0, np = 0, rr0 = 0;
#pragma unroll
                    for (int rr = 0; rr < R; ++rr)
                        if (rr == r) {
                            nc = ncols[rr];
                            np = npairs[rr];
                            rr0 = rs[rr];
                        }
                    scol[w] = row_lookup<FMT>(sidx, nc, np, rr0, col);
                }
                tb += step_tb;
                b += step_b;
                if (b >= k) {
                    b -= k;
                    ++tb;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int tb = 0; tb < B; ++tb) {
            if (t0 + tb < T) {
                const int64_t t = bound[0] + t0 + tb;
                int r = 0;
#pragma unroll
                for (int rr = 1; rr < R; ++rr) r += (t >= bound[rr]);
                int32_t nc = 0;
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    if (rr == r) nc = ncols[rr];
                double* acc =
                    reinterpret_cast<double*>(reinterpret_cast<char*>(lds_d) + r * A.group_bytes);
#pragma unroll
                for (int u = 0; u < J; ++u) {
                    const int j = l + u * 64;
                    if (j < dn) {
                        const int32_t off = scol[tb * k + jb[u]];
                        if (off >= 0) atomicAdd(acc + jc1[u] * nc + off + jc[u], val[tb][u]);
                    }
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r < nrows) {
            const double* acc =
                reinterpret_cast<const double*>(reinterpret_cast<char*>(lds_d) + r * A.group_bytes);
            double* out = A.values + rs[r];
            if (A.accumulate)
                for (int x = l; x < d * ncols[r]; x += 64) out[x] += acc[x];
            else
                for (int x = l; x < d * ncols[r]; x += 64) out[x] = acc[x];
        }
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
    const int64_t tiles = ceil_div(p->n_nodes, NG);
    const size_t lds = (size_t)A.group_bytes * NG;
    auto kern = k_owner<FMT, G, J, B>;
    int64_t blocks = tiles;
    A.persistent = 0;
    if (p->tune_owner_blocks_per_cu > 0) {
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int64_t cap = (int64_t)(cus > 0 ? cus : 256) * p->tune_owner_blocks_per_cu;
        if (cap < tiles) {
            blocks = cap;
            A.persistent = 1;
        }
    }
    kern<<<(unsigned)blocks, 64, lds, s>>>(A);
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
    // Default: two node rows per wavefront while a row's accumulator is small
    // enough that occupancy is not bound by LDS.
    int rows = p->tune_owner_rows;
    if (rows == 0) rows = (sh.g == 64 && A.group_bytes <= 3072) ? 2 : 1;
    if (sh.g == 64 && rows > 1 && (sh.j == 1 || sh.j == 2)) {
        const int R = rows;
        const int B = p->tune_owner_batch > 0 ? p->tune_owner_batch : 8;
        const size_t lds = (size_t)A.group_bytes * R + (size_t)B * p->k * 4;
        if (lds <= 64 * 1024) {
            const unsigned blocks = (unsigned)ceil_div(p->n_nodes, R);
#define FEASM_ROWS(RR, JJ, BB)                                                          \
    if (R == RR && sh.j == JJ && B == BB) {                                            \
        k_owner_rows<FMT, RR, JJ, BB><<<blocks, 64, lds, s>>>(A);                      \
        FEASM_HIP(hipGetLastError());                                                   \
        return FEASM_OK;                                                                \
    }
            FEASM_ROWS(2, 1, 8) FEASM_ROWS(2, 1, 16) FEASM_ROWS(2, 2, 8) FEASM_ROWS(2, 2, 16)
            FEASM_ROWS(4, 1, 8) FEASM_ROWS(4, 1, 16) FEASM_ROWS(4, 2, 8) FEASM_ROWS(4, 2, 16)
#undef FEASM_ROWS
        }
    }
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
    A.inc_elem = p->inc_elem;
    A.inc_local = p->inc_local;
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
Shape choose_shape(int32_t n, int32_t tuned) {
    const int64_t n2 = (int64_t)n * n;
    int tpe = tuned;
    if (tpe == 0) tpe = n2 <= 16 ? 16 : n2 <= 64 ? 32 : n2 <= 1024 ? 64 : 256;
    const int64_t u = ceil_div(n2, tpe);
    return {tpe, (int)(u <= 1 ? 1 : u <= 2 ? 2 : u <= 4 ? 4 : u <= 8 ? 8 : 16)};
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
int launch_f(const AsmArgs& A, const Shape& sh, hipStream_t s) {
#define FEASM_CASE(T, UU)                                                        \
    if (sh.tpe == T && sh.u == UU) return launch_t<FMT, ATOMIC, T, UU>(A, s);
    FEASM_CASE(16, 1) FEASM_CASE(16, 2) FEASM_CASE(16, 4) FEASM_CASE(16, 8) FEASM_CASE(16, 16)
    FEASM_CASE(32, 1) FEASM_CASE(32, 2) FEASM_CASE(32, 4) FEASM_CASE(32, 8) FEASM_CASE(32, 16)
    FEASM_CASE(64, 1) FEASM_CASE(64, 2) FEASM_CASE(64, 4) FEASM_CASE(64, 8) FEASM_CASE(64, 16)
    FEASM_CASE(128, 1) FEASM_CASE(128, 2) FEASM_CASE(128, 4) FEASM_CASE(128, 8) FEASM_CASE(128, 16)
    FEASM_CASE(256, 1) FEASM_CASE(256, 2) FEASM_CASE(256, 4) FEASM_CASE(256, 8) FEASM_CASE(256, 16)
#undef FEASM_CASE
    FEASM_FAIL(FEASM_EINVAL, "unsupported element launch shape");
}

int launch(int fmt, bool atomic, const AsmArgs& A, const Shape& sh, hipStream_t s) {
    if (fmt == kCSR)
        return atomic ? launch_f<kCSR, true>(A, sh, s) : launch_f<kCSR, false>(A, sh, s);
    return atomic ? launch_f<kCRAC, true>(A, sh, s) : launch_f<kCRAC, false>(A, sh, s);
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
    const Shape sh = choose_shape(p->n, p->tune_atomic_tpe);
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
        return launch(fmt, true, A, sh, s);
    }
    // Elements of one colour share no node, so no two of them touch the same
    // value; an element that lists a node twice touches some values twice
    // itself, and then the adds stay atomic.
    for (int32_t c = 0; c < p->n_colours; ++c) {
        A.elem_list = p->colour_elems + p->colour_ptr[c];
        A.count = p->colour_ptr[c + 1] - p->colour_ptr[c];
        const int rc = launch(fmt, p->has_repeats, A, sh, s);
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

extern "C" int pattern_tune(feasm_pattern* p, int key, int64_t value) {
    if (!p) FEASM_FAIL(FEASM_EINVAL, "pattern_tune: null handle");
    if (key == FEASM_TUNE_OWNER_BLOCKS_PER_CU) {
        if (value < 0 || value > 64)
            FEASM_FAIL(FEASM_EINVAL, "pattern_tune: owner blocks per CU must be in [0, 64]");
        p->tune_owner_blocks_per_cu = (int32_t)value;
        return FEASM_OK;
    }
    if (key == FEASM_TUNE_THREADS_PER_ELEM) {
        if (value != 0 && value != 16 && value != 32 && value != 64 && value != 128 && value != 256)
            FEASM_FAIL(FEASM_EINVAL, "pattern_tune: threads per element must be 16, 32, 64, 128 or 256");
        if (value != 0 && (int64_t)p->n * p->n > value * 16)
            FEASM_FAIL(FEASM_EINVAL, "pattern_tune: too few threads per element for this element size");
        p->tune_atomic_tpe = (int32_t)value;
        return FEASM_OK;
    }
    if (key == FEASM_TUNE_OWNER_ROWS) {
        if (value != 0 && value != 1 && value != 2 && value != 4)
            FEASM_FAIL(FEASM_EINVAL, "pattern_tune: owner rows per wavefront must be 1, 2 or 4");
        p->tune_owner_rows = (int32_t)value;
        return FEASM_OK;
    }
    if (key == FEASM_TUNE_OWNER_BATCH) {
        if (value != 0 && value != 8 && value != 16)
            FEASM_FAIL(FEASM_EINVAL, "pattern_tune: owner batch must be 8 or 16");
        p->tune_owner_batch = (int32_t)value;
        return FEASM_OK;
    }
    FEASM_FAIL(FEASM_EINVAL, "pattern_tune: unknown key");
}
