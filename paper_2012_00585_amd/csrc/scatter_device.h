// Device-side scatter routines shared by the single-mesh kernels and the
// batched persistent kernel.
#pragma once

#include "internal.h"

namespace feasm {
namespace scatter {

constexpr int kBlock = 256;

// kMap: the row-owned kernels with their lookups replaced by a record of
// them (value-only re-assembly; positions are the same for both formats).
enum { kCSR = 0, kCRAC = 1, kMap = 2 };

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

// Element-centric scatter of the EPB = BLOCK/TPE elements of logical block
// `blk` (elements blk*EPB .. blk*EPB+EPB-1 of the launch's list).
template <int FMT, bool ATOMIC, int TPE, int U, int BLOCK>
__device__ inline void elem_tile(const AsmArgs& A, int64_t blk, int32_t* lds) {
    constexpr int EPB = BLOCK / TPE;
    const int g = threadIdx.x / TPE, t = threadIdx.x % TPE;
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
    const int64_t* node_ptr;  // kMap: row starts and lengths from the node pattern
    const int32_t* map;       // kMap: per incidence entry t, map[t*k + b] = offset of
                              // element node b's first column in the owned row
    const int32_t* node_list;  // optional: block i owns node node_list[i]
};

// A pointer read from memory (a batch's table of meshes) is generic to the
// compiler, which then accesses it with flat instructions: 64-bit addresses
// in vector registers and waits that also count LDS operations.  Rebuilding
// it from its integer value as a global-address-space pointer gives global
// loads and stores, as for a pointer passed as a kernel argument.
template <class T>
__device__ inline T* global_ptr(T* p) {
    using G = __attribute__((address_space(1))) T*;
    return (T*)(G)(uintptr_t)p;
}

__device__ inline void to_global(OwnArgs& A) {
    A.conn = global_ptr(A.conn);
    A.inc_ptr = global_ptr(A.inc_ptr);
    A.inc_q = global_ptr(A.inc_q);
    A.inc_elem = global_ptr(A.inc_elem);
    A.inc_local = global_ptr(A.inc_local);
    A.row_ptr = global_ptr(A.row_ptr);
    A.col_idx = global_ptr(A.col_idx);
    A.crac_row_ptr = global_ptr(A.crac_row_ptr);
    A.ca = global_ptr(A.ca);
    A.ke = global_ptr(A.ke);
    A.values = global_ptr(A.values);
    A.node_ptr = global_ptr(A.node_ptr);
    A.map = global_ptr(A.map);
    A.node_list = global_ptr(A.node_list);
}

// A load from a pattern array, which no kernel here writes while reading
// it: through the constant address space, a wave-uniform address becomes a
// scalar load even after the kernel's own stores (in a loop over rows the
// compiler cannot tell on its own that those stores miss the pattern).
template <class T>
__device__ inline T ldc(const T* p) {
    using C = const __attribute__((address_space(4))) T*;
    return *(C)(uintptr_t)p;
}

__device__ inline void to_global(AsmArgs& A) {
    A.conn = global_ptr(A.conn);
    A.row_ptr = global_ptr(A.row_ptr);
    A.col_idx = global_ptr(A.col_idx);
    A.crac_row_ptr = global_ptr(A.crac_row_ptr);
    A.ca = global_ptr(A.ca);
    A.ke = global_ptr(A.ke);
    A.values = global_ptr(A.values);
    A.elem_list = global_ptr(A.elem_list);
    A.cache = global_ptr(A.cache);
    A.cache_out = global_ptr(A.cache_out);
}

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
// Row-owned assembly of node-row tiles [first, last) (NG = 64/G node rows
// per tile, G lanes per row) by one 64-lane block.
template <int FMT, int G, int J, int B>
__device__ inline void owner_tiles(const OwnArgs& A, int64_t first, int64_t last, double* lds_d) {
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

    for (int64_t tile = first; tile < last; ++tile) {
        const int64_t v = tile * NG + g;
        const bool active = v < A.n_nodes;
        int32_t rs = 0, ncols = 0, npairs = 0, L = 0;
        int64_t ib = 0;
        if (active) {
            const int32_t R = d * (int32_t)v;
            ib = ldc(A.inc_ptr + v);
            L = (int32_t)(ldc(A.inc_ptr + v + 1) - ib);
            if (FMT == kMap) {
                const int64_t nb = ldc(A.node_ptr + v);
                rs = (int32_t)((int64_t)d * d * nb);
                ncols = (int32_t)(d * (ldc(A.node_ptr + v + 1) - nb));
            } else if (FMT == kCSR) {
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
            if (FMT == kMap) {
            } else if (FMT == kCSR) {
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
                    if (FMT == kMap && t0 + tb < L) {
                        scol[w] = A.map[(ib + t0 + tb) * k + b];
                    } else if (t0 + tb < L) {
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
                for (int x = l; x < d * ncols; x += G) __builtin_nontemporal_store(acc[x], out + x);
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
__device__ inline void owner_rows_tile(const OwnArgs& A, int64_t blk, double* lds_d) {
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

    const int64_t v0 = blk * R;
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
            if (FMT == kMap) {
                const int64_t nb = A.node_ptr[v0 + r];
                rs[r] = (int32_t)((int64_t)d * d * nb);
                ncols[r] = (int32_t)(d * (A.node_ptr[v0 + r + 1] - nb));
            } else if (FMT == kCSR) {
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
            if (FMT == kMap) {
            } else if (FMT == kCSR) {
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
                if (FMT == kMap && t0 + tb < T) {
                    scol[w] = A.map[t * k + b];
                } else if (t0 + tb < T) {
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
                for (int x = l; x < d * ncols[r]; x += 64) __builtin_nontemporal_store(acc[x], out + x);
        }
    }
}

// One wavefront owns one node row and walks its incidence entries in batches
// of B.  The element rows of a batch are read as one flat array: value u of
// lane l is value l + 64u of the batch, so every load instruction is full
// and no register holds padding (V = ceil(B*D*N/64) values per lane).  The
// element shape is fixed at compile time, so the lane indexing reduces to
// constants.  Since D*N >= 64, the lanes of one instruction cover at most two
// consecutive entries, lo = 64u/(D*N) and lo + 1, whose element numbers come
// from scalar loads.  The adds of the two entries are issued as two
// instructions, the lower entry first, so every value still receives its
// contributions in element order.
//
// A batch's index loads (column nodes, or the recorded offsets) are issued
// before its element-row loads, and the first batch's loads before the row's
// own index words are staged, so a wavefront waits for memory about once per
// batch rather than once per dependent load.  The incidence array is padded
// by kIncPad entries, which lets a batch's element numbers be read with
// unconditional scalar loads.

// The lane id, hidden from the optimiser so that per-lane index arithmetic is
// recomputed where it is used instead of being kept live across a loop.
__device__ inline int opaque_lane() {
    int l = (int)threadIdx.x;
    asm volatile("" : "+v"(l));
    return l;
}

template <int FMT, int D, int N, int B>
struct PipeBatch {
    static constexpr int DN = D * N, K = N / D, V = (B * DN + 63) / 64, KB = B * K, W = (KB + 63) / 64;
    double val[V];
    int32_t ix[W];
};

template <int FMT, int D, int N, int B, bool OPAQUE>
__device__ inline void pipe_issue(const OwnArgs& A, int64_t tbeg, int64_t T, int64_t t0,
                                  PipeBatch<FMT, D, N, B>& bt) {
    using P = PipeBatch<FMT, D, N, B>;
    constexpr int DN = P::DN, K = P::K, V = P::V, KB = P::KB, W = P::W;
    const int l = OPAQUE ? opaque_lane() : (int)threadIdx.x;
    int32_t qs[B];
#pragma unroll
    for (int tb = 0; tb < B; ++tb) qs[tb] = ldc(A.inc_q + tbeg + t0 + tb);
    // index loads first: their waits then leave the element rows in flight
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const int w = l + 64 * i, tb = w / K, b = w % K;
        bt.ix[i] = -1;
        if (w < KB && t0 + tb < T) {
            if (FMT == kMap) {
                bt.ix[i] = A.map[(tbeg + t0 + tb) * K + b];
            } else {
                int32_t q = qs[0];
#pragma unroll
                for (int x = 1; x < B; ++x)
                    if (tb == x) q = qs[x];
                bt.ix[i] = A.conn[(int64_t)(q / K) * K + b];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < V; ++u) {
        const int lo = (64 * u) / DN, split = (lo + 1) * DN - 64 * u;
        const int hi = l >= split;
        const int j = l + 64 * u - (lo + hi) * DN;
        const int32_t q = (hi && lo + 1 < B) ? qs[lo + 1 < B ? lo + 1 : lo] : qs[lo];
        bt.val[u] = 0.0;
        if (lo + hi < B && t0 + lo + hi < T)
            bt.val[u] = __builtin_nontemporal_load(A.ke + (int64_t)q * DN + j);
    }
}

template <int FMT, int D, int N, int B, bool OPAQUE>
__device__ inline void pipe_consume(const OwnArgs& A, int64_t T, int64_t t0, int32_t rs, int32_t ncols,
                                    int32_t npairs, const PipeBatch<FMT, D, N, B>& bt, double* acc,
                                    const int32_t* sidx, int32_t* scol) {
    using P = PipeBatch<FMT, D, N, B>;
    constexpr int DN = P::DN, K = P::K, V = P::V, KB = P::KB, W = P::W;
    const int l = OPAQUE ? opaque_lane() : (int)threadIdx.x;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const int w = l + 64 * i, tb = w / K;
        if (w < KB && t0 + tb < T)
            scol[w] = FMT == kMap ? bt.ix[i] : row_lookup<FMT>(sidx, ncols, npairs, rs, D * bt.ix[i]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < V; ++u) {
        const int lo = (64 * u) / DN, split = (lo + 1) * DN - 64 * u;
        if (t0 + lo < T) {
            const int hi = l >= split;
            const int j = l + 64 * u - (lo + hi) * DN;
            const int c1 = j / N, s = j % N, b = s / D, c = s % D;
            const bool valid = lo + hi < B && t0 + lo + hi < T;
            int32_t off = -1;
            if (valid) off = scol[(lo + hi) * K + b];
            double* dst = acc + c1 * ncols + off + c;
            if (valid && off >= 0 && !hi) atomicAdd(dst, bt.val[u]);
            if (split < 64) {
                if (valid && off >= 0 && hi) atomicAdd(dst, bt.val[u]);
            }
        }
    }
    __syncthreads();
}

// MODE 0: every row has at most B entries (one batch, no loop); 1: batches
// one after another; 2: the next batch is issued before the current one is
// added (two batches of registers).  OPQ: per-lane index arithmetic is
// recomputed where it is used rather than hoisted out of the loops and kept
// live (the batch loops, and MODE 1 and 2, would otherwise hold it in
// registers across every row).
template <int FMT, int D, int N, int B, int MODE, bool OPQ = (MODE != 0)>
__device__ inline void owner_pipe_row(const OwnArgs& A, int64_t v, double* lds_d) {
    static_assert(D * N >= 64 && N % D == 0 && B <= kIncPad, "pipelined rows need D*N >= 64");
    using P = PipeBatch<FMT, D, N, B>;
    constexpr int SI = 4;  // index words per lane staged ahead of the first batch
    // the row set-up's lane arithmetic too, in a one-batch row inside a
    // caller's loop (MODE 1 and 2 take more registers that way)
    const int l = (OPQ && MODE == 0) ? opaque_lane() : (int)threadIdx.x;
    double* acc = lds_d;
    int32_t* sidx = reinterpret_cast<int32_t*>(acc + A.acc_doubles);
    int32_t* scol0 = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(lds_d) + A.group_bytes);
    int32_t* scol1 = scol0 + P::KB;

    const int64_t tbeg = ldc(A.inc_ptr + v), T = ldc(A.inc_ptr + v + 1) - tbeg;
    const int32_t Rw = D * (int32_t)v;
    int32_t rs = 0, ncols = 0, npairs = 0, nidx = 0;
    const int32_t* isrc = nullptr;
    if (FMT == kMap) {
        const int64_t nb = ldc(A.node_ptr + v);
        rs = (int32_t)((int64_t)D * D * nb);
        ncols = (int32_t)(D * (ldc(A.node_ptr + v + 1) - nb));
    } else if (FMT == kCSR) {
        rs = ldc(A.row_ptr + Rw);
        ncols = ldc(A.row_ptr + Rw + 1) - rs;
        isrc = A.col_idx + rs;
        nidx = ncols;
    } else {
        const int32_t pb = ldc(A.crac_row_ptr + Rw), pe = ldc(A.crac_row_ptr + Rw + 1);
        npairs = (pe - pb) >> 1;
        rs = npairs > 0 ? ldc(A.ca + pb + 1) : 0;
        ncols = npairs > 0 ? ldc(A.ca + pe + 1) - rs : 0;
        isrc = A.ca + pb;
        nidx = npairs > 0 ? 2 * npairs + 2 : 0;
    }
    // the row's index words: loaded first, stored to LDS once the first
    // batch's loads are in flight
    int32_t sreg[SI];
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        const int x = l + 64 * i;
        sreg[i] = x < nidx ? isrc[x] : 0;
    }
    P b0;
    if (T > 0) pipe_issue<FMT, D, N, B, OPQ>(A, tbeg, T, 0, b0);
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        const int x = l + 64 * i;
        if (x < nidx) sidx[x] = sreg[i];
    }
    for (int x = l + 64 * SI; x < nidx; x += 64) sidx[x] = isrc[x];
    for (int x = l; x < D * ncols; x += 64) acc[x] = 0.0;
    __syncthreads();
    if (MODE == 2) {
        P b1;
        for (int64_t t0 = 0; t0 < T; t0 += 2 * B) {
            if (t0 + B < T) pipe_issue<FMT, D, N, B, OPQ>(A, tbeg, T, t0 + B, b1);
            pipe_consume<FMT, D, N, B, OPQ>(A, T, t0, rs, ncols, npairs, b0, acc, sidx, scol0);
            if (t0 + B >= T) break;
            if (t0 + 2 * B < T) pipe_issue<FMT, D, N, B, OPQ>(A, tbeg, T, t0 + 2 * B, b0);
            pipe_consume<FMT, D, N, B, OPQ>(A, T, t0 + B, rs, ncols, npairs, b1, acc, sidx, scol1);
        }
    } else {
        if (T > 0) pipe_consume<FMT, D, N, B, OPQ>(A, T, 0, rs, ncols, npairs, b0, acc, sidx, scol0);
        if (MODE == 1) {
            for (int64_t t0 = B; t0 < T; t0 += B) {
                pipe_issue<FMT, D, N, B, OPQ>(A, tbeg, T, t0, b0);
                pipe_consume<FMT, D, N, B, OPQ>(A, T, t0, rs, ncols, npairs, b0, acc, sidx, scol0);
            }
        }
    }
    double* out = A.values + rs;
    if (A.accumulate)
        for (int x = l; x < D * ncols; x += 64) out[x] += acc[x];
    else
        for (int x = l; x < D * ncols; x += 64) __builtin_nontemporal_store(acc[x], out + x);
}

// One node row per lane, for one DOF per node and K-node elements (short
// rows: 2-D meshes).  The 64 rows of a wavefront, nodes v0 .. v0 + 63, are
// consecutive, so their values form one contiguous range of the values
// array, and their index words one contiguous range of col_idx (CSR) or
// col_align (CRAC, plus the pair that closes the last row).  Both ranges
// are staged in LDS; each lane adds its incident elements' row entries, in
// element order, into an LDS image of the value range at its own row (no
// other lane touches it), and the wavefront then writes the image with
// coalesced stores.  Layout: acc_doubles doubles of image, then idx_ints
// index words.
template <int FMT, int K, int B>
__device__ inline void owner_lanes(const OwnArgs& A, int64_t v0, double* lds_d) {
    const int l = threadIdx.x;
    const int64_t nn = A.n_nodes;
    const int64_t v = v0 + l;
    const bool active = v < nn;
    const int64_t vend = v0 + 64 < nn ? v0 + 64 : nn;
    double* acc = lds_d;
    int32_t* sidx = reinterpret_cast<int32_t*>(acc + A.acc_doubles);
    // the wavefront's value range [base, end) and index-word range [i0, i1)
    int32_t base, end, i0, i1;
    const int32_t* isrc;
    if (FMT == kCSR) {
        base = ldc(A.row_ptr + v0);
        end = ldc(A.row_ptr + vend);
        i0 = base;
        i1 = end;
        isrc = A.col_idx;
    } else {
        i0 = ldc(A.crac_row_ptr + v0);
        i1 = ldc(A.crac_row_ptr + vend) + 2;
        base = ldc(A.ca + i0 + 1);
        end = ldc(A.ca + i1 - 1);
        isrc = A.ca;
    }
    // this lane's row: value start, length, runs, its index words in LDS
    int32_t rs = 0, ncols = 0, npairs = 0, ioff = 0, L = 0;
    int64_t ib = 0;
    if (active) {
        if (FMT == kCSR) {
            rs = A.row_ptr[v];
            ncols = A.row_ptr[v + 1] - rs;
            ioff = rs - i0;
        } else {
            const int32_t pb = A.crac_row_ptr[v], pe = A.crac_row_ptr[v + 1];
            npairs = (pe - pb) >> 1;
            rs = A.ca[pb + 1];  // an empty row's pb is the next row's first pair
            ncols = A.ca[pe + 1] - rs;
            ioff = pb - i0;
        }
        ib = A.inc_ptr[v];
        L = (int32_t)(A.inc_ptr[v + 1] - ib);
    }
    for (int32_t x = l; x < i1 - i0; x += 64) sidx[x] = isrc[i0 + x];
    for (int32_t x = l; x < end - base; x += 64) acc[x] = 0.0;
    __syncthreads();
    const int32_t* my_idx = sidx + ioff;
    double* my_acc = acc + (rs - base);
    const int32_t lmax = wave_max(L);
    for (int32_t t0 = 0; t0 < lmax; t0 += B) {
        int32_t cn[B][K];
        double kv[B][K];
#pragma unroll
        for (int tb = 0; tb < B; ++tb) {
            if (active && t0 + tb < L) {
                const int64_t e = A.inc_elem[ib + t0 + tb];
                const int64_t a = A.inc_local[ib + t0 + tb];
#pragma unroll
                for (int b = 0; b < K; ++b) cn[tb][b] = A.conn[e * K + b];
#pragma unroll
                for (int b = 0; b < K; ++b)
                    kv[tb][b] = __builtin_nontemporal_load(A.ke + (e * K + a) * K + b);
            }
        }
#pragma unroll
        for (int tb = 0; tb < B; ++tb) {
            if (active && t0 + tb < L) {
#pragma unroll
                for (int b = 0; b < K; ++b) {
                    const int32_t off = row_lookup<FMT>(my_idx, ncols, npairs, rs, cn[tb][b]);
                    if (off >= 0) my_acc[off] += kv[tb][b];
                }
            }
        }
    }
    __syncthreads();
    double* out = A.values + base;
    if (A.accumulate)
        for (int32_t x = l; x < end - base; x += 64) out[x] += acc[x];
    else
        for (int32_t x = l; x < end - base; x += 64) __builtin_nontemporal_store(acc[x], out + x);
}

// LDS bytes of owner_lanes for a mesh with rows of at most max_deg columns.
inline size_t owner_lanes_lds(int fmt, int64_t max_deg) {
    const int64_t idx = fmt == kCSR ? 64 * max_deg : 2 * 64 * max_deg + 2;
    return (size_t)(64 * max_deg * 8 + ((idx * 4 + 7) / 8) * 8);
}

// Records, for every incidence entry t of node v and every element node b,
// the offset of b's first column inside v's rows (the lookups of the
// row-owned kernels, done once for value-only re-assembly).  One 64-lane
// block per node; FMT picks the CSR or CRAC search, as in owner_tiles.
template <int FMT>
__device__ inline void owner_map_node(const OwnArgs& A, int64_t v, int32_t* sidx, int32_t* out) {
    const int l = threadIdx.x;
    const int32_t k = A.k, d = A.d;
    const int32_t R = d * (int32_t)v;
    int32_t rs = 0, ncols = 0, npairs = 0;
    if (FMT == kCSR) {
        rs = A.row_ptr[R];
        ncols = A.row_ptr[R + 1] - rs;
        for (int x = l; x < ncols; x += 64) sidx[x] = A.col_idx[rs + x];
    } else {
        const int32_t pb = A.crac_row_ptr[R], pe = A.crac_row_ptr[R + 1];
        npairs = (pe - pb) >> 1;
        if (npairs > 0) {
            rs = A.ca[pb + 1];
            ncols = A.ca[pe + 1] - rs;
            for (int x = l; x < 2 * npairs + 2; x += 64) sidx[x] = A.ca[pb + x];
        }
    }
    __syncthreads();
    const int64_t ib = A.inc_ptr[v], ie = A.inc_ptr[v + 1];
    for (int64_t w = ib * k + l; w < ie * k; w += 64) {
        const int64_t t = w / k;
        const int32_t b = (int32_t)(w - t * k);
        const int32_t col = d * A.conn[(int64_t)A.inc_elem[t] * k + b];
        out[w] = row_lookup<FMT>(sidx, ncols, npairs, rs, col);
    }
    __syncthreads();
}

}  // namespace scatter
}  // namespace feasm
