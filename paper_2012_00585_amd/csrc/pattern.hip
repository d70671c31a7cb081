// Symbolic phase: CSR and CRAC sparsity structure from element connectivity.
//
// The pattern is the union over elements of the DOF cliques (Section 3
// intro, Fig. 1b).  With node-major DOFs (Section 2.1) every DOF row of a
// node has the same columns, so the work is done once per node and then
// expanded:
//
//   1. node -> incident (element, local node) lists (count, scan, fill)
//   2. per node: gather the nodes of the incident elements into LDS, bitonic
//      sort, unique and run flags by ballot + popcount  -> degree, node runs
//   3. scan degrees and run counts; read nnz once on the host
//   4. per node again: write its sorted unique neighbour list
//   5. expand node rows to DOF rows: CSR row_ptr/col_idx, CRAC pairs
//
// A CRAC run (Section 2.2, Fig. 1d) of DOF row d*v+c is a maximal run of
// consecutive columns; since each neighbour node contributes d consecutive
// columns, DOF runs are exactly the runs of consecutive neighbour node ids.
#include <climits>
#include <cstring>
#include <new>

#include "internal.h"

namespace feasm {

namespace {

struct BuildStatus {
    unsigned long long first_bad;  // first out-of-range conn index, ULLONG_MAX if none
    int32_t big_count;             // nodes whose candidate list overflows the wave path
    int32_t limit_hit;             // a node exceeds the large-node path too
    int32_t repeats;               // some element lists a node twice
    int32_t max_deg;               // largest number of neighbour nodes of a node
    int32_t max_inc;               // largest number of incident (element, local) entries
};

constexpr int kSmallBlock = 64;    // one wavefront per node
constexpr int kSmallCap = 1024;    // candidate entries sorted in LDS by the wave path
constexpr int kBigBlock = 1024;
constexpr int kBigCap = 8192;      // documented limit of candidate entries per node

__global__ void k_count_nodes(const int32_t* __restrict__ conn, int64_t ek, int64_t n_nodes,
                              int32_t* __restrict__ inc_count, BuildStatus* st) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < ek;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = conn[q];
        if (v < 0 || (int64_t)v >= n_nodes)
            atomicMin(&st->first_bad, (unsigned long long)q);
        else
            atomicAdd(&inc_count[v], 1);
    }
}

__global__ void k_check_repeats(const int32_t* __restrict__ conn, int64_t n_elem, int32_t k,
                                BuildStatus* st) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* c = conn + e * k;
        for (int32_t a = 1; a < k; ++a)
            for (int32_t b = 0; b < a; ++b)
                if (c[a] == c[b]) st->repeats = 1;
    }
}

__global__ void k_fill_incidence(const int32_t* __restrict__ conn, int64_t ek,
                                 const int64_t* __restrict__ inc_ptr, int32_t* __restrict__ cursor,
                                 int32_t* __restrict__ inc_q) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < ek;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = conn[q];
        const int32_t slot = atomicAdd(&cursor[v], 1);
        inc_q[inc_ptr[v] + slot] = (int32_t)q;
    }
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T val) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

__device__ inline uint64_t lanes_below() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Ascending bitonic sort of keys[0, M) (M a power of two) by a whole block.
template <int BLOCK>
__device__ inline void block_bitonic_sort(int32_t* keys, int M) {
    const int tid = threadIdx.x;
    for (int size = 2; size <= M; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < (M >> 1); t += BLOCK) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const int32_t x = keys[lo], y = keys[hi];
                if ((x > y) == up) {
                    keys[lo] = y;
                    keys[hi] = x;
                }
            }
            __syncthreads();
        }
    }
}

// Sorts each node's incidence list (entries e*k + a) ascending, so that
// element order is fixed whatever order the atomic fill produced.  Same node
// split as k_node_rows: lists whose candidate count exceeds CAP of the
// wavefront path are done by the large-node path.
template <int BLOCK, int CAP>
__global__ void __launch_bounds__(BLOCK)
    k_sort_incidence(int32_t k, const int64_t* __restrict__ inc_ptr, int32_t* __restrict__ inc_q,
                     int64_t n_nodes, const int32_t* __restrict__ list,
                     const int32_t* __restrict__ list_len) {
    __shared__ int32_t keys[CAP];
    const int64_t count = list ? (int64_t)*list_len : n_nodes;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        const int64_t v = list ? list[i] : i;
        const int64_t b = inc_ptr[v];
        const int64_t L = inc_ptr[v + 1] - b;
        if (L * k > CAP || L < 2) continue;
        int M = 1;
        while (M < L) M <<= 1;
        for (int t = threadIdx.x; t < M; t += BLOCK) keys[t] = t < L ? inc_q[b + t] : INT_MAX;
        __syncthreads();
        block_bitonic_sort<BLOCK>(keys, M);
        for (int t = threadIdx.x; t < L; t += BLOCK) inc_q[b + t] = keys[t];
        __syncthreads();
    }
}

// Splits sorted entries e*k + a into element and local-node arrays.
__global__ void k_split_incidence(int64_t ek, int32_t k, const int32_t* __restrict__ inc,
                                  int32_t* __restrict__ elem, int32_t* __restrict__ local) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ek;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t q = inc[t];
        elem[t] = q / k;
        local[t] = q - (q / k) * k;
    }
}

// Per node v: sorted unique neighbour nodes.  COUNT pass writes degree and
// number of runs; FILL pass writes the list at node_ptr[v].  Nodes are taken
// from `list` (length *list_len) if given, else all of [0, n_nodes).
template <int BLOCK, int CAP, bool FILL>
__global__ void __launch_bounds__(BLOCK)
    k_node_rows(const int32_t* __restrict__ conn, int32_t k, const int64_t* __restrict__ inc_ptr,
                const int32_t* __restrict__ inc_q, int64_t n_nodes, const int32_t* __restrict__ list,
                const int32_t* __restrict__ list_len, int32_t* __restrict__ deg,
                int32_t* __restrict__ nruns, const int64_t* __restrict__ node_ptr,
                int32_t* __restrict__ node_col, int32_t* __restrict__ big_list, BuildStatus* st) {
    constexpr int W = BLOCK / 64;
    __shared__ int32_t keys[CAP];
    __shared__ int32_t wtot[2 * W];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t count = list ? (int64_t)*list_len : n_nodes;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        const int64_t v = list ? list[i] : i;
        const int64_t b = inc_ptr[v];
        const int64_t C = (inc_ptr[v + 1] - b) * k;
        if (C > CAP) {
            if (tid == 0) {
                if (list == nullptr && !FILL) {
                    const int32_t slot = atomicAdd(&st->big_count, 1);
                    big_list[slot] = (int32_t)v;
                } else if (list != nullptr) {
                    atomicExch(&st->limit_hit, 1);
                }
            }
            continue;
        }
        int M = 1;
        while (M < C) M <<= 1;
        for (int t = tid; t < M; t += BLOCK) {
            int32_t key = INT_MAX;
            if (t < C) {
                const int32_t q = inc_q[b + t / k];
                key = conn[(int64_t)(q / k) * k + t % k];
            }
            keys[t] = key;
        }
        __syncthreads();
        block_bitonic_sort<BLOCK>(keys, M);
        // unique entries and run starts, compacted in order
        int64_t n_unique = 0, n_run = 0;
        for (int base = 0; base < C; base += BLOCK) {
            const int t = base + tid;
            bool uq = false, rs = false;
            int32_t key = 0;
            if (t < C) {
                key = keys[t];
                uq = (t == 0) || keys[t - 1] != key;
                rs = (t == 0) || (uq && keys[t - 1] + 1 != key);
            }
            const uint64_t bu = __ballot(uq), br = __ballot(rs);
            if (lane == 0) {
                wtot[w] = __popcll(bu);
                wtot[W + w] = __popcll(br);
            }
            __syncthreads();
            int64_t before = 0, tot_u = 0, tot_r = 0;
            for (int x = 0; x < W; ++x) {
                if (x < w) before += wtot[x];
                tot_u += wtot[x];
                tot_r += wtot[W + x];
            }
            if (FILL && uq)
                node_col[node_ptr[v] + n_unique + before + __popcll(bu & lanes_below())] = key;
            n_unique += tot_u;
            n_run += tot_r;
            __syncthreads();
        }
        if (!FILL && tid == 0) {
            deg[v] = (int32_t)n_unique;
            nruns[v] = (int32_t)n_run;
            atomicMax(&st->max_deg, (int32_t)n_unique);
            atomicMax(&st->max_inc, (int32_t)(C / k));
        }
        __syncthreads();
    }
}

// CSR expansion: row d*v+c has d*deg(v) columns d*u + c2 for the sorted
// neighbours u of v.  One wavefront per node.
__global__ void __launch_bounds__(64)
    k_expand_csr(int64_t n_nodes, int32_t d, const int64_t* __restrict__ node_ptr,
                 const int32_t* __restrict__ node_col, int32_t* __restrict__ row_ptr,
                 int32_t* __restrict__ col_idx) {
    for (int64_t v = blockIdx.x; v < n_nodes; v += gridDim.x) {
        const int64_t nb = node_ptr[v];
        const int64_t deg = node_ptr[v + 1] - nb;
        for (int32_t c = 0; c < d; ++c) {
            const int64_t start = (int64_t)d * d * nb + (int64_t)c * d * deg;
            if (threadIdx.x == 0) row_ptr[(int64_t)d * v + c] = (int32_t)start;
            if (col_idx)
                for (int64_t t = threadIdx.x; t < d * deg; t += 64)
                    col_idx[start + t] = d * node_col[nb + t / d] + (int32_t)(t % d);
        }
    }
}

// CRAC pairs: for each run of consecutive neighbour nodes starting at
// neighbour index j, row d*v+c gets (first column d*u_j, value position
// rowstart + d*j).  Row d*v+c starts at integer 2*(d*runs_before(v) + c*runs(v)).
__global__ void __launch_bounds__(64)
    k_build_crac(int64_t n_nodes, int32_t d, const int64_t* __restrict__ node_ptr,
                 const int32_t* __restrict__ node_col, const int32_t* __restrict__ node_nruns,
                 const int64_t* __restrict__ noderun_ptr, int32_t* __restrict__ crac_row_ptr,
                 int32_t* __restrict__ ca) {
    for (int64_t v = blockIdx.x; v < n_nodes; v += gridDim.x) {
        const int64_t nb = node_ptr[v];
        const int64_t deg = node_ptr[v + 1] - nb;
        const int64_t runs = node_nruns[v];
        const int64_t rb = noderun_ptr[v];
        for (int32_t c = threadIdx.x; c < d; c += 64)
            crac_row_ptr[(int64_t)d * v + c] = (int32_t)(2 * ((int64_t)d * rb + (int64_t)c * runs));
        int64_t seen = 0;
        for (int64_t base = 0; base < deg; base += 64) {
            const int64_t j = base + threadIdx.x;
            const bool start =
                j < deg && (j == 0 || node_col[nb + j] != node_col[nb + j - 1] + 1);
            const uint64_t bal = __ballot(start);
            if (start) {
                const int64_t q = seen + __popcll(bal & lanes_below());
                for (int32_t c = 0; c < d; ++c) {
                    const int64_t at = 2 * ((int64_t)d * rb + (int64_t)c * runs) + 2 * q;
                    ca[at] = d * node_col[nb + j];
                    ca[at + 1] = (int32_t)((int64_t)d * d * nb + (int64_t)c * d * deg + (int64_t)d * j);
                }
            }
            seen += __popcll(bal);
        }
    }
}

// Writes the closing entries: row_ptr[n_rows] = nnz, crac_row_ptr[n_rows] =
// 2B, final CRAC pair (n_cols, nnz).
__global__ void k_close(int64_t n_rows, int64_t nnz, int64_t two_b, int32_t* row_ptr,
                        int32_t* crac_row_ptr, int32_t* ca) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (row_ptr) row_ptr[n_rows] = (int32_t)nnz;
        if (crac_row_ptr) {
            crac_row_ptr[n_rows] = (int32_t)two_b;
            ca[two_b] = (int32_t)n_rows;
            ca[two_b + 1] = (int32_t)nnz;
        }
    }
}

unsigned grid_for(int64_t n, int block, int64_t cap = 65536) {
    int64_t g = ceil_div(n > 0 ? n : 1, block);
    return (unsigned)(g < cap ? g : cap);
}

// Temporary device buffers of one build, released after the stream has
// drained.
struct TempFree {
    Allocator a;
    hipStream_t s;
    std::vector<void*> ptrs;
    TempFree(const Allocator& al, hipStream_t st) : a(al), s(st) {}
    ~TempFree() {
        (void)hipStreamSynchronize(s);
        for (void* q : ptrs) dev_free(a, q, s);
    }
    template <typename T>
    int alloc(T** p, int64_t count) {
        int rc = dev_alloc_n(a, p, count, s, "pattern_build");
        if (rc == FEASM_OK) ptrs.push_back(*p);
        return rc;
    }
};

#define TRY(x)                        \
    do {                              \
        int rc__ = (x);               \
        if (rc__ != FEASM_OK) return rc__; \
    } while (0)

int build(feasm_pattern* p, const int32_t* conn_in, hipStream_t s) {
    const int64_t E = p->n_elem, k = p->k, d = p->d, nn = p->n_nodes;
    const int64_t ek = E * k;
    TempFree tmp(p->alloc, s);

    TRY(dev_alloc_n(p->alloc, &p->conn, ek, s, "pattern_build"));
    FEASM_HIP(hipMemcpyAsync(p->conn, conn_in, sizeof(int32_t) * ek, hipMemcpyDeviceToDevice, s));

    BuildStatus* st;
    TRY(tmp.alloc((char**)&st, sizeof(BuildStatus)));
    BuildStatus st0{ULLONG_MAX, 0, 0, 0, 0, 0};
    FEASM_HIP(hipMemcpyAsync(st, &st0, sizeof(st0), hipMemcpyHostToDevice, s));

    // 1. incidence
    int32_t *inc_count, *cursor;
    TRY(tmp.alloc(&inc_count, nn));
    TRY(tmp.alloc(&cursor, nn));
    k_fill<int32_t><<<grid_for(nn, 256), 256, 0, s>>>(inc_count, nn, 0);
    k_fill<int32_t><<<grid_for(nn, 256), 256, 0, s>>>(cursor, nn, 0);
    k_count_nodes<<<grid_for(ek, 256), 256, 0, s>>>(p->conn, ek, nn, inc_count, st);
    k_check_repeats<<<grid_for(E, 256), 256, 0, s>>>(p->conn, E, (int32_t)k, st);
    FEASM_HIP(hipGetLastError());
    BuildStatus hst;
    FEASM_HIP(hipMemcpyAsync(&hst, st, sizeof(hst), hipMemcpyDeviceToHost, s));
    FEASM_HIP(hipStreamSynchronize(s));
    if (hst.first_bad != ULLONG_MAX) {
        const int64_t q = (int64_t)hst.first_bad;
        FEASM_FAIL(FEASM_ERANGE, "pattern_build: node id out of range at element " +
                                     std::to_string(q / k) + ", local node " +
                                     std::to_string(q % k));
    }
    int64_t* scratch;
    const int64_t scratch_n = scan_scratch_elems(nn + 1);
    TRY(tmp.alloc(&scratch, scratch_n));
    TRY(dev_alloc_n(p->alloc, &p->inc_ptr, nn + 1, s, "pattern_build"));
    // padded so that a row's incidence entries can be read in whole
    // batches of up to kIncPad entries with scalar loads
    TRY(dev_alloc_n(p->alloc, &p->inc_q, ek + kIncPad, s, "pattern_build"));
    FEASM_HIP(hipMemsetAsync(p->inc_q + ek, 0, sizeof(int32_t) * kIncPad, s));
    TRY(exclusive_scan<int32_t>(inc_count, nn, p->inc_ptr, scratch, s));
    k_fill_incidence<<<grid_for(ek, 256), 256, 0, s>>>(p->conn, ek, p->inc_ptr, cursor, p->inc_q);
    FEASM_HIP(hipGetLastError());

    // 2. per-node degree and run count
    int32_t *deg, *big_list;
    TRY(tmp.alloc(&deg, nn));
    TRY(dev_alloc_n(p->alloc, &p->node_nruns, nn, s, "pattern_build"));
    TRY(tmp.alloc(&big_list, nn));
    k_node_rows<kSmallBlock, kSmallCap, false><<<grid_for(nn, 1, 1 << 20), kSmallBlock, 0, s>>>(
        p->conn, (int32_t)k, p->inc_ptr, p->inc_q, nn, nullptr, nullptr, deg, p->node_nruns,
        nullptr, nullptr, big_list, st);
    FEASM_HIP(hipGetLastError());
    k_node_rows<kBigBlock, kBigCap, false><<<256, kBigBlock, 0, s>>>(
        p->conn, (int32_t)k, p->inc_ptr, p->inc_q, nn, big_list, &st->big_count, deg,
        p->node_nruns, nullptr, nullptr, nullptr, st);
    FEASM_HIP(hipGetLastError());

    // 3. offsets; the single read-back of sizes
    TRY(dev_alloc_n(p->alloc, &p->node_ptr, nn + 1, s, "pattern_build"));
    TRY(dev_alloc_n(p->alloc, &p->noderun_ptr, nn + 1, s, "pattern_build"));
    TRY(exclusive_scan<int32_t>(deg, nn, p->node_ptr, scratch, s));
    TRY(exclusive_scan<int32_t>(p->node_nruns, nn, p->noderun_ptr, scratch, s));
    int64_t totals[2];
    FEASM_HIP(hipMemcpyAsync(&totals[0], p->node_ptr + nn, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FEASM_HIP(hipMemcpyAsync(&totals[1], p->noderun_ptr + nn, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FEASM_HIP(hipMemcpyAsync(&hst, st, sizeof(hst), hipMemcpyDeviceToHost, s));
    FEASM_HIP(hipStreamSynchronize(s));
    if (hst.limit_hit)
        FEASM_FAIL(FEASM_ELIMIT, "pattern_build: a node is shared by so many elements that its "
                                 "candidate neighbour list exceeds " +
                                     std::to_string(kBigCap) + " entries");
    p->has_repeats = hst.repeats != 0;
    p->max_deg = hst.max_deg;
    p->max_inc = hst.max_inc;
    p->node_nnz = totals[0];
    p->node_runs = totals[1];
    p->nnz = d * d * p->node_nnz;
    p->n_ca = 2 * d * p->node_runs + 2;
    if (p->nnz > INT32_MAX || p->n_ca > INT32_MAX)
        FEASM_FAIL(FEASM_EOVERFLOW, "pattern_build: nnz = " + std::to_string(p->nnz) +
                                        " or CRAC length = " + std::to_string(p->n_ca) +
                                        " does not fit int32");

    // 4. neighbour lists
    TRY(dev_alloc_n(p->alloc, &p->node_col, p->node_nnz, s, "pattern_build"));
    k_node_rows<kSmallBlock, kSmallCap, true><<<grid_for(nn, 1, 1 << 20), kSmallBlock, 0, s>>>(
        p->conn, (int32_t)k, p->inc_ptr, p->inc_q, nn, nullptr, nullptr, nullptr, nullptr,
        p->node_ptr, p->node_col, nullptr, st);
    FEASM_HIP(hipGetLastError());
    k_node_rows<kBigBlock, kBigCap, true><<<256, kBigBlock, 0, s>>>(
        p->conn, (int32_t)k, p->inc_ptr, p->inc_q, nn, big_list, &st->big_count, nullptr,
        nullptr, p->node_ptr, p->node_col, nullptr, st);
    FEASM_HIP(hipGetLastError());
    k_sort_incidence<kSmallBlock, kSmallCap><<<grid_for(nn, 1, 1 << 20), kSmallBlock, 0, s>>>(
        (int32_t)k, p->inc_ptr, p->inc_q, nn, nullptr, nullptr);
    k_sort_incidence<kBigBlock, kBigCap><<<256, kBigBlock, 0, s>>>(
        (int32_t)k, p->inc_ptr, p->inc_q, nn, big_list, &st->big_count);
    TRY(dev_alloc_n(p->alloc, &p->inc_local, ek, s, "pattern_build"));
    TRY(dev_alloc_n(p->alloc, &p->inc_elem, ek, s, "pattern_build"));
    k_split_incidence<<<grid_for(ek, 256), 256, 0, s>>>(ek, (int32_t)k, p->inc_q, p->inc_elem,
                                                        p->inc_local);
    FEASM_HIP(hipGetLastError());

    // 5. DOF-level arrays
    const bool want_csr = p->flags & FEASM_BUILD_CSR;
    const bool want_crac = p->flags & FEASM_BUILD_CRAC;
    TRY(dev_alloc_n(p->alloc, &p->row_ptr, p->n_rows + 1, s, "pattern_build"));
    if (want_csr) TRY(dev_alloc_n(p->alloc, &p->col_idx, p->nnz, s, "pattern_build"));
    k_expand_csr<<<grid_for(nn, 1, 1 << 20), 64, 0, s>>>(nn, (int32_t)d, p->node_ptr, p->node_col,
                                                         p->row_ptr, p->col_idx);
    FEASM_HIP(hipGetLastError());
    if (want_crac) {
        TRY(dev_alloc_n(p->alloc, &p->crac_row_ptr, p->n_rows + 1, s, "pattern_build"));
        TRY(dev_alloc_n(p->alloc, &p->ca, p->n_ca, s, "pattern_build"));
        k_build_crac<<<grid_for(nn, 1, 1 << 20), 64, 0, s>>>(
            nn, (int32_t)d, p->node_ptr, p->node_col, p->node_nruns, p->noderun_ptr,
            p->crac_row_ptr, p->ca);
        FEASM_HIP(hipGetLastError());
    }
    k_close<<<1, 64, 0, s>>>(p->n_rows, p->nnz, p->n_ca - 2, p->row_ptr, p->crac_row_ptr, p->ca);
    FEASM_HIP(hipGetLastError());

    // 6. node order for the row-owned kernels
    int64_t n_light = nn;
    TRY(build_node_order(p, s, &n_light));

    if (p->flags & FEASM_BUILD_COLOUR) TRY(build_colouring(p, s));
    if (p->flags & FEASM_BUILD_TILES) TRY(build_tiles(p, s));
    if (p->flags & FEASM_BUILD_OWNER_MAP) TRY(build_owner_record(p, s));
    FEASM_HIP(hipStreamSynchronize(s));
    p->owner_map_valid = p->owner_map != nullptr;
    p->n_light = n_light;
    return FEASM_OK;
}

}  // namespace

void release_pattern(feasm_pattern* p) {
    void* arrs[] = {p->conn,    p->node_ptr,     p->node_col, p->node_nruns, p->noderun_ptr,
                    p->inc_ptr, p->inc_q,        p->inc_elem, p->inc_local,
                    p->row_ptr,  p->col_idx,    p->crac_row_ptr,
                    p->ca,      p->colour_elems, p->elem_colour, p->node_order,
                    p->row_locks, p->spin_aborts};
    for (void* a : arrs) dev_free(p->alloc, a, nullptr);
    release_cache(p);
    release_owner_map(p);
    release_tiles(p);
}

}  // namespace feasm

extern "C" int pattern_build(const int32_t* conn, int64_t n_elem, int32_t nodes_per_elem,
                             int32_t dofs_per_node, int64_t n_nodes, uint32_t build_flags,
                             hipStream_t stream, feasm_pattern** out) {
    return feasm::guarded("pattern_build", [&]() -> int {
        using namespace feasm;
        if (!out) FEASM_FAIL(FEASM_EINVAL, "pattern_build: out is NULL");
        *out = nullptr;
        if (!conn) FEASM_FAIL(FEASM_EINVAL, "pattern_build: conn is NULL");
        if (n_elem <= 0 || nodes_per_elem <= 0 || dofs_per_node <= 0 || n_nodes <= 0)
            FEASM_FAIL(FEASM_EINVAL, "pattern_build: n_elem, nodes_per_elem, dofs_per_node and "
                                     "n_nodes must be positive");
        if (build_flags & ~(uint32_t)(FEASM_BUILD_CSR | FEASM_BUILD_CRAC | FEASM_BUILD_COLOUR |
                                      FEASM_BUILD_TILES | FEASM_BUILD_OWNER_MAP))
            FEASM_FAIL(FEASM_EINVAL, "pattern_build: unknown build flag");
        if (!(build_flags & (FEASM_BUILD_CSR | FEASM_BUILD_CRAC)))
            FEASM_FAIL(FEASM_EINVAL, "pattern_build: request FEASM_BUILD_CSR and/or FEASM_BUILD_CRAC");
        if (n_elem * (int64_t)nodes_per_elem > INT32_MAX)
            FEASM_FAIL(FEASM_EOVERFLOW, "pattern_build: n_elem * nodes_per_elem must be < 2^31");
        if ((int64_t)dofs_per_node * n_nodes >= INT32_MAX)
            FEASM_FAIL(FEASM_EOVERFLOW, "pattern_build: dofs_per_node * n_nodes must be < 2^31 - 1");
        if ((int64_t)nodes_per_elem * dofs_per_node > 4096)
            FEASM_FAIL(FEASM_ELIMIT, "pattern_build: element matrices larger than 4096 x 4096 are "
                                     "not supported");
        feasm_pattern* p = new (std::nothrow) feasm_pattern();
        if (!p) FEASM_FAIL(FEASM_ENOMEM, "pattern_build: out of host memory");
        (void)hipGetDevice(&p->device);
        p->alloc = current_allocator();
        p->n_elem = n_elem;
        p->k = nodes_per_elem;
        p->d = dofs_per_node;
        p->n = nodes_per_elem * dofs_per_node;
        p->n_nodes = n_nodes;
        p->n_rows = (int64_t)dofs_per_node * n_nodes;
        p->flags = build_flags;
        const int rc = build(p, conn, stream);
        if (rc != FEASM_OK) {
            (void)hipStreamSynchronize(stream);
            release_pattern(p);
            delete p;
            return rc;
        }
        *out = p;
        return FEASM_OK;
    });
}

extern "C" void pattern_free(feasm_pattern* p) {
    try {
        if (!p) return;
        (void)hipDeviceSynchronize();
        feasm::release_pattern(p);
        delete p;
    } catch (...) {
        // nothing to report: the call has no status
    }
}

extern "C" int pattern_info(const feasm_pattern* p, int64_t* n_rows, int64_t* nnz, int64_t* n_ca,
                            int32_t* n_colours) {
    return feasm::guarded("pattern_info", [&]() -> int {
        if (!p) FEASM_FAIL(FEASM_EINVAL, "pattern_info: null handle");
        if (n_rows) *n_rows = p->n_rows;
        if (nnz) *nnz = p->nnz;
        if (n_ca) *n_ca = (p->flags & FEASM_BUILD_CRAC) ? p->n_ca : 0;
        if (n_colours) *n_colours = p->n_colours;
        return FEASM_OK;
    });
}

extern "C" int pattern_arrays(const feasm_pattern* p, const int32_t** row_ptr,
                              const int32_t** col_idx, const int32_t** crac_row_ptr,
                              const int32_t** col_align) {
    return feasm::guarded("pattern_arrays", [&]() -> int {
        if (!p) FEASM_FAIL(FEASM_EINVAL, "pattern_arrays: null handle");
        const bool csr = p->flags & FEASM_BUILD_CSR;
        if (row_ptr) *row_ptr = csr ? p->row_ptr : nullptr;
        if (col_idx) *col_idx = csr ? p->col_idx : nullptr;
        if (crac_row_ptr) *crac_row_ptr = p->crac_row_ptr;
        if (col_align) *col_align = p->ca;
        return FEASM_OK;
    });
}

extern "C" int pattern_colouring(const feasm_pattern* p, const int64_t** colour_ptr,
                                 const int32_t** colour_elems, const int32_t** element_colour) {
    return feasm::guarded("pattern_colouring", [&]() -> int {
        if (!p) FEASM_FAIL(FEASM_EINVAL, "pattern_colouring: null handle");
        if (!(p->flags & FEASM_BUILD_COLOUR))
            FEASM_FAIL(FEASM_EINVAL, "pattern_colouring: handle was built without FEASM_BUILD_COLOUR");
        if (colour_ptr) *colour_ptr = p->colour_ptr.data();
        if (colour_elems) *colour_elems = p->colour_elems;
        if (element_colour) *element_colour = p->elem_colour;
        return FEASM_OK;
    });
}
