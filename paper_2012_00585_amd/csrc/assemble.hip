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
//
// The row-owned strategy (the default) instead gives each node's d DOF rows
// to one wavefront, which walks the node's incident elements in element
// order, adds their row slabs into an LDS accumulator and writes the rows
// once (the static form of the paper's row-exclusive spin_int methods,
// Sections 3.2-3.3; device code in scatter_device.h).  launch_owner picks
// the kernel: the flat single-row kernels (k_owner_pipe) for the element
// shapes they are compiled for, else several rows per wavefront
// (k_owner_rows) or several lane groups per wavefront (k_owner).
#include <algorithm>
#include <climits>
#include <new>

#include "internal.h"
#include "scatter_device.h"

namespace feasm {

struct OffsetCache {
    int fmt = -1;
    bool valid = false;       // filled completely by an element-path assembly
    int32_t* base = nullptr;  // dev [n_elem][k][k]: run offsets inside each row node's row
};

namespace {

using namespace scatter;

template <int FMT, bool ATOMIC, int TPE, int U>
__global__ void __launch_bounds__(kBlock) k_assemble(AsmArgs A) {
    extern __shared__ int32_t lds[];
    elem_tile<FMT, ATOMIC, TPE, U, kBlock>(A, xcd_block(blockIdx.x, gridDim.x), lds);
}

template <int FMT, int G, int J, int B>
__global__ void __launch_bounds__(64) k_owner(OwnArgs A) {
    extern __shared__ double lds_d[];
    constexpr int NG = 64 / G;
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
    owner_tiles<FMT, G, J, B>(A, first, last, lds_d);
}

template <int FMT, int D, int N, int B, int MODE>
__global__ void __launch_bounds__(64) k_owner_pipe(OwnArgs A) {
    extern __shared__ double lds_d[];
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    owner_pipe_row<FMT, D, N, B, MODE>(A, A.node_list ? A.node_list[blk] : blk, lds_d);
}

template <int FMT, int R, int J, int B>
__global__ void __launch_bounds__(64) k_owner_rows(OwnArgs A) {
    extern __shared__ double lds_d[];
    owner_rows_tile<FMT, R, J, B>(A, xcd_block(blockIdx.x, gridDim.x), lds_d);
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
        const int jj = j <= 1 ? 1 : j <= 2 ? 2 : j <= 4 ? 4 : j <= 8 ? 8 : j <= 16 ? 16 : 32;
        const int b = jj <= 2 ? 8 : jj == 4 ? 4 : jj == 8 ? 2 : 1;
        const int64_t idx = fmt == kMap ? 0
                            : fmt == kCSR ? (int64_t)p->d * p->max_deg : 2 * (int64_t)p->max_deg + 2;
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
    A.idx_ints = FMT == kMap ? 0 : FMT == kCSR ? p->d * p->max_deg : 2 * p->max_deg + 2;
    A.acc_doubles = p->d * p->d * p->max_deg;
    A.group_bytes = sh.group_bytes;
    // Flat batches: one node row per wavefront, B entries per batch, for the
    // element shapes they are compiled for: 8-node hexes and 10-node tets
    // with 3 DOFs per node (every mode), and, for rows of at most B entries,
    // Q3/Q4 quads with 4 DOFs and Q1 quads with 4 to 8.  (High-order quads
    // with 1 DOF, whose rows mostly have one entry, are faster with several
    // rows per wavefront.)  By default (setting 0) they are used wherever
    // they are compiled, with B = 4 for rows of more than 192 values, else 8
    // where no node has more incident entries, else 16; meshes with heavier
    // nodes run the light rows (at most 8 entries) and the rest as two
    // launches over the handle's node order.
    if (p->tune_owner_flat == 0 && sh.g == 64 && p->node_order && p->max_inc > kLightInc &&
        ((p->d == 3 && p->n == 24) || (p->d == 3 && p->n == 30))) {
        const size_t lds8 = (size_t)A.group_bytes + (size_t)2 * 8 * p->k * 4;
        const size_t lds16 = (size_t)A.group_bytes + (size_t)2 * 16 * p->k * 4;
        const size_t lds24 = (size_t)A.group_bytes + (size_t)2 * 24 * p->k * 4;
        // heavy rows of at most 24 entries (vertex nodes of tet10 meshes)
        // take one batch of 24, with every load issued at once
        const bool one24 = p->max_inc <= 24 && lds24 <= 64 * 1024 && !p->tune_owner_prefetch;
        if (lds16 <= 64 * 1024) {
            const int64_t nl = p->n_light, nh = p->n_nodes - p->n_light;
            OwnArgs L = A, H = A;
            L.node_list = p->node_order;
            H.node_list = p->node_order + nl;
#define FEASM_SPLIT(DD, NN)                                                             \
    if (p->d == DD && p->n == NN) {                                                    \
        if (nl > 0) k_owner_pipe<FMT, DD, NN, 8, 0><<<(unsigned)nl, 64, lds8, s>>>(L);  \
        if (nh > 0) {                                                                  \
            if (one24)                                                                 \
                k_owner_pipe<FMT, DD, NN, 24, 0><<<(unsigned)nh, 64, lds24, s>>>(H);   \
            else if (p->tune_owner_prefetch)                                           \
                k_owner_pipe<FMT, DD, NN, 16, 2><<<(unsigned)nh, 64, lds16, s>>>(H);   \
            else                                                                       \
                k_owner_pipe<FMT, DD, NN, 16, 1><<<(unsigned)nh, 64, lds16, s>>>(H);   \
        }                                                                              \
        FEASM_HIP(hipGetLastError());                                                   \
        return FEASM_OK;                                                                \
    }
            FEASM_SPLIT(3, 24) FEASM_SPLIT(3, 30)
#undef FEASM_SPLIT
        }
    }
    if (p->tune_owner_flat >= 0 && sh.g == 64) {
        const int dn = p->d * p->n;
        const int B = p->tune_owner_flat > 0 ? p->tune_owner_flat
                      : dn > 192             ? 4
                      : p->max_inc <= 8      ? 8
                                             : 16;
        const size_t lds = (size_t)A.group_bytes + (size_t)2 * B * p->k * 4;
        if (lds <= 64 * 1024) {
            // node id order: each XCD takes a contiguous block range, which
            // stays balanced only while light and heavy rows are mixed
            const unsigned blocks = (unsigned)p->n_nodes;
#define FEASM_PIPE(DD, NN, BB)                                                          \
    if (p->d == DD && p->n == NN && B == BB) {                                         \
        if (p->max_inc <= BB)                                                          \
            k_owner_pipe<FMT, DD, NN, BB, 0><<<blocks, 64, lds, s>>>(A);               \
        else if (p->tune_owner_prefetch)                                               \
            k_owner_pipe<FMT, DD, NN, BB, 2><<<blocks, 64, lds, s>>>(A);               \
        else                                                                           \
            k_owner_pipe<FMT, DD, NN, BB, 1><<<blocks, 64, lds, s>>>(A);               \
        FEASM_HIP(hipGetLastError());                                                   \
        return FEASM_OK;                                                                \
    }
#define FEASM_PIPE_ONE(DD, NN, BB)                                                      \
    if (p->d == DD && p->n == NN && B == BB && p->max_inc <= BB) {                     \
        k_owner_pipe<FMT, DD, NN, BB, 0><<<blocks, 64, lds, s>>>(A);                   \
        FEASM_HIP(hipGetLastError());                                                   \
        return FEASM_OK;                                                                \
    }
#define FEASM_PIPE_SHAPE(DD, NN) FEASM_PIPE_ONE(DD, NN, 4) FEASM_PIPE_ONE(DD, NN, 8)
            FEASM_PIPE(3, 24, 8) FEASM_PIPE(3, 24, 16) FEASM_PIPE(3, 30, 8) FEASM_PIPE(3, 30, 16)
            FEASM_PIPE_SHAPE(4, 64) FEASM_PIPE_SHAPE(4, 100) FEASM_PIPE_SHAPE(4, 16)
            FEASM_PIPE_SHAPE(5, 20)
            FEASM_PIPE_SHAPE(6, 24) FEASM_PIPE_SHAPE(7, 28) FEASM_PIPE_SHAPE(8, 32)
#undef FEASM_PIPE_SHAPE
#undef FEASM_PIPE_ONE
#undef FEASM_PIPE
        }
    }
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
        case 6416: return launch_owner_t<FMT, 64, 16, 1>(p, A, s);
        default: return launch_owner_t<FMT, 64, 32, 1>(p, A, s);
    }
}

bool owner_fits(const feasm_pattern* p, int fmt) {
    return (int64_t)p->d * p->n <= 2048 && owner_shape(p, fmt).g != 0;
}

// Records every row-owned lookup (owner_map_node) for one node per block.
template <int FMT>
__global__ void __launch_bounds__(64) k_owner_map(OwnArgs A, int32_t* out) {
    extern __shared__ int32_t sidx[];
    for (int64_t v = blockIdx.x; v < A.n_nodes; v += gridDim.x) owner_map_node<FMT>(A, v, sidx, out);
}

int launch_owner(const feasm_pattern* p, int fmt, const double* ke, double* values, bool accumulate,
                 hipStream_t s, const int32_t* map = nullptr) {
    if ((int64_t)p->d * p->n > 2048)
        FEASM_FAIL(FEASM_ELIMIT, "row-owned assembly supports d * n <= 2048");
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
    A.node_ptr = p->node_ptr;
    A.map = map;
    if (map) return launch_owner_f<kMap>(p, A, s);
    return fmt == kCSR ? launch_owner_f<kCSR>(p, A, s) : launch_owner_f<kCRAC>(p, A, s);
}

// Builds the row-owned lookup record of a handle (same for both formats).
size_t owner_map_lds(const feasm_pattern* p) {
    return sizeof(int32_t) *
           (size_t)std::max<int64_t>((int64_t)p->d * p->max_deg, 2 * (int64_t)p->max_deg + 2);
}

int build_owner_map(feasm_pattern* p, int fmt, hipStream_t s) {
    OwnArgs A{};
    A.conn = p->conn;
    A.k = p->k;
    A.d = p->d;
    A.n = p->n;
    A.inc_ptr = p->inc_ptr;
    A.inc_elem = p->inc_elem;
    A.row_ptr = p->row_ptr;
    A.col_idx = p->col_idx;
    A.crac_row_ptr = p->crac_row_ptr;
    A.ca = p->ca;
    A.n_nodes = p->n_nodes;
    const size_t lds = owner_map_lds(p);
    if (lds > 64 * 1024)
        FEASM_FAIL(FEASM_ELIMIT, "row-owned lookup record: node rows too long for the LDS");
    const unsigned grid = (unsigned)std::min<int64_t>(p->n_nodes, 1 << 20);
    if (fmt == kCSR)
        k_owner_map<kCSR><<<grid, 64, lds, s>>>(A, p->owner_map);
    else
        k_owner_map<kCRAC><<<grid, 64, lds, s>>>(A, p->owner_map);
    FEASM_HIP(hipGetLastError());
    return FEASM_OK;
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
                  const int32_t* cache, int32_t* cache_out, hipStream_t s, const char* who,
                  const int32_t* owner_map = nullptr) {
    if (!p) FEASM_FAIL(FEASM_EINVAL, std::string(who) + ": null handle");
    if (!ke || !values) FEASM_FAIL(FEASM_EINVAL, std::string(who) + ": ke or values is NULL");
    if (fmt == kCSR && !(p->flags & FEASM_BUILD_CSR))
        FEASM_FAIL(FEASM_EINVAL, std::string(who) + ": handle was built without CSR");
    if (fmt == kCRAC && !(p->flags & FEASM_BUILD_CRAC))
        FEASM_FAIL(FEASM_EINVAL, std::string(who) + ": handle was built without CRAC");
    const bool accumulate = (scatter & FEASM_ACCUMULATE) != 0;
    scatter &= ~FEASM_ACCUMULATE;
    if (scatter == FEASM_SCATTER_AUTO) {
        // the handle's tuned choice; row-owned unless its rows do not fit
        scatter = p->tune_strategy;
        if (scatter == FEASM_SCATTER_AUTO || (scatter == FEASM_SCATTER_OWNER && !owner_fits(p, fmt)))
            scatter = owner_fits(p, fmt) ? FEASM_SCATTER_OWNER : FEASM_SCATTER_ATOMIC;
    }
    if (scatter != FEASM_SCATTER_ATOMIC && scatter != FEASM_SCATTER_COLOURED &&
        scatter != FEASM_SCATTER_OWNER && scatter != FEASM_SCATTER_SPIN)
        FEASM_FAIL(FEASM_EINVAL, std::string(who) + ": unknown scatter strategy");
    if (scatter == FEASM_SCATTER_OWNER) {
        // a record built with the pattern replaces the connectivity reads and
        // row searches of every row-owned call
        if (!owner_map && (p->flags & FEASM_BUILD_OWNER_MAP)) owner_map = p->owner_map;
        return launch_owner(p, fmt, ke, values, accumulate, s, owner_map);
    }
    if (scatter == FEASM_SCATTER_SPIN) {
        if (!accumulate) {
            k_zero<<<(unsigned)std::min<int64_t>(ceil_div(p->nnz / 2 + 1, 256), 16384), 256, 0, s>>>(
                values, p->nnz);
            FEASM_HIP(hipGetLastError());
        }
        return launch_spin(p, fmt, ke, values, s);
    }
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
        if (p->n_tiles > 0 && !cache && !cache_out) {
            // tiles: LDS sums per distinct (row, column), one write each;
            // elements of tiles beyond the accumulator one atomic per entry
            const int rc = launch_tiled_atomic(p, fmt, ke, values, accumulate, s);
            if (rc != FEASM_OK || p->n_tile_direct == 0) return rc;
            A.elem_list = p->tile_direct;
            A.count = p->n_tile_direct;
            return launch(fmt, true, A, sh, s);
        }
        A.elem_list = nullptr;
        A.count = p->n_elem;
        return launch(fmt, true, A, sh, s);
    }
    // Elements of one colour share no node, so no two of them touch the same
    // value; an element that lists a node twice touches some values twice
    // itself, and then the adds stay atomic.
    // Element block by element block, the colours in order within a block:
    // consecutive launches then touch the same values rows (set_colour_blocks).
    const int64_t nb = p->colour_blocks;
    for (int64_t b = 0; b < nb; ++b) {
        for (int32_t c = 0; c < p->n_colours; ++c) {
            const int64_t lo = p->colour_block_ptr[(size_t)c * (nb + 1) + b];
            const int64_t hi = p->colour_block_ptr[(size_t)c * (nb + 1) + b + 1];
            if (hi <= lo) continue;
            A.elem_list = p->colour_elems + lo;
            A.count = hi - lo;
            const int rc = launch(fmt, p->has_repeats, A, sh, s);
            if (rc != FEASM_OK) return rc;
        }
    }
    return FEASM_OK;
}

}  // namespace

int assemble_on_stream(const feasm_pattern* p, int fmt, const double* ke, double* values,
                       int scatter, hipStream_t s) {
    return assemble_impl(p, fmt, ke, values, scatter, nullptr, nullptr, s, "assemble_batch");
}

int build_owner_record(feasm_pattern* p, hipStream_t s) {
    const int rc = dev_alloc_n(p->alloc, &p->owner_map, p->n_elem * p->k * p->k, s,
                               "pattern_build (lookup record)");
    if (rc != FEASM_OK) return rc;
    return build_owner_map(p, (p->flags & FEASM_BUILD_CRAC) ? kCRAC : kCSR, s);
}

void release_owner_map(feasm_pattern* p) {
    dev_free(p->alloc, p->owner_map, nullptr);
    p->owner_map = nullptr;
    p->owner_map_valid = false;
}

void release_cache(feasm_pattern* p) {
    if (p->cache) {
        dev_free(p->alloc, p->cache->base, nullptr);
        delete p->cache;
        p->cache = nullptr;
    }
}

}  // namespace feasm

extern "C" int assemble_csr(const feasm_pattern* p, const double* ke, double* values, int scatter,
                            hipStream_t stream) {
    return feasm::guarded("assemble_csr", [&]() -> int {
        return feasm::assemble_impl(p, 0, ke, values, scatter, nullptr, nullptr, stream,
                                    "assemble_csr");
    });
}

extern "C" int assemble_crac(const feasm_pattern* p, const double* ke, double* values, int scatter,
                             hipStream_t stream) {
    return feasm::guarded("assemble_crac", [&]() -> int {
        return feasm::assemble_impl(p, 1, ke, values, scatter, nullptr, nullptr, stream,
                                    "assemble_crac");
    });
}

extern "C" int reassemble_values(feasm_pattern* p, int fmt, const double* ke, double* values,
                                 int scatter, hipStream_t stream) {
    return feasm::guarded("reassemble_values", [&]() -> int {
        using namespace feasm;
        if (!p) FEASM_FAIL(FEASM_EINVAL, "reassemble_values: null handle");
        if (fmt != FEASM_FMT_CSR && fmt != FEASM_FMT_CRAC)
            FEASM_FAIL(FEASM_EINVAL, "reassemble_values: fmt must be FEASM_FMT_CSR or FEASM_FMT_CRAC");
        if (fmt == FEASM_FMT_CSR && !(p->flags & FEASM_BUILD_CSR))
            FEASM_FAIL(FEASM_EINVAL, "reassemble_values: handle was built without CSR");
        if (fmt == FEASM_FMT_CRAC && !(p->flags & FEASM_BUILD_CRAC))
            FEASM_FAIL(FEASM_EINVAL, "reassemble_values: handle was built without CRAC");
        // Both strategy families record their lookups on the first call and read
        // the record afterwards instead of searching: the element-centric ones
        // each element's (row node, run) offsets, the row-owned one the column
        // offset of every element node in every owned row.
        int strategy = scatter & ~FEASM_ACCUMULATE;
        if (strategy == FEASM_SCATTER_AUTO) {
            strategy = p->tune_strategy;
            if (strategy == FEASM_SCATTER_AUTO ||
                (strategy == FEASM_SCATTER_OWNER && !owner_fits(p, fmt)))
                strategy = owner_fits(p, fmt) ? FEASM_SCATTER_OWNER : FEASM_SCATTER_ATOMIC;
            scatter = strategy | (scatter & FEASM_ACCUMULATE);
        }
        if (strategy == FEASM_SCATTER_SPIN)
            return assemble_impl(p, fmt, ke, values, scatter, nullptr, nullptr, stream,
                                 "reassemble_values");
        // the lookup records are created once, by whichever thread comes first
        std::lock_guard<std::mutex> lazy(p->lazy_mu);
        if (strategy == FEASM_SCATTER_OWNER || strategy == FEASM_SCATTER_AUTO) {
            if (!p->owner_map_valid) {
                if (!p->owner_map) {
                    const int rc = dev_alloc_n(p->alloc, &p->owner_map, p->n_elem * p->k * p->k, stream,
                                               "reassemble_values (lookup record)");
                    if (rc != FEASM_OK) return rc;
                }
                const int rc = build_owner_map(p, fmt, stream);
                if (rc != FEASM_OK) return rc;
                // the record is complete before any call, on any stream, may read it
                FEASM_HIP(hipStreamSynchronize(stream));
                p->owner_map_valid = true;
            }
            return assemble_impl(p, fmt, ke, values, scatter, nullptr, nullptr, stream,
                                 "reassemble_values", p->owner_map);
        }
        if (strategy == FEASM_SCATTER_ATOMIC && p->n_tiles > 0)
            // the tiles' lookups are one per distinct node pair: nothing to record
            return assemble_impl(p, fmt, ke, values, scatter, nullptr, nullptr, stream,
                                 "reassemble_values");
        if (p->cache && p->cache->valid && p->cache->fmt == fmt)
            return assemble_impl(p, fmt, ke, values, scatter, p->cache->base, nullptr, stream,
                                 "reassemble_values");
        if (p->cache) {
            // queued calls may still read the old cache
            FEASM_HIP(hipDeviceSynchronize());
            release_cache(p);
        }
        p->cache = new (std::nothrow) OffsetCache();
        if (!p->cache) FEASM_FAIL(FEASM_ENOMEM, "reassemble_values: out of host memory");
        {
            const int rc = dev_alloc_n(p->alloc, &p->cache->base, p->n_elem * p->k * p->k, stream,
                                       "reassemble_values (lookup cache)");
            if (rc != FEASM_OK) {
                release_cache(p);
                return rc;
            }
        }
        p->cache->fmt = fmt;
        const int rc = assemble_impl(p, fmt, ke, values, scatter, nullptr, p->cache->base, stream,
                                     "reassemble_values");
        if (rc != FEASM_OK) {
            release_cache(p);
            return rc;
        }
        // the record is complete before any call, on any stream, may read it
        FEASM_HIP(hipStreamSynchronize(stream));
        p->cache->valid = true;
        return FEASM_OK;
    });
}

extern "C" int pattern_tune(feasm_pattern* p, int key, int64_t value) {
    return feasm::guarded("pattern_tune", [&]() -> int {
        if (!p) FEASM_FAIL(FEASM_EINVAL, "pattern_tune: null handle");
        if (key == FEASM_TUNE_OWNER_BLOCKS_PER_CU) {
            if (value < 0 || value > 64)
                FEASM_FAIL(FEASM_EINVAL, "pattern_tune: owner blocks per CU must be in [0, 64]");
            p->tune_owner_blocks_per_cu = (int32_t)value;
            return FEASM_OK;
        }
        if (key == FEASM_TUNE_COLOUR_BLOCKS) {
            if (value < 0 || value > 256)
                FEASM_FAIL(FEASM_EINVAL, "pattern_tune: colour blocks must be in [0, 256]");
            if (!(p->flags & FEASM_BUILD_COLOUR))
                FEASM_FAIL(FEASM_EINVAL, "pattern_tune: handle was built without FEASM_BUILD_COLOUR");
            return feasm::set_colour_blocks(p, value, nullptr);
        }
        if (key == FEASM_TUNE_TILE_CAP) {
            if (value < 0 || value > 64)
                FEASM_FAIL(FEASM_EINVAL, "pattern_tune: tile cap must be in [0, 64]");
            if (!(p->flags & FEASM_BUILD_TILES))
                FEASM_FAIL(FEASM_EINVAL, "pattern_tune: handle was built without FEASM_BUILD_TILES");
            FEASM_HIP(hipDeviceSynchronize());  // queued calls may still read the tiles
            feasm::release_tiles(p);
            p->tune_tile_cap = (int32_t)value;
            const int rc = feasm::build_tiles(p, nullptr);
            if (rc != FEASM_OK) feasm::release_tiles(p);
            return rc;
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
        if (key == FEASM_TUNE_SPMV_CHUNK) {
            if (value != 0 && value != 256 && value != 512 && value != 1024 && value != 2048)
                FEASM_FAIL(FEASM_EINVAL, "pattern_tune: spmv chunk must be 256, 512, 1024 or 2048");
            p->tune_spmv_chunk = (int32_t)value;
            return FEASM_OK;
        }
        if (key == FEASM_TUNE_SPIN_LIMIT) {
            if (value < -1 || value > ((int64_t)1 << 40))
                FEASM_FAIL(FEASM_EINVAL, "pattern_tune: spin limit must be -1 or in [0, 2^40]");
            p->tune_spin_limit = value;
            return FEASM_OK;
        }
        if (key == FEASM_TUNE_HEX8_PIPE) {
            if (value < -1 || value > 16)
                FEASM_FAIL(FEASM_EINVAL, "pattern_tune: hex8 pipeline must be -1, 0 or 1..16 blocks per CU");
            p->tune_hex8_pipe = (int32_t)value;
            return FEASM_OK;
        }
        if (key == FEASM_TUNE_OWNER_PREFETCH) {
            if (value != 0 && value != 1)
                FEASM_FAIL(FEASM_EINVAL, "pattern_tune: owner prefetch must be 0 or 1");
            p->tune_owner_prefetch = (int32_t)value;
            return FEASM_OK;
        }
        if (key == FEASM_TUNE_OWNER_FLAT) {
            if (value != -1 && value != 0 && value != 4 && value != 8 && value != 16)
                FEASM_FAIL(FEASM_EINVAL,
                           "pattern_tune: flat batch must be -1 (off), 0 (auto), 4, 8 or 16");
            p->tune_owner_flat = (int32_t)value;
            return FEASM_OK;
        }
        if (key == FEASM_TUNE_STRATEGY) {
            if (value < FEASM_SCATTER_AUTO || value > FEASM_SCATTER_OWNER)
                FEASM_FAIL(FEASM_EINVAL, "pattern_tune: unknown strategy");
            if (value == FEASM_SCATTER_COLOURED && !(p->flags & FEASM_BUILD_COLOUR))
                FEASM_FAIL(FEASM_EINVAL, "pattern_tune: coloured strategy needs FEASM_BUILD_COLOUR");
            p->tune_strategy = (int32_t)value;
            return FEASM_OK;
        }
        FEASM_FAIL(FEASM_EINVAL, "pattern_tune: unknown key");
    });
}
