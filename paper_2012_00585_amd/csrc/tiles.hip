// Element tiles for the hardware-atomic scatter (Section 3.3, "Parallel
// assembly using atomic addition": every contribution reaches the global
// values array through an atomic add).
//
// The atomic method as listed issues one atomic per element-matrix entry.
// On MI355X each FP64 atomic costs a fabric transaction, and a node pair of
// a structured hexahedral mesh receives up to eight contributions, so the
// scatter is bound by atomic throughput long before HBM bandwidth.  Tiles
// cut the number of atomics without changing what is summed:
//   * a tile is a small set of elements close together in the mesh;
//   * a workgroup adds the element matrices of its tile into an LDS
//     accumulator holding one d x d block per distinct node pair of the
//     tile (LDS atomics, since the tile's elements share pairs);
//   * it then writes each accumulated entry to the global values once: with
//     a plain store when every element that couples the two nodes belongs
//     to the tile (the entry is complete), with one hardware FP64 atomic add
//     otherwise.
// Positions are still found by the format's own search in the numeric
// phase (CSR binary search, CRAC block search), once per distinct node pair
// of a tile instead of once per element row.
//
// Tiles are built in the symbolic phase from the connectivity alone:
//   1. a distance-2 maximal independent set of the element graph (elements
//      are adjacent when they share a node), chosen by fixed hashed
//      priorities in parallel rounds (Luby's scheme on the squared graph);
//   2. each chosen element roots an aggregate of itself and its neighbours
//      (disjoint, the roots being three steps apart); every other element
//      is two steps from a root and joins the aggregate of a neighbour (the
//      smallest root id);
//   3. each aggregate, its elements in increasing id, is cut into tiles of
//      at most `cap` elements;
//   4. per tile, one workgroup sorts the tile's nodes and node pairs in LDS,
//      numbers the distinct pairs, records for every element entry its pair
//      and marks each pair complete or not (its contributions within the
//      tile against all of them, from the node -> element incidence).
// Every step is deterministic.  A tile whose distinct pairs do not fit the
// accumulator leaves its elements to the element-centric atomic kernel.
#include <algorithm>
#include <climits>

#include "internal.h"
#include "scatter_device.h"

namespace feasm {
namespace {

using scatter::kCRAC;
using scatter::kCSR;

constexpr int kPatternThreads = 256;
constexpr int kMaxTileNodes = 1024;    // element nodes of one tile (sort width)
constexpr int kMaxTileEntries = 4096;  // element node pairs of one tile (sort width)
constexpr int kMaxAggregate = 1024;    // elements of one aggregate (sort width)
constexpr int kTileThreads = 1024;     // numeric kernel block (16 waves share one tile)
constexpr int64_t kTileLdsBytes = 160 * 1024;     // numeric kernel LDS per block at most
constexpr int64_t kTileLdsTarget = 52 * 1024;     // default tile size: three blocks per CU

// MurmurHash3's 32-bit finaliser (Appleby): a fixed pseudo-random priority.
__device__ inline uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

// Ordered tuple of an element: state (0 out, 1 undecided, 2 chosen), then a
// 30-bit priority, then the id (unique tuples).
__device__ inline uint64_t mis_tuple(int32_t state, uint32_t e) {
    return ((uint64_t)state << 62) | ((uint64_t)(mix32(e) & 0x3FFFFFFFu) << 32) | e;
}

__global__ void k_mis_tuples(const int32_t* __restrict__ state, int64_t n_elem,
                             uint64_t* __restrict__ t) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x)
        t[e] = mis_tuple(state[e], (uint32_t)e);
}

// out[e] = max of in[] over e and every element sharing a node with e.
__global__ void k_nbr_max(const int32_t* __restrict__ conn, int32_t k, int64_t n_elem,
                          const int64_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc_elem,
                          const uint64_t* __restrict__ in, uint64_t* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint64_t m = in[e];
        for (int32_t a = 0; a < k; ++a) {
            const int32_t v = conn[e * k + a];
            for (int64_t t = inc_ptr[v]; t < inc_ptr[v + 1]; ++t) m = max(m, in[inc_elem[t]]);
        }
        out[e] = m;
    }
}

// An undecided element whose tuple is the largest within two steps is
// chosen; one with a chosen element within two steps drops out.
__global__ void k_mis_decide(int32_t* __restrict__ state, const uint64_t* __restrict__ t0,
                             const uint64_t* __restrict__ t2, int64_t n_elem,
                             int32_t* __restrict__ undecided) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (state[e] != 1) continue;
        if (t2[e] == t0[e])
            state[e] = 2;
        else if ((t2[e] >> 62) == 2)
            state[e] = 0;
        else
            atomicAdd(undecided, 1);
    }
}

// agg[e] = e for a root, the root among e's neighbours otherwise, or -1.
__global__ void k_agg_roots(const int32_t* __restrict__ conn, int32_t k, int64_t n_elem,
                            const int64_t* __restrict__ inc_ptr,
                            const int32_t* __restrict__ inc_elem, const int32_t* __restrict__ state,
                            int32_t* __restrict__ agg) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t r = state[e] == 2 ? (int32_t)e : -1;
        for (int32_t a = 0; a < k && r < 0; ++a) {
            const int32_t v = conn[e * k + a];
            for (int64_t t = inc_ptr[v]; t < inc_ptr[v + 1]; ++t) {
                const int32_t f = inc_elem[t];
                if (state[f] == 2) {
                    r = f;
                    break;
                }
            }
        }
        agg[e] = r;
    }
}

// Elements without an aggregate join the one of a neighbour with the
// smallest root id.
__global__ void k_agg_fill(const int32_t* __restrict__ conn, int32_t k, int64_t n_elem,
                           const int64_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc_elem,
                           const int32_t* __restrict__ agg_in, int32_t* __restrict__ agg_out,
                           int32_t* __restrict__ unassigned) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t r = agg_in[e];
        if (r < 0) {
            int32_t best = INT_MAX;
            for (int32_t a = 0; a < k; ++a) {
                const int32_t v = conn[e * k + a];
                for (int64_t t = inc_ptr[v]; t < inc_ptr[v + 1]; ++t) {
                    const int32_t g = agg_in[inc_elem[t]];
                    if (g >= 0 && g < best) best = g;
                }
            }
            if (best == INT_MAX)
                atomicAdd(unassigned, 1);
            else
                r = best;
        }
        agg_out[e] = r;
    }
}

__global__ void k_root_flags(const int32_t* __restrict__ state, int64_t n_elem,
                             int32_t* __restrict__ flag) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x)
        flag[e] = state[e] == 2 ? 1 : 0;
}

// Aggregate index of each element (the rank of its root) and aggregate sizes.
__global__ void k_agg_count(const int32_t* __restrict__ agg, const int64_t* __restrict__ root_rank,
                            int64_t n_elem, int32_t* __restrict__ gid, int32_t* __restrict__ count,
                            int32_t* __restrict__ max_size) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t g = (int32_t)root_rank[agg[e]];
        gid[e] = g;
        const int32_t c = atomicAdd(count + g, 1) + 1;
        atomicMax(max_size, c);
    }
}

__global__ void k_agg_scatter(const int32_t* __restrict__ gid, int64_t n_elem,
                              const int64_t* __restrict__ agg_ptr, int32_t* __restrict__ cursor,
                              int32_t* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t g = gid[e];
        out[agg_ptr[g] + atomicAdd(cursor + g, 1)] = (int32_t)e;
    }
}

// In-place ascending bitonic sort of keys[0, n2) (n2 a power of two) by the
// whole block.
template <typename T>
__device__ inline void block_bitonic(T* keys, int n2) {
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < (n2 >> 1); i += blockDim.x) {
                const int lo = 2 * stride * (i / stride) + (i % stride);
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const T a = keys[lo], b = keys[hi];
                if ((a > b) == up) {
                    keys[lo] = b;
                    keys[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

__device__ inline int pow2_at_least(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Sorts each aggregate's element list (the scatter left it in arrival order).
__global__ void __launch_bounds__(kPatternThreads)
    k_agg_sort(const int64_t* __restrict__ agg_ptr, int32_t* __restrict__ elems) {
    __shared__ int32_t keys[kMaxAggregate];
    const int64_t g = blockIdx.x;
    const int64_t b = agg_ptr[g];
    const int n = (int)(agg_ptr[g + 1] - b);
    const int n2 = pow2_at_least(n);
    for (int i = threadIdx.x; i < n2; i += blockDim.x) keys[i] = i < n ? elems[b + i] : INT_MAX;
    __syncthreads();
    block_bitonic(keys, n2);
    for (int i = threadIdx.x; i < n; i += blockDim.x) elems[b + i] = keys[i];
}

__global__ void k_sub_count(const int64_t* __restrict__ agg_ptr, int64_t n_agg, int32_t cap,
                            int32_t* __restrict__ n_sub) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_agg;
         g += (int64_t)gridDim.x * blockDim.x)
        n_sub[g] = (int32_t)ceil_div(agg_ptr[g + 1] - agg_ptr[g], cap);
}

__global__ void k_sub_fill(const int64_t* __restrict__ agg_ptr, const int64_t* __restrict__ sub_ptr,
                           int64_t n_agg, int32_t cap, int32_t* __restrict__ tile_ptr) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_agg;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t nt = sub_ptr[g + 1] - sub_ptr[g];
        for (int64_t j = 0; j < nt; ++j) tile_ptr[sub_ptr[g] + j] = (int32_t)(agg_ptr[g] + j * cap);
    }
}

// Entries of node A that are element e, counting repeated local nodes.
__device__ inline int32_t run_at(const int32_t* __restrict__ inc_elem, int64_t t, int64_t end,
                                 int32_t e) {
    int32_t c = 0;
    while (t + c < end && inc_elem[t + c] == e) ++c;
    return c;
}

// Contributions to node pair (A, B) over the whole mesh: the sum over
// elements of (local entries of A) x (local entries of B), from the two
// ascending incidence lists.
__device__ inline int32_t pair_multiplicity(const int64_t* __restrict__ inc_ptr,
                                            const int32_t* __restrict__ inc_elem, int32_t A,
                                            int32_t B) {
    int64_t i = inc_ptr[A], ie = inc_ptr[A + 1], j = inc_ptr[B], je = inc_ptr[B + 1];
    int32_t m = 0;
    while (i < ie && j < je) {
        const int32_t ea = inc_elem[i], eb = inc_elem[j];
        if (ea < eb) {
            ++i;
        } else if (eb < ea) {
            ++j;
        } else {
            const int32_t ca = run_at(inc_elem, i, ie, ea), cb = run_at(inc_elem, j, je, eb);
            m += ca * cb;
            i += ca;
            j += cb;
        }
    }
    return m;
}

struct TileBuild {
    const int32_t* conn;
    const int64_t* inc_ptr;
    const int32_t* inc_elem;
    const int64_t* node_ptr;    // node-level pattern: neighbours of each node
    const int32_t* node_nruns;  // runs of consecutive neighbours of each node
    const int32_t* tile_ptr;  // [n_tiles+1]
    const int32_t* elems;     // tile-ordered element ids
    int32_t k;
    int32_t* tile_meta;    // [n_tiles][4]: distinct pairs, local nodes, staged CSR and CRAC ints
    int32_t* tile_nodes;   // [n_elem*k]
    uint32_t* tile_pairs;  // [n_elem*k*k]
    uint16_t* tile_slot;   // [n_elem*k*k]
    int32_t* maxima;  // [4]: most distinct pairs, local nodes, staged CSR, staged CRAC ints
};

// Marks positions [0, n) with first(i), the block's threads each taking a
// contiguous chunk; part[t] receives the number of marks before thread t's
// chunk.  Returns the total.  Ends with a barrier.
template <typename F>
__device__ inline int32_t block_ranks(int n, int32_t* part, F first) {
    const int per = (n + (int)blockDim.x - 1) / (int)blockDim.x;
    const int beg = (int)threadIdx.x * per, end = min(n, beg + per);
    int32_t c = 0;
    for (int i = beg; i < end; ++i) c += first(i) ? 1 : 0;
    part[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t sum = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) {
            const int32_t v = part[i];
            part[i] = sum;
            sum += v;
        }
        part[blockDim.x] = sum;
    }
    __syncthreads();
    return part[blockDim.x];
}

// Local pattern of one tile (one block per tile).
__global__ void __launch_bounds__(kPatternThreads) k_tile_pattern(TileBuild B) {
    __shared__ int32_t nodes_all[kMaxTileNodes];
    __shared__ int32_t nodes[kMaxTileNodes];
    __shared__ uint64_t keys[kMaxTileEntries];
    __shared__ int32_t part[kPatternThreads + 1];
    const int64_t t = blockIdx.x;
    const int32_t e0 = B.tile_ptr[t], ne = B.tile_ptr[t + 1] - e0;
    const int32_t k = B.k, kk = k * k;
    const int64_t base_k = (int64_t)e0 * k, base_kk = (int64_t)e0 * kk;

    // 1. the tile's nodes, sorted and unique
    const int nn = ne * k, nn2 = pow2_at_least(nn);
    for (int i = threadIdx.x; i < nn2; i += blockDim.x)
        nodes_all[i] = i < nn ? B.conn[(int64_t)B.elems[e0 + i / k] * k + i % k] : INT_MAX;
    __syncthreads();
    block_bitonic(nodes_all, nn2);
    const int32_t L = block_ranks(nn, part, [&](int i) {
        return i == 0 || nodes_all[i] != nodes_all[i - 1];
    });
    {
        const int per = (nn + (int)blockDim.x - 1) / (int)blockDim.x;
        const int beg = (int)threadIdx.x * per, end = min(nn, beg + per);
        int32_t r = part[threadIdx.x];
        for (int i = beg; i < end; ++i)
            if (i == 0 || nodes_all[i] != nodes_all[i - 1]) {
                nodes[r] = nodes_all[i];
                B.tile_nodes[base_k + r] = nodes_all[i];
                ++r;
            }
    }
    __syncthreads();

    // 2. element node pairs as (local a, local b, entry) keys
    const int np = ne * kk, np2 = pow2_at_least(np);
    for (int i = threadIdx.x; i < np2; i += blockDim.x) {
        uint64_t key = ~0ull;
        if (i < np) {
            const int32_t el = i / kk, ab = i % kk;
            const int64_t e = B.elems[e0 + el];
            const int32_t A = B.conn[e * k + ab / k], Bn = B.conn[e * k + ab % k];
            int32_t lo = 0, hi = L - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (nodes[mid] < A) lo = mid + 1; else hi = mid;
            }
            const int32_t la = lo;
            lo = 0;
            hi = L - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (nodes[mid] < Bn) lo = mid + 1; else hi = mid;
            }
            const int32_t lb = lo;
            key = ((uint64_t)la << 43) | ((uint64_t)lb << 22) | (uint64_t)i;
        }
        keys[i] = key;
    }
    __syncthreads();
    block_bitonic(keys, np2);

    // 3. distinct pairs numbered in key order; each entry records its pair
    const int32_t P = block_ranks(np, part, [&](int i) {
        return i == 0 || (keys[i] >> 22) != (keys[i - 1] >> 22);
    });
    const int per = (np + (int)blockDim.x - 1) / (int)blockDim.x;
    const int beg = (int)threadIdx.x * per, end = min(np, beg + per);
    int32_t slot = part[threadIdx.x] - 1;
    for (int i = beg; i < end; ++i) {
        const bool first = i == 0 || (keys[i] >> 22) != (keys[i - 1] >> 22);
        if (first) ++slot;
        const int32_t entry = (int32_t)(keys[i] & 0x3FFFFFu);
        B.tile_slot[base_kk + entry] = (uint16_t)slot;
        if (first) {
            // contributions within the tile against those of the whole mesh
            int32_t m_tile = 0;
            while (i + m_tile < np && (keys[i + m_tile] >> 22) == (keys[i] >> 22)) ++m_tile;
            const int32_t la = (int32_t)(keys[i] >> 43), lb = (int32_t)((keys[i] >> 22) & 0x1FFFFFu);
            const int32_t m_all = pair_multiplicity(B.inc_ptr, B.inc_elem, nodes[la], nodes[lb]);
            B.tile_pairs[base_kk + slot] =
                (uint32_t)la | ((uint32_t)lb << 11) | (m_tile == m_all ? 0x80000000u : 0u);
        }
    }
    // 4. index data the numeric kernel stages per local node: CSR, the
    //    node's columns (one per neighbour node); CRAC, two ints per run
    __shared__ int32_t stage_sum[2];
    if (threadIdx.x == 0) stage_sum[0] = stage_sum[1] = 0;
    __syncthreads();
    int32_t s_csr = 0, s_crac = 0;
    for (int la = threadIdx.x; la < L; la += blockDim.x) {
        const int32_t v = nodes[la];
        s_csr += (int32_t)(B.node_ptr[v + 1] - B.node_ptr[v]);
        s_crac += 2 * B.node_nruns[v];
    }
    atomicAdd(&stage_sum[0], s_csr);
    atomicAdd(&stage_sum[1], s_crac);
    __syncthreads();
    if (threadIdx.x == 0) {
        B.tile_meta[4 * t] = P;
        B.tile_meta[4 * t + 1] = L;
        B.tile_meta[4 * t + 2] = stage_sum[0];
        B.tile_meta[4 * t + 3] = stage_sum[1];
        atomicMax(B.maxima, P);
        atomicMax(B.maxima + 1, L);
        atomicMax(B.maxima + 2, stage_sum[0]);
        atomicMax(B.maxima + 3, stage_sum[1]);
    }
}

// Tiles too large for the accumulator: flag their elements.
__global__ void k_direct_flags(const int32_t* __restrict__ tile_ptr, const int32_t* __restrict__ meta,
                               int64_t n_tiles, int32_t max_p, int32_t* __restrict__ flag) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t f = meta[4 * t] > max_p ? 1 : 0;
        for (int32_t i = tile_ptr[t]; i < tile_ptr[t + 1]; ++i) flag[i] = f;
    }
}

__global__ void k_direct_fill(const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
                              const int32_t* __restrict__ elems, int64_t n_elem,
                              int32_t* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_elem;
         i += (int64_t)gridDim.x * blockDim.x)
        if (flag[i]) out[pos[i]] = elems[i];
}

__global__ void k_fill(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}


// ---------------------------------------------------------------------------
// Numeric phase: one workgroup per tile.

struct TileArgs {
    const int32_t* tile_ptr;
    const int32_t* elems;
    const int32_t* meta;
    const int32_t* nodes;
    const uint32_t* pairs;
    const uint16_t* slot;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const int32_t* crac_row_ptr;
    const int32_t* ca;
    const double* ke;
    double* values;
    int64_t n_tiles;
    int32_t k, d, n;
    int32_t max_pairs;  // accumulator capacity; tiles with more pairs are skipped
    int32_t cap;        // elements per tile at most
    int32_t max_nodes;  // local nodes per tile at most
    int32_t max_stage;  // staged index entries per tile at most (this format)
};

// LDS layout of a tile, in 4-byte words after the accumulator:
//   acc[max_pairs*d*d] doubles | pos[max_pairs] | len[max_pairs] (sign bit:
//   complete) | elem[cap] | row start, row length, staged count, staged
//   source [4*max_nodes], staged offset, first pair [2*(max_nodes + 1)] |
//   stage[max_stage] |
//   slot[cap*k*k] (uint16)
size_t tile_lds_bytes(int32_t max_pairs, int32_t d, int32_t cap, int32_t k, int32_t max_nodes,
                      int32_t max_stage) {
    return (size_t)max_pairs * d * d * 8 +
           4 * ((size_t)2 * max_pairs + cap + 6 * (size_t)max_nodes + 2 + max_stage) +
           2 * ((size_t)cap * k * k + 1);
}

// Element shape known at compile time (K, D > 0) or read from the arguments.
template <int K, int D>
struct Shape {
    int32_t k, d;
    __device__ explicit Shape(const TileArgs& A) : k(K > 0 ? K : A.k), d(D > 0 ? D : A.d) {}
};

template <int FMT, bool ACCUM, int K, int D>
__global__ void __launch_bounds__(kTileThreads) k_tile_scatter(TileArgs A) {
    extern __shared__ double lds_acc[];
    const int64_t t = xcd_block(blockIdx.x, gridDim.x);
    const int32_t P = A.meta[4 * t];
    if (P > A.max_pairs) return;  // its elements go through the element-centric kernel
    const int32_t L = A.meta[4 * t + 1];
    const Shape<K, D> sh(A);
    const int32_t k = sh.k, d = sh.d, n = k * d, dd = d * d, kk = k * k, n2 = n * n;
    const int32_t e0 = A.tile_ptr[t], ne = A.tile_ptr[t + 1] - e0;
    double* acc = lds_acc;
    int32_t* pos = reinterpret_cast<int32_t*>(acc + (size_t)A.max_pairs * dd);
    int32_t* len = pos + A.max_pairs;
    int32_t* elem = len + A.max_pairs;
    int32_t* r_start = elem + A.cap;
    int32_t* r_len = r_start + A.max_nodes;
    int32_t* r_cnt = r_len + A.max_nodes;
    int32_t* r_src = r_cnt + A.max_nodes;
    int32_t* r_off = r_src + A.max_nodes;    // [max_nodes + 1]
    int32_t* r_first = r_off + A.max_nodes + 1;  // [max_nodes + 1]
    int32_t* stage = r_first + A.max_nodes + 1;
    uint16_t* slot = reinterpret_cast<uint16_t*>(stage + A.max_stage);
    const int64_t base_k = (int64_t)e0 * k, base_kk = (int64_t)e0 * kk;

    // 1. tile data into LDS; per local node, where its first row's index
    //    data lies (CSR: the node's columns, every d-th entry of the row;
    //    CRAC: the row's (first column, value position) pairs)
    for (int i = threadIdx.x; i < P * dd; i += blockDim.x) acc[i] = 0.0;
    for (int i = threadIdx.x; i < ne; i += blockDim.x) elem[i] = A.elems[e0 + i];
    for (int i = threadIdx.x; i < ne * kk; i += blockDim.x) slot[i] = A.slot[base_kk + i];
    for (int la = threadIdx.x; la < L; la += blockDim.x) {
        const int32_t R = d * A.nodes[base_k + la];
        int32_t rs, rn, cnt, src;
        if (FMT == kCSR) {
            rs = A.row_ptr[R];
            rn = A.row_ptr[R + 1];
            cnt = (rn - rs) / d;
            src = rs;
        } else {
            const int32_t cb = A.crac_row_ptr[R], ce = A.crac_row_ptr[R + 1];
            rs = A.ca[cb + 1];
            rn = A.ca[ce + 1];
            cnt = ce - cb;
            src = cb;
        }
        r_start[la] = rs;
        r_len[la] = rn - rs;
        r_cnt[la] = cnt;
        r_src[la] = src;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t sum = 0;
        for (int la = 0; la < L; ++la) {
            r_off[la] = sum;
            sum += r_cnt[la];
        }
        r_off[L] = sum;
    }
    __syncthreads();

    // 2. the index data of every local node, all loads in flight together
    {
        const int32_t total = r_off[L];
        constexpr int S = 8;
        for (int b = 0; b < total; b += S * kTileThreads) {
            int32_t val[S], at[S];
#pragma unroll
            for (int u = 0; u < S; ++u) {
                const int32_t i = b + u * kTileThreads + threadIdx.x;
                at[u] = -1;
                val[u] = 0;
                if (i < total) {
                    int32_t lo = 0, hi = L - 1;  // the local node whose range holds i
                    while (lo < hi) {
                        const int32_t mid = (lo + hi + 1) >> 1;
                        if (r_off[mid] <= i) lo = mid; else hi = mid - 1;
                    }
                    const int32_t j = i - r_off[lo];
                    val[u] = FMT == kCSR ? A.col_idx[r_src[lo] + d * j] : A.ca[r_src[lo] + j];
                    at[u] = i;
                }
            }
#pragma unroll
            for (int u = 0; u < S; ++u)
                if (at[u] >= 0) stage[at[u]] = val[u];
        }
    }
    __syncthreads();

    // 3. position of every distinct pair (row d*NA, column d*NB), searched in
    //    the staged data: CSR binary search over the node's columns, CRAC
    //    block search over the row's runs
    for (int q = threadIdx.x; q < P; q += blockDim.x) {
        const uint32_t w = A.pairs[base_kk + q];
        const int32_t la = (int32_t)(w & 0x7FFu), lb = (int32_t)((w >> 11) & 0x7FFu);
        const int32_t C = d * A.nodes[base_k + lb];
        const int32_t* st = stage + r_off[la];
        const int32_t cnt = r_cnt[la];
        int32_t p0 = -1;
        if (FMT == kCSR) {
            int32_t lo = 0, hi = cnt;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (st[mid] < C) lo = mid + 1; else hi = mid;
            }
            if (lo < cnt && st[lo] == C) p0 = r_start[la] + d * lo;
        } else {
            int32_t lo = 0, hi = cnt / 2 - 1;  // last run whose first column is <= C
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (st[2 * mid] <= C) lo = mid; else hi = mid - 1;
            }
            if (cnt >= 2 && st[2 * lo] <= C) p0 = st[2 * lo + 1] + (C - st[2 * lo]);
        }
        pos[q] = p0;
        len[q] = r_len[la] | (int32_t)(w & 0x80000000u);
        // every local node has its diagonal pair, so each node starts a run
        if (q == 0 || (A.pairs[base_kk + q - 1] & 0x7FFu) != (w & 0x7FFu)) r_first[la] = q;
        if (q == P - 1) r_first[L] = P;
    }

    // 4. every element entry into its pair's block (the tile's elements
    //    share pairs: LDS atomics)
    constexpr int U = 8;
    const int total = ne * n2;
    for (int b = 0; b < total; b += U * kTileThreads) {
        double v[U];
        int32_t where[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = b + u * kTileThreads + threadIdx.x;
            where[u] = -1;
            v[u] = 0.0;
            if (idx < total) {
                const int el = idx / n2, rsx = idx - el * n2;
                const int r = rsx / n, c = rsx - r * n;
                v[u] = __builtin_nontemporal_load(A.ke + (int64_t)elem[el] * n2 + rsx);
                where[u] = (int32_t)slot[el * kk + (r / d) * k + c / d] * dd + (r % d) * d + c % d;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (where[u] >= 0) atomicAdd(acc + where[u], v[u]);
    }
    __syncthreads();

    // 5. each accumulated entry to the global values once, row by row: the
    //    pairs of a local node are consecutive (sorted by node, then column
    //    node), so lanes walk (node, row of the node, pair, column) and
    //    neighbouring lanes write neighbouring values of one row
    for (int i = threadIdx.x; i < P * dd; i += blockDim.x) {
        int32_t lo = 0, hi = L - 1;  // the local node whose pairs hold entry i
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (r_first[mid] * dd <= i) lo = mid; else hi = mid - 1;
        }
        const int32_t qb = r_first[lo], m = r_first[lo + 1] - qb;
        const int32_t j = i - qb * dd, cr = j / (m * d), rem = j - cr * m * d;
        const int32_t q = qb + rem / d, cc = rem - (rem / d) * d;
        const int32_t p0 = pos[q];
        if (p0 < 0) continue;  // not in the pattern: cannot happen for a handle's own tiles
        const int32_t l = len[q];
        const int64_t gp = (int64_t)p0 + (int64_t)cr * (l & 0x7FFFFFFF) + cc;
        const double v = acc[q * dd + cr * d + cc];
        if (l < 0) {
            if (ACCUM)
                A.values[gp] += v;
            else
                A.values[gp] = v;
        } else {
            unsafeAtomicAdd(A.values + gp, v);
        }
    }
}

template <int FMT, bool ACCUM, int K, int D>
hipError_t launch_tile_kernel(const TileArgs& A, size_t lds, hipStream_t s) {
    auto kern = k_tile_scatter<FMT, ACCUM, K, D>;
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    kern<<<(unsigned)A.n_tiles, kTileThreads, lds, s>>>(A);
    return hipGetLastError();
}

template <int FMT, bool ACCUM>
hipError_t launch_tile_shape(const TileArgs& A, size_t lds, hipStream_t s) {
    if (A.k == 8 && A.d == 3) return launch_tile_kernel<FMT, ACCUM, 8, 3>(A, lds, s);
    if (A.k == 10 && A.d == 3) return launch_tile_kernel<FMT, ACCUM, 10, 3>(A, lds, s);
    if (A.k == 4 && A.d == 1) return launch_tile_kernel<FMT, ACCUM, 4, 1>(A, lds, s);
    if (A.k == 8 && A.d == 1) return launch_tile_kernel<FMT, ACCUM, 8, 1>(A, lds, s);
    return launch_tile_kernel<FMT, ACCUM, 0, 0>(A, lds, s);
}

unsigned grid_of(int64_t n, int block) {
    const int64_t g = ceil_div(n > 0 ? n : 1, block);
    return (unsigned)std::min<int64_t>(g, 65536);
}

// Temporaries of one tile build, released (after the stream drains) on
// every exit.
struct Scratch {
    Allocator a;
    hipStream_t s;
    std::vector<void*> ptrs;
    Scratch(const Allocator& al, hipStream_t st) : a(al), s(st) {}
    ~Scratch() {
        (void)hipStreamSynchronize(s);
        for (void* q : ptrs) dev_free(a, q, s);
    }
    template <typename T>
    int alloc(T** p, int64_t n) {
        const int rc = dev_alloc_n(a, p, n, s, "pattern_build (tiles)");
        if (rc == FEASM_OK) ptrs.push_back(*p);
        return rc;
    }
};

#define TRY(x)                          \
    do {                                \
        const int rc__ = (x);           \
        if (rc__ != FEASM_OK) return rc__; \
    } while (0)

// Distinct pairs the accumulator can hold within `budget` bytes of LDS.
int32_t tile_pair_limit(int64_t budget, int32_t d, int32_t cap, int32_t k, int32_t max_nodes,
                        int32_t max_stage) {
    const int64_t rest = budget - (int64_t)tile_lds_bytes(0, d, cap, k, max_nodes, max_stage);
    return rest > 0 ? (int32_t)std::min<int64_t>(rest / ((int64_t)d * d * 8 + 8), INT32_MAX) : 0;
}

// Elements per tile by default: the most that keep a compact tile's LDS
// (about 2/3 k^2 distinct node pairs per element, k local nodes and k^2/2
// staged ints per element, estimated) within three blocks per CU.
int32_t tile_default_cap(int32_t k, int32_t d) {
    for (int32_t cap : {64, 48, 32, 24, 16, 12, 8, 6, 4, 2}) {
        const int64_t pairs = (int64_t)cap * k * k * 2 / 3;
        const int32_t nodes = cap * k, stage = cap * k * k / 2;
        if ((int64_t)tile_lds_bytes((int32_t)pairs, d, cap, k, nodes, stage) <= kTileLdsTarget)
            return cap;
    }
    return 1;
}

}  // namespace

int build_tiles(feasm_pattern* p, hipStream_t s) {
    const int64_t E = p->n_elem;
    const int32_t k = p->k;
    const int64_t kk = (int64_t)k * k;
    if (kk > kMaxTileEntries) return FEASM_OK;  // elements too large: no tiles
    int32_t cap = (int32_t)std::min<int64_t>(kMaxTileEntries / kk, kMaxTileNodes / k);
    cap = std::min(cap, p->tune_tile_cap > 0 ? p->tune_tile_cap : tile_default_cap(k, p->d));
    if (cap < 1) return FEASM_OK;
    Scratch tmp(p->alloc, s);
    const unsigned g = grid_of(E, 256);

    // 1. distance-2 maximal independent set
    int32_t *state, *counter;
    uint64_t *t0, *t1, *t2;
    TRY(tmp.alloc(&state, E));
    TRY(tmp.alloc(&counter, 8));
    TRY(tmp.alloc(&t0, E));
    TRY(tmp.alloc(&t1, E));
    TRY(tmp.alloc(&t2, E));
    k_fill<<<g, 256, 0, s>>>(state, E, 1);
    FEASM_HIP(hipGetLastError());
    for (int round = 0;; ++round) {
        k_fill<<<1, 64, 0, s>>>(counter, 8, 0);
        k_mis_tuples<<<g, 256, 0, s>>>(state, E, t0);
        k_nbr_max<<<g, 256, 0, s>>>(p->conn, k, E, p->inc_ptr, p->inc_elem, t0, t1);
        k_nbr_max<<<g, 256, 0, s>>>(p->conn, k, E, p->inc_ptr, p->inc_elem, t1, t2);
        k_mis_decide<<<g, 256, 0, s>>>(state, t0, t2, E, counter);
        FEASM_HIP(hipGetLastError());
        int32_t undecided = 0;
        FEASM_HIP(hipMemcpyAsync(&undecided, counter, sizeof(undecided), hipMemcpyDeviceToHost, s));
        FEASM_HIP(hipStreamSynchronize(s));
        if (undecided == 0) break;
        if (round > 4096) FEASM_FAIL(FEASM_EHIP, "pattern_build: tile selection did not converge");
    }

    // 2. aggregates
    int32_t *agg, *agg2;
    TRY(tmp.alloc(&agg, E));
    TRY(tmp.alloc(&agg2, E));
    k_agg_roots<<<g, 256, 0, s>>>(p->conn, k, E, p->inc_ptr, p->inc_elem, state, agg);
    k_agg_fill<<<g, 256, 0, s>>>(p->conn, k, E, p->inc_ptr, p->inc_elem, agg, agg2, counter + 1);
    FEASM_HIP(hipGetLastError());

    // 3. elements grouped by aggregate, ascending within each, cut into tiles
    int32_t *flag, *gid, *count, *cursor;
    int64_t *rank, *scan_tmp;
    TRY(tmp.alloc(&flag, E));
    TRY(tmp.alloc(&rank, E + 1));
    TRY(tmp.alloc(&scan_tmp, scan_scratch_elems(E)));
    k_root_flags<<<g, 256, 0, s>>>(state, E, flag);
    FEASM_HIP(hipGetLastError());
    TRY(exclusive_scan<int32_t>(flag, E, rank, scan_tmp, s));
    int64_t n_agg = 0;
    int32_t hc[4];
    FEASM_HIP(hipMemcpyAsync(&n_agg, rank + E, sizeof(n_agg), hipMemcpyDeviceToHost, s));
    FEASM_HIP(hipMemcpyAsync(hc, counter, sizeof(hc), hipMemcpyDeviceToHost, s));
    FEASM_HIP(hipStreamSynchronize(s));
    if (hc[1] != 0 || n_agg <= 0)
        FEASM_FAIL(FEASM_EHIP, "pattern_build: tile aggregation left elements unassigned");
    int64_t* agg_ptr;
    TRY(tmp.alloc(&gid, E));
    TRY(tmp.alloc(&count, n_agg));
    TRY(tmp.alloc(&cursor, n_agg));
    TRY(tmp.alloc(&agg_ptr, n_agg + 1));
    k_fill<<<grid_of(n_agg, 256), 256, 0, s>>>(count, n_agg, 0);
    k_fill<<<grid_of(n_agg, 256), 256, 0, s>>>(cursor, n_agg, 0);
    k_agg_count<<<g, 256, 0, s>>>(agg2, rank, E, gid, count, counter + 2);
    FEASM_HIP(hipGetLastError());
    TRY(exclusive_scan<int32_t>(count, n_agg, agg_ptr, scan_tmp, s));
    int32_t* elems;
    TRY(dev_alloc_n(p->alloc, &elems, E, s, "pattern_build (tiles)"));
    p->tile_elems = elems;
    k_agg_scatter<<<g, 256, 0, s>>>(gid, E, agg_ptr, cursor, elems);
    FEASM_HIP(hipGetLastError());
    int32_t max_agg = 0;
    FEASM_HIP(hipMemcpyAsync(&max_agg, counter + 2, sizeof(max_agg), hipMemcpyDeviceToHost, s));
    FEASM_HIP(hipStreamSynchronize(s));
    if (max_agg > kMaxAggregate) {
        // aggregates too large to sort: no tiles (the element-centric kernel serves)
        dev_free(p->alloc, p->tile_elems, s);
        p->tile_elems = nullptr;
        return FEASM_OK;
    }
    k_agg_sort<<<(unsigned)n_agg, kPatternThreads, 0, s>>>(agg_ptr, elems);
    FEASM_HIP(hipGetLastError());
    int32_t* n_sub;
    int64_t* sub_ptr;
    TRY(tmp.alloc(&n_sub, n_agg));
    TRY(tmp.alloc(&sub_ptr, n_agg + 1));
    k_sub_count<<<grid_of(n_agg, 256), 256, 0, s>>>(agg_ptr, n_agg, cap, n_sub);
    FEASM_HIP(hipGetLastError());
    TRY(exclusive_scan<int32_t>(n_sub, n_agg, sub_ptr, scan_tmp, s));
    int64_t n_tiles = 0;
    FEASM_HIP(hipMemcpyAsync(&n_tiles, sub_ptr + n_agg, sizeof(n_tiles), hipMemcpyDeviceToHost, s));
    FEASM_HIP(hipStreamSynchronize(s));
    TRY(dev_alloc_n(p->alloc, &p->tile_ptr, n_tiles + 1, s, "pattern_build (tiles)"));
    k_sub_fill<<<grid_of(n_agg, 256), 256, 0, s>>>(agg_ptr, sub_ptr, n_agg, cap, p->tile_ptr);
    k_fill<<<1, 64, 0, s>>>(p->tile_ptr + n_tiles, 1, (int32_t)E);
    FEASM_HIP(hipGetLastError());

    // 4. local pattern of every tile
    TRY(dev_alloc_n(p->alloc, &p->tile_meta, 4 * n_tiles, s, "pattern_build (tiles)"));
    TRY(dev_alloc_n(p->alloc, &p->tile_nodes, E * k, s, "pattern_build (tiles)"));
    TRY(dev_alloc_n(p->alloc, &p->tile_pairs, E * kk, s, "pattern_build (tiles)"));
    TRY(dev_alloc_n(p->alloc, &p->tile_slot, E * kk, s, "pattern_build (tiles)"));
    TileBuild B{};
    B.conn = p->conn;
    B.inc_ptr = p->inc_ptr;
    B.inc_elem = p->inc_elem;
    B.node_ptr = p->node_ptr;
    B.node_nruns = p->node_nruns;
    B.tile_ptr = p->tile_ptr;
    B.elems = elems;
    B.k = k;
    B.tile_meta = p->tile_meta;
    B.tile_nodes = p->tile_nodes;
    B.tile_pairs = p->tile_pairs;
    B.tile_slot = p->tile_slot;
    B.maxima = counter + 4;
    k_tile_pattern<<<(unsigned)n_tiles, kPatternThreads, 0, s>>>(B);
    FEASM_HIP(hipGetLastError());

    // 5. elements of tiles too large for the accumulator
    int32_t mx[4];
    FEASM_HIP(hipMemcpyAsync(mx, counter + 4, sizeof(mx), hipMemcpyDeviceToHost, s));
    FEASM_HIP(hipStreamSynchronize(s));
    const int32_t max_pairs = mx[0];
    const int32_t limit =
        tile_pair_limit(kTileLdsBytes, p->d, cap, k, mx[1], std::max(mx[2], mx[3]));
    int64_t n_direct = 0;
    if (max_pairs > limit) {
        int32_t* dflag;
        int64_t* dpos;
        TRY(tmp.alloc(&dflag, E));
        TRY(tmp.alloc(&dpos, E + 1));
        k_direct_flags<<<grid_of(n_tiles, 256), 256, 0, s>>>(p->tile_ptr, p->tile_meta, n_tiles,
                                                             limit, dflag);
        FEASM_HIP(hipGetLastError());
        TRY(exclusive_scan<int32_t>(dflag, E, dpos, scan_tmp, s));
        FEASM_HIP(hipMemcpyAsync(&n_direct, dpos + E, sizeof(n_direct), hipMemcpyDeviceToHost, s));
        FEASM_HIP(hipStreamSynchronize(s));
        TRY(dev_alloc_n(p->alloc, &p->tile_direct, n_direct, s, "pattern_build (tiles)"));
        k_direct_fill<<<g, 256, 0, s>>>(dflag, dpos, elems, E, p->tile_direct);
        FEASM_HIP(hipGetLastError());
    }
    p->n_tiles = n_tiles;
    p->tile_cap = cap;
    p->tile_max_pairs = std::min(max_pairs, limit);
    p->tile_max_nodes = mx[1];
    p->tile_max_stage_csr = mx[2];
    p->tile_max_stage_crac = mx[3];
    p->n_tile_direct = n_direct;
    FEASM_HIP(hipStreamSynchronize(s));
    return FEASM_OK;
}


int launch_tiled_atomic(const feasm_pattern* p, int fmt, const double* ke, double* values,
                        bool accumulate, hipStream_t s) {
    TileArgs A{};
    A.tile_ptr = p->tile_ptr;
    A.elems = p->tile_elems;
    A.meta = p->tile_meta;
    A.nodes = p->tile_nodes;
    A.pairs = p->tile_pairs;
    A.slot = p->tile_slot;
    A.row_ptr = p->row_ptr;
    A.col_idx = p->col_idx;
    A.crac_row_ptr = p->crac_row_ptr;
    A.ca = p->ca;
    A.ke = ke;
    A.values = values;
    A.n_tiles = p->n_tiles;
    A.k = p->k;
    A.d = p->d;
    A.n = p->n;
    A.max_pairs = p->tile_max_pairs;
    A.cap = p->tile_cap;
    A.max_nodes = p->tile_max_nodes;
    A.max_stage = fmt == kCSR ? p->tile_max_stage_csr : p->tile_max_stage_crac;
    const size_t lds = tile_lds_bytes(A.max_pairs, A.d, A.cap, A.k, A.max_nodes, A.max_stage);
    hipError_t e;
    if (fmt == kCSR)
        e = accumulate ? launch_tile_shape<kCSR, true>(A, lds, s) : launch_tile_shape<kCSR, false>(A, lds, s);
    else
        e = accumulate ? launch_tile_shape<kCRAC, true>(A, lds, s)
                       : launch_tile_shape<kCRAC, false>(A, lds, s);
    FEASM_HIP(e);
    return FEASM_OK;
}

void release_tiles(feasm_pattern* p) {
    void* arrs[] = {p->tile_ptr, p->tile_elems, p->tile_meta, p->tile_nodes,
                    p->tile_pairs, p->tile_slot, p->tile_direct};
    for (void* a : arrs) dev_free(p->alloc, a, nullptr);
    p->tile_ptr = p->tile_elems = p->tile_meta = p->tile_nodes = p->tile_direct = nullptr;
    p->tile_pairs = nullptr;
    p->tile_slot = nullptr;
    p->n_tiles = 0;
}

}  // namespace feasm
