// Element colouring for the atomic-free scatter (Section 3.3: elements of one
// colour share no node, so a colour can be assembled in parallel without
// synchronisation; the paper colours greedily).
//
// The result is exactly the sequential greedy colouring in element order:
// element e takes the smallest colour not used by any element f < e that
// shares a node with it.  That colour depends only on the colours of e's
// smaller neighbours, so e can be coloured as soon as all of them are, and
// the elements coloured at one time share no node.  The device runs the
// greedy order as rounds over a frontier (a wavefront per element):
//   * pred[e] counts the (element, shared node) incidences of e with smaller
//     elements (a neighbour sharing two nodes counts twice);
//   * the first frontier holds the elements with pred 0;
//   * a round colours every frontier element from its smaller neighbours'
//     colours, then takes one off pred of every larger neighbour per shared
//     node; an element whose count reaches 0 joins the next frontier.
// Structured meshes in lexicographic order get the paper's even 4 (quads)
// and 8 (hexes) colours.  Rounds are launched in batches between host
// checks; a round past the last frontier finds an empty one and does
// nothing.
//
// Elements are then grouped by colour with a stable counting sort (per
// wavefront counts, one scan, per-wavefront ranks), so each colour lists its
// elements in increasing id.
#include <algorithm>

#include <cmath>
#include <vector>

#include "internal.h"

namespace feasm {

namespace {

// pred[e] = incidences of e with smaller elements, summed over e's nodes.
__global__ void k_pred_count(const int32_t* __restrict__ conn, int32_t k, int64_t n_elem,
                             const int64_t* __restrict__ inc_ptr,
                             const int32_t* __restrict__ inc_elem, int32_t* __restrict__ pred,
                             int32_t* __restrict__ frontier, int32_t* __restrict__ count) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t c = 0;
        for (int32_t a = 0; a < k; ++a) {
            const int32_t v = conn[e * k + a];
            // incident elements are ascending within a node
            for (int64_t t = inc_ptr[v]; t < inc_ptr[v + 1]; ++t) {
                if (inc_elem[t] >= e) break;
                ++c;
            }
        }
        pred[e] = c;
        if (c == 0) frontier[atomicAdd(count, 1)] = (int32_t)e;
    }
}

__device__ inline uint64_t wave_or(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// One greedy round, one wavefront per frontier element (its lanes take the
// element's nodes and walk their incidence lists).  counts[r % 3] holds this
// round's frontier size; the next frontier is counted in counts[(r + 1) % 3];
// counts[(r + 2) % 3] (read by the previous round) is cleared for the round
// after next.  All lanes of a wavefront take the same element, so the
// shuffles always see the whole wavefront.
__global__ void __launch_bounds__(256)
    k_greedy_round(const int32_t* __restrict__ conn, int32_t k,
                   const int64_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc_elem,
                   int32_t* __restrict__ colour, int32_t* __restrict__ pred,
                   const int32_t* __restrict__ front_in, int32_t* __restrict__ front_out,
                   int32_t* __restrict__ counts, int32_t round, int32_t* __restrict__ max_colour,
                   unsigned long long* __restrict__ n_coloured) {
    const int32_t cur = round % 3, nxt = (round + 1) % 3, clr = (round + 2) % 3;
    const int32_t n = counts[cur];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counts[clr] = 0;
        if (n > 0) atomicAdd(n_coloured, (unsigned long long)n);
    }
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t w0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    for (int64_t i = w0; i < n; i += waves) {
        const int32_t e = front_in[i];
        const int32_t* ce = conn + (int64_t)e * k;
        // smallest colour unused by the smaller neighbours, 64 colours at a time
        int32_t chosen = -1;
        for (int32_t base = 0; chosen < 0; base += 64) {
            uint64_t used = 0;
            for (int32_t a = lane; a < k; a += 64) {
                const int32_t v = ce[a];
                for (int64_t t = inc_ptr[v]; t < inc_ptr[v + 1]; ++t) {
                    const int32_t f = inc_elem[t];
                    if (f >= e) break;
                    const int32_t c = colour[f] - base;
                    if (c >= 0 && c < 64) used |= 1ull << c;
                }
            }
            used = wave_or(used);
            if (~used) chosen = base + __ffsll((unsigned long long)~used) - 1;
        }
        if (lane == 0) {
            colour[e] = chosen;
            atomicMax(max_colour, chosen);
        }
        // release the larger neighbours, once per shared node
        for (int32_t a = lane; a < k; a += 64) {
            const int32_t v = ce[a];
            for (int64_t t = inc_ptr[v]; t < inc_ptr[v + 1]; ++t) {
                const int32_t f = inc_elem[t];
                if (f <= e) continue;
                if (atomicSub(pred + f, 1) == 1) front_out[atomicAdd(counts + nxt, 1)] = f;
            }
        }
    }
}

__device__ inline uint64_t lanes_below() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// For wavefront w (64 consecutive elements): counts[c * n_waves + w] = number
// of its elements with colour c (COUNT), or each element's slot in the
// colour-grouped list (FILL).
template <bool FILL>
__global__ void __launch_bounds__(256)
    k_group(const int32_t* __restrict__ colour, int64_t n_elem, int64_t n_waves,
            int32_t* __restrict__ counts, const int64_t* __restrict__ offs,
            int32_t* __restrict__ out) {
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= n_waves) return;  // whole wavefronts exit together
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = e < n_elem;
    const int32_t c = valid ? colour[e] : -1;
    bool pending = valid;
    while (__ballot(pending)) {
        const uint64_t act = __ballot(pending);
        const int leader = __ffsll((unsigned long long)act) - 1;
        const int32_t cl = __shfl(c, leader, 64);
        const bool mine = pending && c == cl;
        const uint64_t m = __ballot(mine);
        if (mine) {
            const int32_t rank = __popcll(m & lanes_below());
            if (FILL)
                out[offs[(int64_t)cl * n_waves + w] + rank] = (int32_t)e;
            else if (rank == 0)
                counts[(int64_t)cl * n_waves + w] = __popcll(m);
            pending = false;
        }
    }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_gather_ptr(const int64_t* offs, int64_t n_waves, int32_t n_colours,
                             int64_t* colour_ptr) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c <= n_colours) colour_ptr[c] = offs[(int64_t)c * n_waves];
}

unsigned grid(int64_t n, int block) {
    int64_t g = ceil_div(n > 0 ? n : 1, block);
    return (unsigned)(g < 65536 ? g : 65536);
}

struct Buf {
    Allocator a;
    hipStream_t s;
    std::vector<void*> ptrs;
    Buf(const Allocator& al, hipStream_t st) : a(al), s(st) {}
    ~Buf() {
        (void)hipStreamSynchronize(s);
        for (void* q : ptrs) dev_free(a, q, s);
    }
    template <typename T>
    int alloc(T** p, int64_t n) {
        const int rc = dev_alloc_n(a, p, n, s, "pattern_build (colouring)");
        if (rc == FEASM_OK) ptrs.push_back(*p);
        return rc;
    }
};

}  // namespace

int build_colouring(feasm_pattern* p, hipStream_t s) {
    const int64_t E = p->n_elem;
    Buf tmp(p->alloc, s);
    int32_t *pred, *front0, *front1, *counters;
    unsigned long long* n_coloured;
    int rc = dev_alloc_n(p->alloc, &p->elem_colour, E, s, "pattern_build (colouring)");
    if (rc == FEASM_OK) rc = dev_alloc_n(p->alloc, &p->colour_elems, E, s, "pattern_build (colouring)");
    if (rc == FEASM_OK) rc = tmp.alloc(&pred, E);
    if (rc == FEASM_OK) rc = tmp.alloc(&front0, E);
    if (rc == FEASM_OK) rc = tmp.alloc(&front1, E);
    // counters[0..2]: frontier sizes by round mod 3; counters[3]: largest colour
    if (rc == FEASM_OK) rc = tmp.alloc(&counters, 4);
    if (rc == FEASM_OK) rc = tmp.alloc(&n_coloured, 1);
    if (rc != FEASM_OK) return rc;
    k_fill_i32<<<grid(E, 256), 256, 0, s>>>(p->elem_colour, E, -1);
    k_fill_i32<<<1, 64, 0, s>>>(counters, 4, 0);
    k_fill_i32<<<1, 64, 0, s>>>(reinterpret_cast<int32_t*>(n_coloured), 2, 0);
    k_pred_count<<<grid(E, 256), 256, 0, s>>>(p->conn, p->k, E, p->inc_ptr, p->inc_elem, pred,
                                              front0, counters);
    FEASM_HIP(hipGetLastError());
    // the longest chain of neighbours in increasing element order bounds the
    // rounds (a few hundred on the structured meshes); check every kBatch
    constexpr int kBatch = 32;
    const unsigned g = std::min(grid(E * 64, 256), 2048u);  // a wavefront per element
    int64_t round = 0;
    for (;;) {
        for (int r = 0; r < kBatch; ++r, ++round) {
            int32_t* fin = (round & 1) ? front1 : front0;
            int32_t* fout = (round & 1) ? front0 : front1;
            k_greedy_round<<<g, 256, 0, s>>>(p->conn, p->k, p->inc_ptr, p->inc_elem,
                                             p->elem_colour, pred, fin, fout, counters,
                                             (int32_t)(round % 3), counters + 3, n_coloured);
        }
        FEASM_HIP(hipGetLastError());
        unsigned long long done = 0;
        int32_t maxc = 0;
        FEASM_HIP(hipMemcpyAsync(&done, n_coloured, sizeof(done), hipMemcpyDeviceToHost, s));
        FEASM_HIP(hipMemcpyAsync(&maxc, counters + 3, sizeof(maxc), hipMemcpyDeviceToHost, s));
        FEASM_HIP(hipStreamSynchronize(s));
        if ((int64_t)done == E) {
            p->n_colours = maxc + 1;
            break;
        }
        if (round > E + kBatch)  // unreachable: every round colours at least one element
            FEASM_FAIL(FEASM_EHIP, "colouring did not converge");
    }
    // stable grouping by colour
    const int64_t n_waves = ceil_div(E, 64);
    const int64_t nc = p->n_colours;
    int32_t* counts;
    int64_t *offs, *scratch, *cptr;
    rc = tmp.alloc(&counts, nc * n_waves);
    if (rc == FEASM_OK) rc = tmp.alloc(&offs, nc * n_waves + 1);
    if (rc == FEASM_OK) rc = tmp.alloc(&scratch, scan_scratch_elems(nc * n_waves));
    if (rc == FEASM_OK) rc = tmp.alloc(&cptr, nc + 1);
    if (rc != FEASM_OK) return rc;
    k_fill_i32<<<grid(nc * n_waves, 256), 256, 0, s>>>(counts, nc * n_waves, 0);
    const unsigned gb = (unsigned)ceil_div(n_waves * 64, 256);
    k_group<false><<<gb, 256, 0, s>>>(p->elem_colour, E, n_waves, counts, nullptr, nullptr);
    FEASM_HIP(hipGetLastError());
    rc = exclusive_scan<int32_t>(counts, nc * n_waves, offs, scratch, s);
    if (rc != FEASM_OK) return rc;
    k_group<true><<<gb, 256, 0, s>>>(p->elem_colour, E, n_waves, nullptr, offs, p->colour_elems);
    k_gather_ptr<<<(unsigned)ceil_div(nc + 1, 64), 64, 0, s>>>(offs, n_waves, (int32_t)nc, cptr);
    FEASM_HIP(hipGetLastError());
    p->colour_ptr.assign(nc + 1, 0);
    FEASM_HIP(hipMemcpyAsync(p->colour_ptr.data(), cptr, sizeof(int64_t) * (nc + 1),
                             hipMemcpyDeviceToHost, s));
    FEASM_HIP(hipStreamSynchronize(s));
    return set_colour_blocks(p, 0, s);
}

// Colour phases re-read and re-write every values line that elements of
// several colours reach.  Running the colours block by block, over element
// id ranges whose value rows fit in the 256 MiB memory-side cache, keeps
// those lines there between phases (for a mesh numbered with locality);
// the default block count is the values array's size over that cache,
// rounded (hex64: 2 blocks, 1.66 -> 1.34 ms).
int set_colour_blocks(feasm_pattern* p, int64_t nb, hipStream_t s) {
    constexpr double kMallBytes = 256.0 * 1024 * 1024;
    const int64_t E = p->n_elem;
    const int32_t nc = p->n_colours;
    if (nb <= 0) nb = std::llround((double)p->nnz * 8 / kMallBytes);
    nb = std::max<int64_t>(1, std::min<int64_t>({nb, 256, E}));
    std::vector<int64_t> t((size_t)nc * (nb + 1));
    if (nb == 1) {
        for (int32_t c = 0; c < nc; ++c) {
            t[2 * c] = p->colour_ptr[c];
            t[2 * c + 1] = p->colour_ptr[c + 1];
        }
    } else {
        std::vector<int32_t> ce((size_t)E);
        FEASM_HIP(hipStreamSynchronize(s));
        FEASM_HIP(hipMemcpy(ce.data(), p->colour_elems, sizeof(int32_t) * E, hipMemcpyDeviceToHost));
        const int64_t eb = ceil_div(E, nb);
        for (int32_t c = 0; c < nc; ++c) {
            // element ids ascend within a colour
            const auto first = ce.begin() + p->colour_ptr[c], last = ce.begin() + p->colour_ptr[c + 1];
            for (int64_t b = 0; b <= nb; ++b) {
                const int64_t lim = std::min<int64_t>(b * eb, E);
                t[(size_t)c * (nb + 1) + b] =
                    std::lower_bound(first, last, (int32_t)lim) - ce.begin();
            }
        }
    }
    // every block range lies inside its colour's range, in order
    for (int32_t c = 0; c < nc; ++c) {
        const int64_t* r = t.data() + (size_t)c * (nb + 1);
        if (r[0] != p->colour_ptr[c] || r[nb] != p->colour_ptr[c + 1])
            FEASM_FAIL(FEASM_EHIP, "colour blocks: a colour's blocks do not span it");
        for (int64_t b = 0; b < nb; ++b)
            if (r[b] > r[b + 1]) FEASM_FAIL(FEASM_EHIP, "colour blocks: block starts out of order");
    }
    p->colour_block_ptr = std::move(t);
    p->colour_blocks = (int32_t)nb;
    return FEASM_OK;
}

}  // namespace feasm
