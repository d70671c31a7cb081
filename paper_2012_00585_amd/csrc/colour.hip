// Element colouring for the atomic-free scatter (Section 3.3: elements of one
// colour share no node, so a colour can be assembled in parallel without
// synchronisation; the paper colours greedily).
//
// The greedy first-fit rule is kept -- an element takes the smallest colour
// unused by its already-coloured neighbours -- but elements are coloured in
// the parallel order of Jones and Plassmann: in each round, every uncoloured
// element whose uncoloured neighbours all have lower priority colours
// itself.  Priorities are a fixed hash of the element id, so the result is
// deterministic.  "Coloured before this round" is read from a round stamp,
// which makes each round independent of thread timing.
//
// Elements are then grouped by colour with a stable counting sort (per
// wavefront counts, one scan, per-wavefront ranks), so each colour lists its
// elements in increasing id.
#include <climits>

#include "internal.h"

namespace feasm {

namespace {

constexpr int32_t kUncoloured = INT_MAX;

// MurmurHash3's 32-bit finaliser (Appleby), used as a fixed pseudo-random
// priority; ties are broken by the element id.
__device__ inline uint64_t priority(uint32_t e) {
    uint32_t x = e;
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return ((uint64_t)x << 32) | e;
}

__global__ void k_jp_round(const int32_t* __restrict__ conn, int32_t k, int64_t n_elem,
                           const int64_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc_elem,
                           int32_t* __restrict__ colour, int32_t* __restrict__ stamp, int32_t round,
                           int32_t* __restrict__ remaining, int32_t* __restrict__ max_colour) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (stamp[e] < round) continue;  // coloured in an earlier round
        const uint64_t mine = priority((uint32_t)e);
        bool ready = true;
        for (int32_t a = 0; a < k && ready; ++a) {
            const int32_t v = conn[e * k + a];
            for (int64_t t = inc_ptr[v]; t < inc_ptr[v + 1]; ++t) {
                const int32_t f = inc_elem[t];
                if (f == e) continue;
                if (stamp[f] >= round && priority((uint32_t)f) > mine) {
                    ready = false;
                    break;
                }
            }
        }
        if (!ready) {
            atomicAdd(remaining, 1);
            continue;
        }
        // smallest colour not used by a neighbour coloured before this round,
        // searched 64 colours at a time
        int32_t chosen = -1;
        for (int32_t base = 0; chosen < 0; base += 64) {
            uint64_t used = 0;
            for (int32_t a = 0; a < k; ++a) {
                const int32_t v = conn[e * k + a];
                for (int64_t t = inc_ptr[v]; t < inc_ptr[v + 1]; ++t) {
                    const int32_t f = inc_elem[t];
                    if (f == e || stamp[f] >= round) continue;
                    const int32_t c = colour[f] - base;
                    if (c >= 0 && c < 64) used |= 1ull << c;
                }
            }
            if (~used) chosen = base + __ffsll((unsigned long long)~used) - 1;
        }
        colour[e] = chosen;
        stamp[e] = round;
        atomicMax(max_colour, chosen);
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
    int32_t *stamp, *counters;
    int rc = dev_alloc_n(p->alloc, &p->elem_colour, E, s, "pattern_build (colouring)");
    if (rc == FEASM_OK) rc = dev_alloc_n(p->alloc, &p->colour_elems, E, s, "pattern_build (colouring)");
    if (rc == FEASM_OK) rc = tmp.alloc(&stamp, E);
    if (rc == FEASM_OK) rc = tmp.alloc(&counters, 2);
    if (rc != FEASM_OK) return rc;
    k_fill_i32<<<grid(E, 256), 256, 0, s>>>(stamp, E, kUncoloured);
    k_fill_i32<<<grid(E, 256), 256, 0, s>>>(p->elem_colour, E, -1);
    k_fill_i32<<<1, 64, 0, s>>>(counters, 2, 0);
    FEASM_HIP(hipGetLastError());
    // rounds: counters[0] = elements left after the round, counters[1] = max colour
    int32_t round = 0;
    for (;;) {
        constexpr int kBatch = 4;
        for (int r = 0; r < kBatch; ++r, ++round) {
            k_fill_i32<<<1, 64, 0, s>>>(counters, 1, 0);
            k_jp_round<<<grid(E, 256), 256, 0, s>>>(p->conn, p->k, E, p->inc_ptr, p->inc_elem,
                                                    p->elem_colour, stamp, round, counters,
                                                    counters + 1);
        }
        FEASM_HIP(hipGetLastError());
        int32_t h[2];
        FEASM_HIP(hipMemcpyAsync(h, counters, sizeof(h), hipMemcpyDeviceToHost, s));
        FEASM_HIP(hipStreamSynchronize(s));
        if (h[0] == 0) {
            p->n_colours = h[1] + 1;
            break;
        }
        if (round > 4 * E + 8)
            FEASM_FAIL(FEASM_EHIP, "colouring did not converge");  // unreachable: >= 1 element per round
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
    return FEASM_OK;
}

}  // namespace feasm
