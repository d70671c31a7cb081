// Batched assembly: many independent meshes in one graph-captured launch.
//
// Every mesh keeps its own pattern handle, element matrices and values
// array.  The host turns the batch into work tiles -- node-row tiles of
// row-owned meshes, element blocks of atomic meshes, and one list per
// colour for coloured meshes -- grouped by code path.  Each (phase, path)
// group runs as one persistent kernel sized to the resident capacity of that
// path, whose blocks pop chunks of tiles from a device counter (the same
// device routines as the single-mesh kernels, so results are identical).
// Path-specialised kernels keep each path's register budget, instead of one
// kernel carrying the union of all paths.  Colours need a grid-wide order,
// so colour phases are chained launches on a second graph branch that runs
// beside the row-owned and atomic launches.  The whole sequence -- counter
// reset, zero fill of the meshes that assemble with atomics or colours, the
// launches -- is captured once into a hipGraph and replayed on the caller's
// stream; a replay with new element-matrix or values pointers only refreshes
// the device pointer table first.
#include <algorithm>
#include <array>
#include <cstring>
#include <utility>
#include <new>
#include <vector>

#include "internal.h"
#include "scatter_device.h"

struct feasm_batch;

namespace feasm {
namespace {

using namespace scatter;

// Kernel paths of the batch (one block of 64 lanes per tile).
enum Path : int32_t {
    kOwnG4 = 0, kOwnG8, kOwnG16, kOwnG32, kOwnG64J1, kOwnG64J2, kOwnG64J4, kOwnG64J8, kOwnG64J16,
    kRows2J1, kRows2J2,
    kPipe24,  // 8-node hexes, 3 DOFs per node, at most 8 incident entries per node:
              // the single-mesh flat row-owned kernel, one node row per tile
    kLanes3, kLanes4,  // one DOF per node, 3- or 4-node elements: a node row per lane,
                       // 64 rows per tile (single-mesh calls keep row groups of 4
                       // lanes: 38 against 41 us on 512^2 quads; in the batch,
                       // where tiles are plentiful, the fatter tiles win)
    kElemA16, kElemA32, kElemA64, kElemP16, kElemP32, kElemP64,
    kNumPaths
};

struct MeshDesc {
    AsmArgs asm_args;   // element paths (ke/values/elem_list filled per tile)
    OwnArgs own_args;   // row-owned paths (ke/values filled per tile)
    const int64_t* colour_ptr;  // dev [n_colours+1]
    int32_t path;
};

struct BatchTile {
    int32_t mesh;
    int32_t colour;  // colour list of element tiles of coloured meshes, else -1
    int64_t index;   // logical block index within the mesh's path
};

struct ZeroChunk {
    int32_t mesh;
    int32_t pad;
    int64_t first;
    int64_t count;
};

constexpr int64_t kZeroChunk = 1 << 16;

__global__ void __launch_bounds__(256)
    k_batch_zero(const ZeroChunk* __restrict__ chunks, int64_t n_chunks, double* const* values) {
    for (int64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const ZeroChunk z = chunks[c];
        double* p = global_ptr(values[z.mesh]) + z.first;
        for (int64_t i = threadIdx.x; i < z.count; i += blockDim.x) p[i] = 0.0;
    }
}

// Tiles of a path are split into kXcds contiguous ranges, one counter each;
// the counters sit kCounterStride words apart (256 bytes), so that the eight
// of one launch are eight separate memory-side atomic streams rather than
// one hot line.
constexpr int kXcds = 8;
constexpr int kCounterStride = 32;

__global__ void k_batch_reset(unsigned long long* counters, int32_t n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0ull;
}

__device__ inline int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One work tile of a batch.  The tile entry and the mesh's arguments are
// wave-uniform scalar loads.  LOOP: the caller runs tiles one after another
// in a loop, where the pipelined row kernel recomputes its per-lane index
// arithmetic instead of keeping it live across tiles.
template <int FMT, int PATH, bool LOOP>
__device__ inline void batch_tile(const MeshDesc* __restrict__ meshes,
                                  const double* const* __restrict__ ke,
                                  double* const* __restrict__ values,
                                  const BatchTile* __restrict__ tile, double* lds) {
    const int32_t cur = ldc(&tile->mesh);
    const int32_t colour = ldc(&tile->colour);
    const int64_t index = ldc(&tile->index);
    if (PATH <= kLanes4) {
        OwnArgs O = meshes[cur].own_args;
        O.ke = ke[cur];
        O.values = values[cur];
        to_global(O);
        if (PATH == kOwnG4) owner_tiles<FMT, 4, 1, 8>(O, index, index + 1, lds);
        if (PATH == kOwnG8) owner_tiles<FMT, 8, 1, 8>(O, index, index + 1, lds);
        if (PATH == kOwnG16) owner_tiles<FMT, 16, 1, 8>(O, index, index + 1, lds);
        if (PATH == kOwnG32) owner_tiles<FMT, 32, 1, 8>(O, index, index + 1, lds);
        if (PATH == kOwnG64J1) owner_tiles<FMT, 64, 1, 8>(O, index, index + 1, lds);
        if (PATH == kOwnG64J2) owner_tiles<FMT, 64, 2, 8>(O, index, index + 1, lds);
        if (PATH == kOwnG64J4) owner_tiles<FMT, 64, 4, 4>(O, index, index + 1, lds);
        if (PATH == kOwnG64J8) owner_tiles<FMT, 64, 8, 2>(O, index, index + 1, lds);
        if (PATH == kOwnG64J16) owner_tiles<FMT, 64, 16, 1>(O, index, index + 1, lds);
        if (PATH == kRows2J1) owner_rows_tile<FMT, 2, 1, 8>(O, index, lds);
        if (PATH == kRows2J2) owner_rows_tile<FMT, 2, 2, 8>(O, index, lds);
        if (PATH == kPipe24) owner_pipe_row<FMT, 3, 24, 8, 0, LOOP>(O, index, lds);
        if (PATH == kLanes3) owner_lanes<FMT, 3, 4>(O, index * 64, lds);
        if (PATH == kLanes4) owner_lanes<FMT, 4, 4>(O, index * 64, lds);
    } else {
        AsmArgs A = meshes[cur].asm_args;
        A.ke = ke[cur];
        A.values = values[cur];
        if (colour >= 0) {
            const int64_t* cp = meshes[cur].colour_ptr;
            const int64_t c0 = ldc(cp + colour);
            const int64_t c1 = ldc(cp + colour + 1);
            A.elem_list = A.elem_list + c0;
            A.count = c1 - c0;
        }
        to_global(A);
        int32_t* li = reinterpret_cast<int32_t*>(lds);
        if (PATH == kElemA16) elem_tile<FMT, true, 16, 1, 64>(A, index, li);
        if (PATH == kElemA32) elem_tile<FMT, true, 32, 2, 64>(A, index, li);
        if (PATH == kElemA64) elem_tile<FMT, true, 64, 16, 64>(A, index, li);
        if (PATH == kElemP16) elem_tile<FMT, false, 16, 1, 64>(A, index, li);
        if (PATH == kElemP32) elem_tile<FMT, false, 32, 2, 64>(A, index, li);
        if (PATH == kElemP64) elem_tile<FMT, false, 64, 16, 64>(A, index, li);
    }
}

// Tile-grid launch (the default): one workgroup per tile of a code path,
// tiles first .. first + gridDim.x - 1, scheduled by the hardware dispatcher
// as a single-mesh launch is; each XCD takes a contiguous part of the range,
// so neighbouring rows share their element matrices' lines in one L2.
template <int FMT, int PATH>
__global__ void __launch_bounds__(64)
    k_batch_grid(const MeshDesc* __restrict__ meshes, const double* const* __restrict__ ke,
                 double* const* __restrict__ values, const BatchTile* __restrict__ tiles,
                 int64_t first) {
    extern __shared__ double lds[];
    batch_tile<FMT, PATH, false>(meshes, ke, values,
                                 tiles + first + xcd_block(blockIdx.x, gridDim.x), lds);
}

// Persistent launch: as many workgroups as are resident at once.  The
// path's tile list is split into one contiguous range per XCD (hardware
// dispatches workgroup b to XCD b % 8); a workgroup pops `chunk` tiles at a
// time from its XCD's range, so neighbouring tiles -- which read the same
// connectivity rows and element matrices -- run on one XCD and share its
// L2; when its range is exhausted it helps the other ranges, and leaves when
// every range is.
template <int FMT, int PATH>
__global__ void __launch_bounds__(64)
    k_batch(const MeshDesc* __restrict__ meshes, const double* const* __restrict__ ke,
            double* const* __restrict__ values, const BatchTile* __restrict__ tiles,
            int64_t n_tiles, int64_t chunk, unsigned long long* counters) {
    extern __shared__ double lds[];
    __shared__ int64_t s_first;
    const int home = (int)(blockIdx.x % kXcds);
    for (int step = 0; step < kXcds; ++step) {
        const int x = (home + step) % kXcds;
        const int64_t lo = n_tiles * x / kXcds, hi = n_tiles * (x + 1) / kXcds;
        for (;;) {
            if (threadIdx.x == 0)
                s_first = lo + (int64_t)atomicAdd(counters + x * kCounterStride,
                                                  (unsigned long long)chunk);
            __syncthreads();
            const int64_t first = uniform64(s_first);
            __syncthreads();
            if (first >= hi) break;
            const int64_t last = first + chunk < hi ? first + chunk : hi;
            for (int64_t t = first; t < last; ++t) {
                batch_tile<FMT, PATH, true>(meshes, ke, values, tiles + t, lds);
                __syncthreads();  // LDS is reused by the next tile
            }
        }
    }
}

using BatchKernel = void (*)(const MeshDesc*, const double* const*, double* const*,
                             const BatchTile*, int64_t, int64_t, unsigned long long*);
using GridKernel = void (*)(const MeshDesc*, const double* const*, double* const*,
                            const BatchTile*, int64_t);

template <int FMT, int... P>
constexpr std::array<BatchKernel, sizeof...(P)> kernel_table(std::integer_sequence<int, P...>) {
    return {&k_batch<FMT, P>...};
}

template <int FMT, int... P>
constexpr std::array<GridKernel, sizeof...(P)> grid_table(std::integer_sequence<int, P...>) {
    return {&k_batch_grid<FMT, P>...};
}

BatchKernel batch_kernel(int fmt, int path) {
    static const auto t0 = kernel_table<0>(std::make_integer_sequence<int, kNumPaths>{});
    static const auto t1 = kernel_table<1>(std::make_integer_sequence<int, kNumPaths>{});
    return fmt == 0 ? t0[path] : t1[path];
}

GridKernel grid_kernel(int fmt, int path) {
    static const auto t0 = grid_table<0>(std::make_integer_sequence<int, kNumPaths>{});
    static const auto t1 = grid_table<1>(std::make_integer_sequence<int, kNumPaths>{});
    return fmt == 0 ? t0[path] : t1[path];
}

// Largest tile-grid launch; longer tile lists take several launches (the
// limit keeps a dispatch's work-item count far within 32 bits, and is low
// enough that the hex path of the 512-mesh mix is split and tested so).
constexpr int64_t kGridTilesMax = int64_t(1) << 22;

}  // namespace
}  // namespace feasm

namespace feasm {
namespace {

// One persistent launch: the tiles of one code path in one phase (phase 0:
// row-owned and atomic meshes; phase c+1: colour c of coloured meshes).
struct Launch {
    int32_t phase = 0;
    int32_t path = 0;
    BatchTile* d_tiles = nullptr;
    int64_t n_tiles = 0;
    size_t lds = 0;
    int64_t grid = 0;
    int64_t chunk = 1;
    double work = 0;
};

}  // namespace
}  // namespace feasm

struct feasm_batch {
    feasm::Allocator alloc;  // every device array of the batch comes from it
    int fmt = 0;
    int64_t count = 0;
    int device = 0;
    int accumulate = 0;
    int per_mesh_graph = 0;  // mode: every mesh's own kernels in one graph
    int persistent = 0;      // mode: persistent launches pulling tiles from counters
    std::vector<const feasm_pattern*> patterns;
    feasm::MeshDesc* d_meshes = nullptr;
    std::vector<int64_t*> d_colour_ptrs;
    std::vector<feasm::Launch> launches;
    int32_t n_phases = 1;
    unsigned long long* d_counters = nullptr;
    feasm::ZeroChunk* d_zero = nullptr;
    int64_t n_zero = 0;
    const double** d_ke = nullptr;
    double** d_values = nullptr;
    std::vector<const double*> h_ke;  // last uploaded tables
    std::vector<double*> h_values;
    static constexpr int kStreams = 3;  // capture origin, phase 0, colours
    hipStream_t streams[kStreams] = {nullptr, nullptr, nullptr};  // capture only
    hipEvent_t events[kStreams] = {nullptr, nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<int32_t> paths;  // per mesh, for batch_info
    static constexpr int kBranches = 4;
    hipStream_t branch[kBranches] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t branch_done[kBranches] = {nullptr, nullptr, nullptr, nullptr};
};

namespace feasm {
namespace {

// Path, per-block LDS bytes and tile granularity of one mesh given its tuning.
int mesh_path(const feasm_pattern* p, int fmt, int strategy, MeshDesc& D, size_t& lds,
              int64_t& per) {
    const int64_t dn = (int64_t)p->d * p->n;
    if (strategy == FEASM_SCATTER_OWNER) {
        if (dn > 1024) FEASM_FAIL(FEASM_ELIMIT, "assemble_batch: row-owned path needs d*n <= 1024");
        int g = 4;
        while (g < dn && g < 64) g <<= 1;
        for (;; g <<= 1) {
            if (g > 64) FEASM_FAIL(FEASM_ELIMIT, "assemble_batch: node rows too long for LDS");
            const int j = (int)ceil_div(dn, g);
            const int jj = j <= 1 ? 1 : j <= 2 ? 2 : j <= 4 ? 4 : j <= 8 ? 8 : 16;
            const int b = jj <= 2 ? 8 : jj == 4 ? 4 : jj == 8 ? 2 : 1;
            const int64_t idx = (fmt == 0) ? (int64_t)p->d * p->max_deg : 2 * (int64_t)p->max_deg + 2;
            const int64_t bytes = (int64_t)p->d * p->d * p->max_deg * 8 + idx * 4 + (int64_t)b * p->k * 4;
            const int64_t gb = ceil_div(bytes, 8) * 8;
            if (gb * (64 / g) > 64 * 1024) continue;
            OwnArgs& A = D.own_args;
            A.idx_ints = (int32_t)idx;
            A.acc_doubles = p->d * p->d * p->max_deg;
            A.group_bytes = (int32_t)gb;
            if (g == 64 && p->d == 3 && p->n == 24 && p->max_inc <= 8 && p->tune_owner_flat >= 0 &&
                p->tune_owner_rows <= 1 && gb + 2 * 8 * p->k * 4 <= 64 * 1024) {
                D.path = kPipe24;
                lds = (size_t)gb + (size_t)2 * 8 * p->k * 4;
                per = 1;  // one node row per tile
                return FEASM_OK;
            }
            if (g < 64 && p->d == 1 && (p->k == 3 || p->k == 4) && p->tune_owner_rows == 0 &&
                owner_lanes_lds(fmt, p->max_deg) <= 32 * 1024) {
                D.path = p->k == 3 ? kLanes3 : kLanes4;
                A.acc_doubles = (int32_t)(64 * p->max_deg);
                lds = owner_lanes_lds(fmt, p->max_deg);
                per = 64;  // node rows per tile
                return FEASM_OK;
            }
            const int rows = p->tune_owner_rows != 0 ? p->tune_owner_rows : (g == 64 && gb <= 3072 ? 2 : 1);
            if (g == 64 && rows == 2 && jj <= 2 && gb * 2 + 8 * p->k * 4 <= 64 * 1024) {
                D.path = jj == 1 ? kRows2J1 : kRows2J2;
                lds = (size_t)gb * 2 + (size_t)8 * p->k * 4;
                per = 2;
            } else {
                static const int32_t gpath[] = {kOwnG4, kOwnG8, kOwnG16, kOwnG32};
                if (g < 64) {
                    int gi = 0;
                    while ((4 << gi) != g) ++gi;
                    D.path = gpath[gi];
                } else {
                    D.path = jj == 1 ? kOwnG64J1 : jj == 2 ? kOwnG64J2 : jj == 4 ? kOwnG64J4
                             : jj == 8 ? kOwnG64J8 : kOwnG64J16;
                }
                lds = (size_t)gb * (64 / g);
                per = 64 / g;  // node rows per tile
            }
            return FEASM_OK;
        }
    }
    // element paths: at most 64 lanes per element (one 64-lane block per tile)
    const int64_t n2 = (int64_t)p->n * p->n;
    int tpe = p->tune_atomic_tpe;
    if (tpe == 0 || tpe > 64) tpe = n2 <= 16 ? 16 : n2 <= 64 ? 32 : 64;
    if (tpe == 16 && n2 > 16) tpe = n2 <= 64 ? 32 : 64;
    if (tpe == 32 && n2 > 64) tpe = 64;
    const bool atomic = strategy == FEASM_SCATTER_ATOMIC || p->has_repeats;
    D.path = atomic ? (tpe == 16 ? kElemA16 : tpe == 32 ? kElemA32 : kElemA64)
                    : (tpe == 16 ? kElemP16 : tpe == 32 ? kElemP32 : kElemP64);
    const int64_t lds_ints = 3 * (int64_t)p->k + 3 * (int64_t)p->n + (int64_t)p->k * p->k;
    lds = (size_t)lds_ints * 4 * (64 / tpe);
    if (lds > 64 * 1024) FEASM_FAIL(FEASM_ELIMIT, "assemble_batch: element too large for LDS");
    D.asm_args.lds_ints = (int32_t)lds_ints;
    per = 64 / tpe;  // elements per tile
    return FEASM_OK;
}

// Launches of phase 0 (row-owned and atomic meshes) run one after another on
// one graph branch, largest work first (two alternating branches measured no
// faster); colour phases are chained on a second branch beside them.
int build_graph(feasm_batch* b) {
    for (int i = 0; i < feasm_batch::kStreams; ++i) {
        FEASM_HIP(hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking));
        FEASM_HIP(hipEventCreateWithFlags(&b->events[i], hipEventDisableTiming));
    }
    hipStream_t s0 = b->streams[0];
    FEASM_HIP(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
    const int32_t nl = (int32_t)b->launches.size();
    if (b->persistent) k_batch_reset<<<1, 256, 0, s0>>>(b->d_counters, nl * kXcds * kCounterStride);
    if (b->n_zero > 0 && !b->accumulate)
        k_batch_zero<<<(unsigned)std::min<int64_t>(b->n_zero, 8192), 256, 0, s0>>>(b->d_zero, b->n_zero,
                                                                                  b->d_values);
    hipError_t err = hipEventRecord(b->events[0], s0);
    bool used[feasm_batch::kStreams] = {true, false, false};
    for (int32_t i = 0; i < nl && err == hipSuccess; ++i) {
        const Launch& L = b->launches[i];
        const int br = L.phase == 0 ? 1 : 2;
        hipStream_t s = b->streams[br];
        if (!used[br]) {
            err = hipStreamWaitEvent(s, b->events[0], 0);
            used[br] = true;
        }
        if (b->persistent) {
            batch_kernel(b->fmt, L.path)<<<(unsigned)L.grid, 64, L.lds, s>>>(
                b->d_meshes, b->d_ke, b->d_values, L.d_tiles, L.n_tiles, L.chunk,
                b->d_counters + (int64_t)i * kXcds * kCounterStride);
        } else {
            for (int64_t f = 0; f < L.n_tiles; f += kGridTilesMax)
                grid_kernel(b->fmt, L.path)<<<(unsigned)std::min(kGridTilesMax, L.n_tiles - f), 64,
                                              L.lds, s>>>(b->d_meshes, b->d_ke, b->d_values,
                                                          L.d_tiles, f);
        }
    }
    for (int br = 1; br < feasm_batch::kStreams && err == hipSuccess; ++br) {
        if (!used[br]) continue;
        err = hipEventRecord(b->events[br], b->streams[br]);
        if (err == hipSuccess) err = hipStreamWaitEvent(s0, b->events[br], 0);
    }
    const hipError_t le = hipGetLastError();
    const hipError_t ce = hipStreamEndCapture(s0, &b->graph);
    FEASM_HIP(err);
    FEASM_HIP(le);
    FEASM_HIP(ce);
    FEASM_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return FEASM_OK;
}

// Per-mesh-graph mode: the single-mesh numeric calls of every mesh, largest
// first, dealt round-robin onto parallel graph branches.  The kernels take
// the element-matrix and values pointers as arguments, so the graph is
// recaptured whenever they change.
int capture_per_mesh(feasm_batch* b, const double* const* ke, double* const* values) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (!b->streams[0]) {
        FEASM_HIP(hipStreamCreateWithFlags(&b->streams[0], hipStreamNonBlocking));
        FEASM_HIP(hipEventCreateWithFlags(&b->events[0], hipEventDisableTiming));
        for (int i = 0; i < feasm_batch::kBranches; ++i) {
            FEASM_HIP(hipStreamCreateWithFlags(&b->branch[i], hipStreamNonBlocking));
            FEASM_HIP(hipEventCreateWithFlags(&b->branch_done[i], hipEventDisableTiming));
        }
    }
    std::vector<int64_t> order(b->count);
    for (int64_t m = 0; m < b->count; ++m) order[m] = m;
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
        return b->patterns[x]->n_elem * b->patterns[x]->n * b->patterns[x]->n >
               b->patterns[y]->n_elem * b->patterns[y]->n * b->patterns[y]->n;
    });
    hipStream_t s0 = b->streams[0];
    FEASM_HIP(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipEventRecord(b->events[0], s0);
    for (int i = 0; i < feasm_batch::kBranches && err == hipSuccess; ++i)
        err = hipStreamWaitEvent(b->branch[i], b->events[0], 0);
    int rc = FEASM_OK;
    const int scatter = FEASM_SCATTER_AUTO | (b->accumulate ? FEASM_ACCUMULATE : 0);
    for (int64_t i = 0; i < b->count && err == hipSuccess && rc == FEASM_OK; ++i) {
        const int64_t m = order[i];
        rc = assemble_on_stream(b->patterns[m], b->fmt, ke[m], values[m], scatter,
                                b->branch[i % feasm_batch::kBranches]);
    }
    for (int i = 0; i < feasm_batch::kBranches && err == hipSuccess; ++i) {
        err = hipEventRecord(b->branch_done[i], b->branch[i]);
        if (err == hipSuccess) err = hipStreamWaitEvent(s0, b->branch_done[i], 0);
    }
    const hipError_t ce = hipStreamEndCapture(s0, &b->graph);
    if (rc != FEASM_OK) return rc;
    FEASM_HIP(err);
    FEASM_HIP(ce);
    FEASM_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return FEASM_OK;
}

void release_batch(feasm_batch* b) {
    for (int i = 0; i < feasm_batch::kBranches; ++i) {
        if (b->branch[i]) (void)hipStreamDestroy(b->branch[i]);
        if (b->branch_done[i]) (void)hipEventDestroy(b->branch_done[i]);
    }
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (int i = 0; i < feasm_batch::kStreams; ++i) {
        if (b->streams[i]) (void)hipStreamDestroy(b->streams[i]);
        if (b->events[i]) (void)hipEventDestroy(b->events[i]);
    }
    void* arrs[] = {b->d_meshes, b->d_counters, b->d_zero, b->d_ke, b->d_values};
    for (void* a : arrs) dev_free(b->alloc, a, nullptr);
    for (auto& L : b->launches) dev_free(b->alloc, L.d_tiles, nullptr);
    for (auto* c : b->d_colour_ptrs) dev_free(b->alloc, c, nullptr);
}

int create(feasm_batch* b, const feasm_pattern* const* patterns, int64_t count, int fmt,
           int accumulate) {
    b->fmt = fmt;
    b->count = count;
    b->accumulate = accumulate;
    (void)hipGetDevice(&b->device);
    b->alloc = current_allocator();
    b->patterns.assign(patterns, patterns + count);
    b->paths.assign(count, 0);
    if (b->per_mesh_graph) {
        for (int64_t m = 0; m < count; ++m) {
            const feasm_pattern* p = patterns[m];
            if (!p) FEASM_FAIL(FEASM_EINVAL, "batch_create: null handle at " + std::to_string(m));
            if (!(p->flags & (fmt == FEASM_FMT_CSR ? FEASM_BUILD_CSR : FEASM_BUILD_CRAC)))
                FEASM_FAIL(FEASM_EINVAL, "batch_create: mesh " + std::to_string(m) +
                                             " lacks the requested format");
        }
        b->h_ke.assign(count, nullptr);
        b->h_values.assign(count, nullptr);
        return FEASM_OK;  // captured on the first assemble_batch
    }
    std::vector<MeshDesc> descs(count);
    // (phase, path) -> tiles, work
    std::vector<std::vector<std::vector<BatchTile>>> lists;  // [phase][path]
    std::vector<std::vector<double>> work;
    std::vector<std::vector<size_t>> ldsv;
    std::vector<int64_t> path_per(kNumPaths, 1);  // rows or elements per tile of a path
    auto ensure = [&](int32_t ph) {
        while ((int32_t)lists.size() <= ph) {
            lists.emplace_back(kNumPaths);
            work.emplace_back(kNumPaths, 0.0);
            ldsv.emplace_back(kNumPaths, (size_t)0);
        }
    };
    ensure(0);
    std::vector<ZeroChunk> zero;
    b->d_colour_ptrs.assign(count, nullptr);
    b->paths.assign(count, 0);
    for (int64_t m = 0; m < count; ++m) {
        const feasm_pattern* p = patterns[m];
        if (!p) FEASM_FAIL(FEASM_EINVAL, "batch_create: null handle at " + std::to_string(m));
        if (fmt == FEASM_FMT_CSR && !(p->flags & FEASM_BUILD_CSR))
            FEASM_FAIL(FEASM_EINVAL, "batch_create: mesh " + std::to_string(m) + " has no CSR");
        if (fmt == FEASM_FMT_CRAC && !(p->flags & FEASM_BUILD_CRAC))
            FEASM_FAIL(FEASM_EINVAL, "batch_create: mesh " + std::to_string(m) + " has no CRAC");
        int strategy = p->tune_strategy;
        if (strategy == FEASM_SCATTER_AUTO) strategy = FEASM_SCATTER_OWNER;
        if (strategy == FEASM_SCATTER_COLOURED && !(p->flags & FEASM_BUILD_COLOUR))
            FEASM_FAIL(FEASM_EINVAL, "batch_create: coloured strategy needs a coloured handle");
        MeshDesc& D = descs[m];
        std::memset(&D, 0, sizeof(D));
        size_t lds = 0;
        int64_t per = 1;
        int rc = mesh_path(p, fmt, strategy, D, lds, per);
        if (rc != FEASM_OK && strategy == FEASM_SCATTER_OWNER) {
            strategy = FEASM_SCATTER_ATOMIC;  // rows too long for LDS: fall back
            rc = mesh_path(p, fmt, strategy, D, lds, per);
        }
        if (rc != FEASM_OK) return rc;
        b->paths[m] = D.path;
        path_per[D.path] = per;
        AsmArgs& A = D.asm_args;
        A.conn = p->conn;
        A.k = p->k;
        A.d = p->d;
        A.n = p->n;
        A.row_ptr = p->row_ptr;
        A.col_idx = p->col_idx;
        A.crac_row_ptr = p->crac_row_ptr;
        A.ca = p->ca;
        A.count = p->n_elem;
        A.elem_list = nullptr;
        OwnArgs& O = D.own_args;
        O.conn = p->conn;
        O.k = p->k;
        O.d = p->d;
        O.n = p->n;
        O.inc_ptr = p->inc_ptr;
        O.inc_q = p->inc_q;
        O.inc_elem = p->inc_elem;
        O.inc_local = p->inc_local;
        O.row_ptr = p->row_ptr;
        O.col_idx = p->col_idx;
        O.crac_row_ptr = p->crac_row_ptr;
        O.ca = p->ca;
        O.n_nodes = p->n_nodes;
        O.accumulate = accumulate;
        O.persistent = 0;
        const double elem_cost = (double)p->n * p->n;
        if (D.path >= kElemA16 && !accumulate)
            for (int64_t f = 0; f < p->nnz; f += kZeroChunk)
                zero.push_back({(int32_t)m, 0, f, std::min<int64_t>(kZeroChunk, p->nnz - f)});
        if (strategy == FEASM_SCATTER_COLOURED) {
            A.elem_list = p->colour_elems;
            const int32_t nc = p->n_colours;
            {
                const int rc__ = dev_alloc(b->alloc, (void**)&b->d_colour_ptrs[m],
                                           sizeof(int64_t) * (nc + 1), nullptr, "batch_create");
                if (rc__ != FEASM_OK) return rc__;
            }
            FEASM_HIP(hipMemcpy(b->d_colour_ptrs[m], p->colour_ptr.data(),
                                sizeof(int64_t) * (nc + 1), hipMemcpyHostToDevice));
            D.colour_ptr = b->d_colour_ptrs[m];
            ensure(nc);
            for (int32_t c = 0; c < nc; ++c) {
                const int64_t sz = p->colour_ptr[c + 1] - p->colour_ptr[c];
                for (int64_t i = 0; i < ceil_div(sz, per); ++i)
                    lists[c + 1][D.path].push_back({(int32_t)m, c, i});
                work[c + 1][D.path] += elem_cost * sz;
                ldsv[c + 1][D.path] = std::max(ldsv[c + 1][D.path], lds);
            }
        } else {
            const int64_t units = D.path >= kElemA16 ? p->n_elem : p->n_nodes;
            for (int64_t i = 0; i < ceil_div(units, per); ++i)
                lists[0][D.path].push_back({(int32_t)m, -1, i});
            work[0][D.path] += elem_cost * p->n_elem;
            ldsv[0][D.path] = std::max(ldsv[0][D.path], lds);
        }
    }
    {
        const int rc__ = dev_alloc(b->alloc, (void**)&b->d_meshes,
                                   sizeof(MeshDesc) * count, nullptr, "batch_create");
        if (rc__ != FEASM_OK) return rc__;
    }
    FEASM_HIP(hipMemcpy(b->d_meshes, descs.data(), sizeof(MeshDesc) * count, hipMemcpyHostToDevice));
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    cus = std::max(cus, 1);
    b->n_phases = (int32_t)lists.size();
    for (int32_t ph = 0; ph < (int32_t)lists.size(); ++ph) {
        std::vector<Launch> here;
        for (int32_t path = 0; path < kNumPaths; ++path) {
            auto& tl = lists[ph][path];
            if (tl.empty()) continue;
            Launch L;
            L.phase = ph;
            L.path = path;
            L.n_tiles = (int64_t)tl.size();
            L.lds = ldsv[ph][path];
            L.work = work[ph][path];
            if (L.lds > 64 * 1024) FEASM_FAIL(FEASM_ELIMIT, "batch_create: LDS per block exceeds 64 KiB");
            int per_cu = 0;
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel(fmt, path), 64,
                                                               L.lds);
            const int64_t cap = (int64_t)cus * std::max(per_cu, 1);
            if (b->persistent) {
                // small chunks keep the in-flight rows of an XCD close together:
                // about four rows or elements per counter pop (four one-row tiles,
                // one 64-row tile) measured best on the 512-mesh mix
                const int64_t want = std::max<int64_t>(1, 4 / path_per[path]);
                L.chunk = std::max<int64_t>(1, std::min<int64_t>(want, L.n_tiles / (cap * 8)));
                L.grid = std::max<int64_t>(1, std::min<int64_t>(cap, ceil_div(L.n_tiles, L.chunk)));
            } else {
                L.chunk = 1;
                L.grid = std::min(L.n_tiles, kGridTilesMax);
            }
            {
                const int rc__ = dev_alloc(b->alloc, (void**)&L.d_tiles,
                                           sizeof(BatchTile) * tl.size(), nullptr, "batch_create");
                if (rc__ != FEASM_OK) return rc__;
            }
            FEASM_HIP(hipMemcpy(L.d_tiles, tl.data(), sizeof(BatchTile) * tl.size(),
                                hipMemcpyHostToDevice));
            here.push_back(L);
        }
        std::stable_sort(here.begin(), here.end(),
                         [](const Launch& x, const Launch& y) { return x.work > y.work; });
        b->launches.insert(b->launches.end(), here.begin(), here.end());
    }
    {
        const int rc = dev_alloc_n(b->alloc, &b->d_counters,
                                   (int64_t)b->launches.size() * kXcds * kCounterStride, nullptr,
                                   "batch_create");
        if (rc != FEASM_OK) return rc;
    }
    if ((int64_t)b->launches.size() > 64)
        FEASM_FAIL(FEASM_ELIMIT, "batch_create: more than 64 (phase, path) launches");
    b->n_zero = (int64_t)zero.size();
    if (!zero.empty()) {
        {
            const int rc__ = dev_alloc(b->alloc, (void**)&b->d_zero,
                                       sizeof(ZeroChunk) * zero.size(), nullptr, "batch_create");
            if (rc__ != FEASM_OK) return rc__;
        }
        FEASM_HIP(hipMemcpy(b->d_zero, zero.data(), sizeof(ZeroChunk) * zero.size(),
                            hipMemcpyHostToDevice));
    }
    {
        const int rc__ = dev_alloc(b->alloc, (void**)&b->d_ke,
                                   sizeof(double*) * count, nullptr, "batch_create");
        if (rc__ != FEASM_OK) return rc__;
    }
    {
        const int rc__ = dev_alloc(b->alloc, (void**)&b->d_values,
                                   sizeof(double*) * count, nullptr, "batch_create");
        if (rc__ != FEASM_OK) return rc__;
    }
    FEASM_HIP(hipMemset(b->d_ke, 0, sizeof(double*) * count));
    FEASM_HIP(hipMemset(b->d_values, 0, sizeof(double*) * count));
    b->h_ke.assign(count, nullptr);
    b->h_values.assign(count, nullptr);
    return build_graph(b);
}

}  // namespace
}  // namespace feasm

extern "C" int batch_create(const feasm_pattern* const* patterns, int64_t count, int fmt,
                            uint32_t flags, feasm_batch** out) {
    return feasm::guarded("batch_create", [&]() -> int {
        using namespace feasm;
        if (!out) FEASM_FAIL(FEASM_EINVAL, "batch_create: out is NULL");
        *out = nullptr;
        if (!patterns || count <= 0) FEASM_FAIL(FEASM_EINVAL, "batch_create: no meshes");
        if (count > INT32_MAX) FEASM_FAIL(FEASM_EOVERFLOW, "batch_create: too many meshes");
        if (fmt != FEASM_FMT_CSR && fmt != FEASM_FMT_CRAC)
            FEASM_FAIL(FEASM_EINVAL, "batch_create: fmt must be FEASM_FMT_CSR or FEASM_FMT_CRAC");
        if (flags & ~(uint32_t)(FEASM_ACCUMULATE | FEASM_BATCH_PER_MESH_GRAPH | FEASM_BATCH_PERSISTENT))
            FEASM_FAIL(FEASM_EINVAL, "batch_create: unknown flag");
        if ((flags & FEASM_BATCH_PER_MESH_GRAPH) && (flags & FEASM_BATCH_PERSISTENT))
            FEASM_FAIL(FEASM_EINVAL, "batch_create: per-mesh-graph and persistent modes exclude each other");
        feasm_batch* b = new (std::nothrow) feasm_batch();
        if (!b) FEASM_FAIL(FEASM_ENOMEM, "batch_create: out of host memory");
        b->per_mesh_graph = (flags & FEASM_BATCH_PER_MESH_GRAPH) ? 1 : 0;
        b->persistent = (flags & FEASM_BATCH_PERSISTENT) ? 1 : 0;
        const int rc = create(b, patterns, count, fmt, (flags & FEASM_ACCUMULATE) ? 1 : 0);
        if (rc != FEASM_OK) {
            (void)hipDeviceSynchronize();
            release_batch(b);
            delete b;
            return rc;
        }
        *out = b;
        return FEASM_OK;
    });
}

extern "C" int assemble_batch(feasm_batch* b, const double* const* ke, double* const* values,
                              hipStream_t stream) {
    return feasm::guarded("assemble_batch", [&]() -> int {
        using namespace feasm;
        if (!b) FEASM_FAIL(FEASM_EINVAL, "assemble_batch: null batch");
        if (!ke || !values) FEASM_FAIL(FEASM_EINVAL, "assemble_batch: ke or values table is NULL");
        bool changed = false;
        for (int64_t m = 0; m < b->count; ++m) {
            if (!ke[m] || !values[m])
                FEASM_FAIL(FEASM_EINVAL, "assemble_batch: null pointer for mesh " + std::to_string(m));
            changed |= ke[m] != b->h_ke[m] || values[m] != b->h_values[m];
        }
        if (b->per_mesh_graph) {
            if (changed || !b->exec) {
                b->h_ke.assign(ke, ke + b->count);
                b->h_values.assign(values, values + b->count);
                const int rc = capture_per_mesh(b, ke, values);
                if (rc != FEASM_OK) return rc;
            }
            FEASM_HIP(hipGraphLaunch(b->exec, stream));
            return FEASM_OK;
        }
        if (changed) {
            // the tables are read by the graph's kernels: update them in stream order
            b->h_ke.assign(ke, ke + b->count);
            b->h_values.assign(values, values + b->count);
            FEASM_HIP(hipMemcpyAsync(b->d_ke, b->h_ke.data(), sizeof(double*) * b->count,
                                     hipMemcpyHostToDevice, stream));
            FEASM_HIP(hipMemcpyAsync(b->d_values, b->h_values.data(), sizeof(double*) * b->count,
                                     hipMemcpyHostToDevice, stream));
            FEASM_HIP(hipStreamSynchronize(stream));  // host tables may change before the copy runs
        }
        FEASM_HIP(hipGraphLaunch(b->exec, stream));
        return FEASM_OK;
    });
}

extern "C" int batch_info(const feasm_batch* b, int32_t* n_phases, int64_t* n_tiles,
                          int64_t* grid, int32_t* paths) {
    return feasm::guarded("batch_info", [&]() -> int {
        if (!b) FEASM_FAIL(FEASM_EINVAL, "batch_info: null batch");
        if (n_phases) *n_phases = b->n_phases;
        int64_t t = 0, g = 0;
        for (const auto& L : b->launches) {
            t += L.n_tiles;
            g = std::max(g, L.grid);
        }
        if (n_tiles) *n_tiles = t;
        if (grid) *grid = g;
        if (paths)
            for (int64_t m = 0; m < b->count; ++m) paths[m] = b->paths[m];
        return FEASM_OK;
    });
}

extern "C" void batch_free(feasm_batch* b) {
    try {
        if (!b) return;
        (void)hipDeviceSynchronize();
        feasm::release_batch(b);
        delete b;
    } catch (...) {
        // nothing to report: the call has no status
    }
}
