// Internal declarations of libfeasm (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <mutex>
#include <string>
#include <vector>

#include "feasm.h"

namespace feasm {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg) noexcept;
// "who: what", without allocating when that fails.
void set_error_for(const char* who, const char* what) noexcept;
// A message with static storage duration, recorded without allocating.
void set_error_literal(const char* msg) noexcept;

// Runs the body of a C entry point.  The library's own code reports errors
// by status; the only exceptions that can reach here come from the standard
// library's host containers and strings running out of memory, and they
// become FEASM_ENOMEM instead of crossing the C ABI.
template <typename F>
int guarded(const char* who, F&& body) noexcept {
    try {
        return body();
    } catch (const std::exception& ex) {
        set_error_for(who, ex.what());
        return FEASM_ENOMEM;
    } catch (...) {
        set_error_for(who, "unexpected C++ exception");
        return FEASM_ENOMEM;
    }
}

struct Status {
    int code = FEASM_OK;
    bool ok() const { return code == FEASM_OK; }
};

#define FEASM_FAIL(code_, msg_)                 \
    do {                                        \
        ::feasm::set_error(msg_);               \
        return (code_);                         \
    } while (0)

#define FEASM_HIP(call_)                                                              \
    do {                                                                              \
        hipError_t e__ = (call_);                                                     \
        if (e__ != hipSuccess) {                                                      \
            ::feasm::set_error(std::string(#call_) + ": " + hipGetErrorString(e__)); \
            return (e__ == hipErrorOutOfMemory ? FEASM_ENOMEM : FEASM_EHIP);          \
        }                                                                             \
    } while (0)

// ---------------------------------------------------------------- memory
// The allocator of set_allocator (alloc == nullptr: hipMalloc / hipFree).
struct Allocator {
    feasm_alloc_fn alloc = nullptr;
    feasm_release_fn release = nullptr;
    void* ctx = nullptr;
};
// The allocator set now (objects keep the one they were created with).
Allocator current_allocator();
// bytes (0 is allowed and allocates a minimal block) of device memory from
// `a`; on failure sets the error message (naming `who`) and returns
// FEASM_ENOMEM or FEASM_EHIP with *ptr = nullptr.
int dev_alloc(const Allocator& a, void** ptr, size_t bytes, hipStream_t s, const char* who);
template <typename T>
int dev_alloc_n(const Allocator& a, T** ptr, int64_t count, hipStream_t s, const char* who) {
    return dev_alloc(a, reinterpret_cast<void**>(ptr), sizeof(T) * (size_t)(count > 0 ? count : 1), s,
                     who);
}
// Gives ptr (may be null) back to `a`; the caller has made sure that no
// queued work still uses it.
void dev_free(const Allocator& a, void* ptr, hipStream_t s);

// ---------------------------------------------------------------- handle
struct OffsetCache;  // value-only re-assembly lookup cache (assemble.hip)

}  // namespace feasm

// Entries of padding after the incidence array (zeros).
constexpr int kIncPad = 64;
// Incident entries of a "light" node row (one batch of the flat row-owned kernel).
constexpr int kLightInc = 8;

struct feasm_pattern {
    int device = 0;
    feasm::Allocator alloc;  // every device array of the handle comes from it
    int64_t n_elem = 0;
    int32_t k = 0, d = 0, n = 0;
    int64_t n_nodes = 0, n_rows = 0;
    uint32_t flags = 0;
    bool has_repeats = false;  // some element lists a node twice
    int32_t max_deg = 0;       // most neighbour nodes of any node
    int32_t max_inc = 0;       // most incident (element, local node) entries of any node

    int32_t* conn = nullptr;  // dev [n_elem*k]

    // node-level pattern: node v couples with node_col[node_ptr[v] .. node_ptr[v+1])
    int64_t node_nnz = 0, node_runs = 0;
    int64_t* node_ptr = nullptr;     // dev [n_nodes+1]
    int32_t* node_col = nullptr;     // dev [node_nnz]
    int32_t* node_nruns = nullptr;   // dev [n_nodes]
    int64_t* noderun_ptr = nullptr;  // dev [n_nodes+1]

    // node -> incident (element*k + local) entries, ascending within a node
    int64_t* inc_ptr = nullptr;  // dev [n_nodes+1]
    int32_t* inc_q = nullptr;      // dev [n_elem*k] entries e*k + a
    int32_t* inc_elem = nullptr;   // dev [n_elem*k] element e of each entry (after build)
    int32_t* inc_local = nullptr;  // dev [n_elem*k] local node a of each entry

    // CSR
    int64_t nnz = 0;
    int32_t* row_ptr = nullptr;  // dev [n_rows+1]
    int32_t* col_idx = nullptr;  // dev [nnz]

    // CRAC
    int64_t n_ca = 0;
    int32_t* crac_row_ptr = nullptr;  // dev [n_rows+1]
    int32_t* ca = nullptr;            // dev [n_ca]

    // colouring
    int32_t n_colours = 0;
    std::vector<int64_t> colour_ptr;  // host [n_colours+1]
    // The coloured scatter runs element block by element block, the colours
    // in order within each block: block b of colour c is colour_elems
    // [colour_block_ptr[c*(colour_blocks+1)+b], ...[...+b+1]) (host table).
    int32_t colour_blocks = 1;
    std::vector<int64_t> colour_block_ptr;
    int32_t* colour_elems = nullptr;  // dev [n_elem]
    int32_t* elem_colour = nullptr;   // dev [n_elem]

    feasm::OffsetCache* cache = nullptr;
    // nodes with at most kLightInc incident entries first, then the rest,
    // each part in increasing id
    int32_t* node_order = nullptr;  // dev [n_nodes]
    int64_t n_light = 0;
    int32_t* owner_map = nullptr;  // dev [n_elem*k][k]: row-owned lookup record
    bool owner_map_valid = false;
    int32_t* row_locks = nullptr;    // dev [n_rows]: row-lock scatter (zero between launches)
    int32_t* spin_aborts = nullptr;  // dev [1]: lanes that reached the spin limit
    // Serialises the creation of the state above that numeric calls add on
    // first use (owner_map, cache, row_locks) between threads sharing a handle.
    mutable std::mutex lazy_mu;

    // element tiles of the atomic scatter (FEASM_BUILD_TILES; tiles.hip)
    int64_t n_tiles = 0;              // 0: none (the element-centric kernel serves)
    int32_t tile_cap = 0;             // elements per tile at most
    int32_t tile_max_pairs = 0;       // distinct node pairs the accumulator holds
    int32_t tile_max_nodes = 0;       // local nodes of a tile at most
    int32_t tile_max_stage_csr = 0;   // index ints a tile stages (CSR, CRAC) at most
    int32_t tile_max_stage_crac = 0;
    int32_t* tile_ptr = nullptr;      // dev [n_tiles+1]: tile t = tile_elems[tile_ptr[t], tile_ptr[t+1])
    int32_t* tile_elems = nullptr;    // dev [n_elem]: element ids, tile by tile, ascending in a tile
    int32_t* tile_meta = nullptr;     // dev [n_tiles][4]: distinct node pairs, local nodes,
                                      //   staged CSR ints, staged CRAC ints
    int32_t* tile_nodes = nullptr;    // dev [n_elem*k]: tile t's nodes at tile_ptr[t]*k, ascending
    uint32_t* tile_pairs = nullptr;   // dev [n_elem*k*k]: at tile_ptr[t]*k*k, local a | local b << 11
                                      //   | complete << 31, in (a, b) order
    uint16_t* tile_slot = nullptr;    // dev [n_elem*k*k]: pair of entry (element i of the tile, a, b)
    int32_t* tile_direct = nullptr;   // dev [n_tile_direct]: elements of tiles beyond the accumulator
    int64_t n_tile_direct = 0;

    // tuning (0 = library default)
    int32_t tune_owner_blocks_per_cu = 0;  // >0: persistent row-owned grid of this size per CU
    int32_t tune_atomic_tpe = 0;           // threads per element of the atomic/coloured scatter
    int32_t tune_owner_rows = 0;           // >1: node rows per wavefront (row-owned, large elements)
    int32_t tune_owner_batch = 0;          // incidence entries loaded per batch (8 or 16)
    int32_t tune_strategy = 0;             // what FEASM_SCATTER_AUTO resolves to (0: row-owned)
    int32_t tune_owner_flat = 0;           // flat batches: -1 off, 0 auto, else entries per batch
    int32_t tune_owner_prefetch = 0;       // flat batches: issue the next batch early
    int32_t tune_spmv_chunk = 0;           // matrix-vector product: values per LDS chunk
    int64_t tune_spin_limit = 0;           // row-lock scatter: acquire attempts per lane
    int32_t tune_tile_cap = 0;             // elements per atomic-scatter tile at most (0: by size)
    int32_t tune_hex8_pipe = 0;            // fused hexahedra: -1 one node per wavefront, 0 auto,
                                           // else pipelined blocks per CU
};

namespace feasm {

// ---------------------------------------------------------------- helpers
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Exclusive scan: out[i] = sum_{j<i} in[j] for i in [0, n]; out[n] is the total.
// `scratch` must hold scan_scratch_elems(n) int64 values.
int64_t scan_scratch_elems(int64_t n);
template <typename T>
int exclusive_scan(const T* in, int64_t n, int64_t* out, int64_t* scratch, hipStream_t s);
// Builds p->node_order (see feasm_pattern) and its count of light nodes;
// synchronises s.
int build_node_order(feasm_pattern* p, hipStream_t s, int64_t* n_light_host);

// Colouring (colour.hip): fills p->elem_colour, colour_elems, colour_ptr, n_colours.
int build_colouring(feasm_pattern* p, hipStream_t s);
// Splits every colour's element list into nb element-id blocks (0: by the
// matrix size) and stores the table of block starts (synchronises s).
int set_colour_blocks(feasm_pattern* p, int64_t nb, hipStream_t s);

// Element tiles of the atomic scatter (tiles.hip): build_tiles fills the
// tile arrays of the handle (or leaves n_tiles = 0 when tiles cannot be
// formed) and synchronises s; launch_tiled_atomic runs the tiles whose pairs
// fit the accumulator (the caller runs the element-centric kernel over
// tile_direct).
int build_tiles(feasm_pattern* p, hipStream_t s);
int launch_tiled_atomic(const feasm_pattern* p, int fmt, const double* ke, double* values,
                        bool accumulate, hipStream_t s);
void release_tiles(feasm_pattern* p);

// Row-lock scatter (spin.hip) of one mesh into reset (or accumulated) values.
int launch_spin(const feasm_pattern* p, int fmt, const double* ke, double* values, hipStream_t s);

// The numeric phase of one mesh on a stream (asynchronous; used by batches).
int assemble_on_stream(const feasm_pattern* p, int fmt, const double* ke, double* values,
                       int scatter, hipStream_t s);

// Free every device array of the handle.
void release_pattern(feasm_pattern* p);
void release_cache(feasm_pattern* p);
void release_owner_map(feasm_pattern* p);
// The row-owned lookup record, built during pattern_build (asynchronous on s).
int build_owner_record(feasm_pattern* p, hipStream_t s);

// XCD-aware block order: hardware dispatches workgroup b to XCD b % 8.
// Maps it to a logical index so that each XCD processes one contiguous range.
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t x = b % 8, q = nb / 8, rem = nb % 8;
    const int64_t start = x * q + (x < rem ? x : rem);
    return start + b / 8;
}

}  // namespace feasm
