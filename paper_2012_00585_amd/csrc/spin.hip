// Row-lock scatter: the GPU form of the paper's spin-lock methods (Section
// 3.3: a row is locked, the element's row slice is added with ordinary
// reads and writes, the row is unlocked).  One lane takes one row r of one
// element e: it finds the value positions of the row's n entries (CSR
// binary search or CRAC block search, once per element node), loads K_e's
// row, then takes the lock of global row R = D_e[r] and adds the n values.
//
// Ordering.  The lock is taken by a compare-and-swap with acquire ordering
// at agent (whole device) scope, so no value access of the critical section
// is performed before the lock is held, and the lane's non-coherent cached
// lines are invalidated.  On MI355X the eight XCDs keep separate L2 caches
// that are not coherent with each other, so the values inside the section
// are read and written with agent-scope atomic loads and stores, which are
// performed at the device's coherence point and bypass that caching.  The
// release is a relaxed agent-scope store of the lock word issued after
// waiting for every earlier memory operation of the lane to be
// acknowledged (s_waitcnt 0): the section's value stores have then reached
// the coherence point, which is what a release store would guarantee.  A
// release-ordered store would also write back the whole L2's dirty lines
// before every unlock; measured on the 64^3 hexahedra, that made the
// scatter 3.6 times slower (21 ms against 5.9 ms), for no store of the
// section that could need it.
//
// The lock words are a per-handle array (the paper keeps the lock in the
// sign bit of the row pointer; a separate array leaves the pattern
// read-only).  A lane never holds two locks, and the critical section sits
// inside the acquire loop, so the lanes of one wavefront that contend for
// one row take it in turn; every acquire loop is bounded (the spin limit),
// and a lane that reaches it gives up, leaving its row's contribution out,
// and counts itself in the abort counter (spin_aborts reports it).
#include "scatter_device.h"

namespace feasm {
namespace {

using scatter::kCRAC;
using scatter::kCSR;
using scatter::row_lookup;

constexpr int kSpinMaxN = 32;  // entries per element row held in registers

struct SpinArgs {
    const int32_t* conn;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const int32_t* crac_row_ptr;
    const int32_t* ca;
    const double* ke;
    double* values;
    int32_t* locks;   // [n_rows], all zero between launches
    int32_t* aborts;  // lanes that reached the spin limit
    int64_t n_elem;
    int32_t k, d, n;
    int64_t spin_limit;
};

// REP: some element lists a node twice, so one lane's row may name a value
// twice.
template <int FMT, bool REP>
__global__ void __launch_bounds__(256) k_spin(SpinArgs A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A.n_elem * A.n) return;
    const int64_t e = t / A.n;
    const int32_t r = (int32_t)(t - e * A.n);
    const int32_t* ce = A.conn + e * A.k;
    const int32_t R = A.d * ce[r / A.d] + r % A.d;
    // the row's index data
    int32_t rs, ncols = 0, npairs = 0;
    const int32_t* sidx;
    if (FMT == kCSR) {
        rs = A.row_ptr[R];
        ncols = A.row_ptr[R + 1] - rs;
        sidx = A.col_idx + rs;
    } else {
        const int32_t pb = A.crac_row_ptr[R], pe = A.crac_row_ptr[R + 1];
        npairs = (pe - pb) >> 1;
        sidx = A.ca + pb;
        rs = npairs > 0 ? sidx[1] : 0;
    }
    // value positions and element values of the row, before the lock
    int32_t pos[kSpinMaxN];
    double add[kSpinMaxN];
#pragma unroll
    for (int s = 0; s < kSpinMaxN; ++s) {
        pos[s] = -1;
        add[s] = 0.0;
    }
    for (int32_t b = 0; b < A.k; ++b) {
        const int32_t off = row_lookup<FMT>(sidx, ncols, npairs, rs, A.d * ce[b]);
#pragma unroll
        for (int s = 0; s < kSpinMaxN; ++s)
            if (s / A.d == b && s < A.n && off >= 0) pos[s] = rs + off + s % A.d;
    }
    const double* kr = A.ke + (e * A.n + r) * A.n;
#pragma unroll
    for (int s = 0; s < kSpinMaxN; ++s)
        if (s < A.n) add[s] = kr[s];

    int32_t* lock = A.locks + R;
    // The loop's exits are uniform across the wavefront (every lane done, or
    // the attempt count reached): with a lane-divergent exit the compiler
    // may move the critical section behind the loop, where a lane that
    // holds a lock waits for lanes of its own wavefront that spin on it.
    bool done = false;
    for (int64_t spin = 0;; ++spin) {
        if (spin >= A.spin_limit) {
            if (!done) atomicAdd(A.aborts, 1);
            break;
        }
        if (!done) {
            int32_t expected = 0;
            if (__hip_atomic_compare_exchange_strong(lock, &expected, 1, __ATOMIC_ACQUIRE,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                double cur[kSpinMaxN];
#pragma unroll
                for (int s = 0; s < kSpinMaxN; ++s)
                    if (s < A.n && pos[s] >= 0)
                        cur[s] = __hip_atomic_load(A.values + pos[s], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                // the same value may be listed twice in a row of an element
                // that repeats a node: add in entry order
#pragma unroll
                for (int s = 0; s < kSpinMaxN; ++s) {
                    if (REP && s < A.n && pos[s] >= 0) {
                        double v = cur[s];
#pragma unroll
                        for (int u = 0; u < s; ++u)
                            if (pos[u] == pos[s]) v = v + add[u];
                        cur[s] = v;
                    }
                }
#pragma unroll
                for (int s = 0; s < kSpinMaxN; ++s)
                    if (s < A.n && pos[s] >= 0)
                        __hip_atomic_store(A.values + pos[s], cur[s] + add[s], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                // release: every value store above is acknowledged by the
                // coherence point before the lock word is freed (the signal
                // fences keep the compiler from moving stores across the wait)
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __builtin_amdgcn_s_waitcnt(0);
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __hip_atomic_store(lock, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                done = true;
            }
        }
        if (__all(done)) break;
    }
}

__global__ void k_fill_zero_i32(int32_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

SpinArgs spin_args(const feasm_pattern* p, const double* ke, double* values, int32_t* locks,
                   int32_t* aborts) {
    SpinArgs A{};
    A.conn = p->conn;
    A.row_ptr = p->row_ptr;
    A.col_idx = p->col_idx;
    A.crac_row_ptr = p->crac_row_ptr;
    A.ca = p->ca;
    A.ke = ke;
    A.values = values;
    A.locks = locks;
    A.aborts = aborts;
    A.n_elem = p->n_elem;
    A.k = p->k;
    A.d = p->d;
    A.n = p->n;
    A.spin_limit = p->tune_spin_limit > 0    ? p->tune_spin_limit
                   : p->tune_spin_limit < 0 ? 0
                                            : ((int64_t)1 << 20);
    return A;
}

hipError_t launch_spin_kernel(const feasm_pattern* p, int fmt, const SpinArgs& A, hipStream_t s) {
    const unsigned blocks = (unsigned)ceil_div(p->n_elem * p->n, 256);
    if (fmt == kCSR)
        p->has_repeats ? k_spin<kCSR, true><<<blocks, 256, 0, s>>>(A)
                       : k_spin<kCSR, false><<<blocks, 256, 0, s>>>(A);
    else
        p->has_repeats ? k_spin<kCRAC, true><<<blocks, 256, 0, s>>>(A)
                       : k_spin<kCRAC, false><<<blocks, 256, 0, s>>>(A);
    return hipGetLastError();
}

}  // namespace

int launch_spin(const feasm_pattern* pc, int fmt, const double* ke, double* values, hipStream_t s) {
    feasm_pattern* p = const_cast<feasm_pattern*>(pc);  // lazily adds the lock words
    if (p->n > kSpinMaxN)
        FEASM_FAIL(FEASM_ELIMIT, "row-lock scatter supports element matrices up to 32 x 32");
    std::lock_guard<std::mutex> lazy(p->lazy_mu);
    if (!p->row_locks) {
        int rc = dev_alloc_n(p->alloc, &p->row_locks, p->n_rows, s, "row-lock scatter");
        if (rc == FEASM_OK) rc = dev_alloc_n(p->alloc, &p->spin_aborts, 1, s, "row-lock scatter");
        if (rc != FEASM_OK) return rc;
        const unsigned g = (unsigned)std::min<int64_t>(ceil_div(p->n_rows + 1, 256), 4096);
        k_fill_zero_i32<<<g, 256, 0, s>>>(p->row_locks, p->n_rows);
        k_fill_zero_i32<<<1, 64, 0, s>>>(p->spin_aborts, 1);
        FEASM_HIP(hipGetLastError());
    }
    const SpinArgs A = spin_args(p, ke, values, p->row_locks, p->spin_aborts);
    FEASM_HIP(launch_spin_kernel(p, fmt, A, s));
    return FEASM_OK;
}

}  // namespace feasm

extern "C" int spin_aborts(feasm_pattern* p, int64_t* count) {
    return feasm::guarded("spin_aborts", [&]() -> int {
        using namespace feasm;
        if (!p || !count) FEASM_FAIL(FEASM_EINVAL, "spin_aborts: null argument");
        *count = 0;
        if (!p->spin_aborts) return FEASM_OK;
        FEASM_HIP(hipDeviceSynchronize());
        int32_t v = 0;
        FEASM_HIP(hipMemcpy(&v, p->spin_aborts, sizeof(v), hipMemcpyDeviceToHost));
        const int32_t zero = 0;
        FEASM_HIP(hipMemcpy(p->spin_aborts, &zero, sizeof(zero), hipMemcpyHostToDevice));
        *count = v;
        if (v > 0) {
            set_error_for("spin_aborts", "row-lock lanes reached the spin limit; results incomplete");
            return FEASM_EINCOMPLETE;
        }
        return FEASM_OK;
    });
}

// ---------------------------------------------------------------------------
// Allocation-free row-lock scatter.  The lock words live in `scratch`, a
// device array of static storage that each GPU holds from module load until
// the process ends (zero at load).  In host code `scratch` only names the
// symbol: its device address is looked up once per device, with that device
// current, and every kernel argument uses the address looked up.
namespace feasm {
namespace {

constexpr int64_t kNoAllocMaxRows = int64_t(1) << 21;  // 8 MiB of lock words
constexpr int kMaxDevices = 64;

__device__ __align__(256) int32_t scratch[kNoAllocMaxRows];

std::mutex g_scratch_mu;
int32_t* g_scratch_dev[kMaxDevices] = {};

__global__ void k_zero_values(double* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// The current device's address of `scratch` (looked up on its first use).
int scratch_address(int device, int32_t** out) {
    std::lock_guard<std::mutex> guard(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            set_error_literal("assemble_spin_noalloc: hipGetSymbolAddress of the lock words failed");
            return FEASM_EHIP;
        }
        g_scratch_dev[device] = static_cast<int32_t*>(ptr);
    }
    *out = g_scratch_dev[device];
    return FEASM_OK;
}

}  // namespace
}  // namespace feasm

extern "C" int assemble_spin_noalloc(const feasm_pattern* p, int fmt, const double* ke,
                                     double* values, int32_t* aborts, int flags,
                                     hipStream_t stream) {
    return feasm::guarded("assemble_spin_noalloc", [&]() -> int {
        using namespace feasm;
        if (!p || !ke || !values || !aborts) {
            set_error_literal("assemble_spin_noalloc: null handle or buffer");
            return FEASM_EINVAL;
        }
        if (fmt != FEASM_FMT_CSR && fmt != FEASM_FMT_CRAC) {
            set_error_literal("assemble_spin_noalloc: fmt must be FEASM_FMT_CSR or FEASM_FMT_CRAC");
            return FEASM_EINVAL;
        }
        if ((fmt == FEASM_FMT_CSR && !(p->flags & FEASM_BUILD_CSR)) ||
            (fmt == FEASM_FMT_CRAC && !(p->flags & FEASM_BUILD_CRAC))) {
            set_error_literal("assemble_spin_noalloc: handle was built without this format");
            return FEASM_EINVAL;
        }
        if (flags != 0 && flags != FEASM_ACCUMULATE) {
            set_error_literal("assemble_spin_noalloc: flags must be 0 or FEASM_ACCUMULATE");
            return FEASM_EINVAL;
        }
        if (p->n > kSpinMaxN) {
            set_error_literal("assemble_spin_noalloc: element matrices up to 32 x 32 only");
            return FEASM_ELIMIT;
        }
        if (p->n_rows > kNoAllocMaxRows) {
            set_error_literal("assemble_spin_noalloc: more than 2^21 rows (the static lock array)");
            return FEASM_ELIMIT;
        }
        int device = -1;
        if (hipGetDevice(&device) != hipSuccess || device != p->device) {
            set_error_literal("assemble_spin_noalloc: the handle's device must be current");
            return FEASM_EINVAL;
        }
        if (device < 0 || device >= kMaxDevices) {
            set_error_literal("assemble_spin_noalloc: device index beyond 63");
            return FEASM_ELIMIT;
        }
        int32_t* locks = nullptr;
        const int rc = scratch_address(device, &locks);
        if (rc != FEASM_OK) return rc;
        // every lock word this launch can take starts free, whatever earlier
        // calls left; the reset is a kernel, so the call can be captured
        const unsigned g = (unsigned)std::min<int64_t>(ceil_div(p->n_rows, 256), 4096);
        k_fill_zero_i32<<<g, 256, 0, stream>>>(locks, p->n_rows);
        if (flags == 0) {
            const unsigned gv = (unsigned)std::min<int64_t>(ceil_div(p->nnz, 256), 16384);
            k_zero_values<<<gv, 256, 0, stream>>>(values, p->nnz);
        }
        const SpinArgs A = spin_args(p, ke, values, locks, aborts);
        if (launch_spin_kernel(p, fmt, A, stream) != hipSuccess) {
            set_error_literal("assemble_spin_noalloc: kernel launch failed");
            return FEASM_EHIP;
        }
        return FEASM_OK;
    });
}
