// Native serving engine: assembly + Newton-style re-assembly requests as
// they arrive, with continuous batching.
//
// One host thread runs the loop.  Requests arrive at given times; the FIFO
// head is admitted into a free slot once the HBM budget (sum of admitted
// footprints: two element-matrix buffers plus one values buffer) allows.
// Each slot has a stream for assembly and a side stream on which the next
// iteration's element matrices are generated (ping-pong buffers) while the
// current iteration assembles.  A slot issues its next iteration as soon as
// it sees the previous one complete (a Newton loop with zero solver time),
// so the work of every admitted request overlaps on the device.  Slot
// buffers are allocated once, at the size of the largest registered mesh.
#include <algorithm>
#include <chrono>
#include <deque>
#include <thread>
#include <vector>

#include "internal.h"

namespace feasm {
namespace {

// Key of iteration `it` of a request (0 = assembly).
inline uint64_t iteration_seed(uint64_t seed, int32_t it) {
    return seed * 1000003ull + (uint64_t)it * 7919ull + 1ull;
}

struct Slot {
    hipStream_t main = nullptr, side = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t gen[2] = {nullptr, nullptr};
    double* ke[2] = {nullptr, nullptr};
    double* values = nullptr;
    int64_t req = -1;
    int32_t it = 0;
    bool flushing = false;  // final copy-out in flight
    double issued = 0.0;
    int64_t footprint = 0;
};

}  // namespace
}  // namespace feasm

extern "C" int serve_run(const feasm_pattern* const* meshes, const int32_t* recipes, int64_t n_meshes,
                         const feasm_request* requests, int64_t n_requests, int fmt, int32_t n_slots,
                         int64_t hbm_budget, feasm_request_result* results,
                         double* reassembly_latency) {
    return feasm::guarded("serve_run", [&]() -> int {
        using namespace feasm;
        using clock = std::chrono::steady_clock;
        if (!meshes || !recipes || n_meshes <= 0 || (n_requests > 0 && (!requests || !results)))
            FEASM_FAIL(FEASM_EINVAL, "serve_run: null argument");
        if (n_slots <= 0 || n_slots > 256) FEASM_FAIL(FEASM_EINVAL, "serve_run: slots must be in [1, 256]");
        if (fmt != FEASM_FMT_CSR && fmt != FEASM_FMT_CRAC)
            FEASM_FAIL(FEASM_EINVAL, "serve_run: fmt must be FEASM_FMT_CSR or FEASM_FMT_CRAC");
        int64_t max_ke = 0, max_nnz = 0;
        for (int64_t m = 0; m < n_meshes; ++m) {
            const feasm_pattern* p = meshes[m];
            if (!p) FEASM_FAIL(FEASM_EINVAL, "serve_run: null mesh handle");
            if (recipes[m] != 0 && recipes[m] != 1) FEASM_FAIL(FEASM_EINVAL, "serve_run: bad recipe");
            if (!(p->flags & (fmt == FEASM_FMT_CSR ? FEASM_BUILD_CSR : FEASM_BUILD_CRAC)))
                FEASM_FAIL(FEASM_EINVAL, "serve_run: a mesh lacks the requested format");
            if ((int64_t)p->n * (p->n + 1) * 8 > 64 * 1024)
                FEASM_FAIL(FEASM_ELIMIT, "serve_run: element matrices too large for the generator");
            max_ke = std::max(max_ke, p->n_elem * p->n * p->n);
            max_nnz = std::max(max_nnz, p->nnz);
        }
        int64_t total_re = 0;
        for (int64_t r = 0; r < n_requests; ++r) {
            if (requests[r].mesh < 0 || requests[r].mesh >= n_meshes || requests[r].n_reassembly < 0)
                FEASM_FAIL(FEASM_EINVAL, "serve_run: bad request " + std::to_string(r));
            if (r > 0 && requests[r].arrival_s < requests[r - 1].arrival_s)
                FEASM_FAIL(FEASM_EINVAL, "serve_run: requests must be sorted by arrival");
            total_re += requests[r].n_reassembly;
        }
        (void)total_re;

        std::vector<Slot> slots(n_slots);
        const Allocator alloc = current_allocator();
        auto cleanup = [&]() {
            for (Slot& s : slots) {
                if (s.main) (void)hipStreamSynchronize(s.main);
                if (s.side) (void)hipStreamSynchronize(s.side);
                for (double* q : {s.ke[0], s.ke[1], s.values}) dev_free(alloc, q, nullptr);
                for (hipEvent_t e : {s.done, s.gen[0], s.gen[1]})
                    if (e) (void)hipEventDestroy(e);
                if (s.main) (void)hipStreamDestroy(s.main);
                if (s.side) (void)hipStreamDestroy(s.side);
            }
        };
        struct Guard {
            decltype(cleanup)& f;
            ~Guard() { f(); }
        } guard{cleanup};
        for (Slot& s : slots) {
            FEASM_HIP(hipStreamCreateWithFlags(&s.main, hipStreamNonBlocking));
            FEASM_HIP(hipStreamCreateWithFlags(&s.side, hipStreamNonBlocking));
            FEASM_HIP(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
            for (int b = 0; b < 2; ++b) {
                FEASM_HIP(hipEventCreateWithFlags(&s.gen[b], hipEventDisableTiming));
                const int rc = dev_alloc_n(alloc, &s.ke[b], max_ke, nullptr, "serve_run");
                if (rc != FEASM_OK) return rc;
            }
            const int rc = dev_alloc_n(alloc, &s.values, max_nnz, nullptr, "serve_run");
            if (rc != FEASM_OK) return rc;
        }
        // Each mesh's re-assembly state (lookup record or cache) is built before
        // the clock starts, by one re-assembly on the first slot's buffers, so
        // that no request pays for it inside the run.
        for (int64_t m = 0; m < n_meshes; ++m) {
            const int rc = reassemble_values(const_cast<feasm_pattern*>(meshes[m]), fmt, slots[0].ke[0],
                                             slots[0].values, FEASM_SCATTER_AUTO, slots[0].main);
            if (rc != FEASM_OK) return rc;
        }
        FEASM_HIP(hipStreamSynchronize(slots[0].main));
        // offsets of each request's re-assembly latencies in the flat output
        std::vector<int64_t> re_off(n_requests + 1, 0);
        for (int64_t r = 0; r < n_requests; ++r) re_off[r + 1] = re_off[r] + requests[r].n_reassembly;

        const auto t0 = clock::now();
        auto now_s = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
        auto footprint = [&](int64_t r) {
            const feasm_pattern* p = meshes[requests[r].mesh];
            return 2 * p->n_elem * p->n * p->n * 8 + p->nnz * 8;
        };
        auto generate = [&](Slot& s, int32_t it) -> int {
            const feasm_request& q = requests[s.req];
            const feasm_pattern* p = meshes[q.mesh];
            const int rc = generate_ke(recipes[q.mesh], p->n_elem, p->n, iteration_seed(q.seed, it), 0,
                                       s.ke[it % 2], s.side);
            if (rc != FEASM_OK) return rc;
            FEASM_HIP(hipEventRecord(s.gen[it % 2], s.side));
            return FEASM_OK;
        };
        auto issue = [&](Slot& s, double t) -> int {
            const feasm_request& q = requests[s.req];
            const feasm_pattern* p = meshes[q.mesh];
            FEASM_HIP(hipStreamWaitEvent(s.main, s.gen[s.it % 2], 0));
            int rc;
            if (s.it == 0)
                rc = assemble_on_stream(p, fmt, s.ke[0], s.values, FEASM_SCATTER_AUTO, s.main);
            else
                rc = reassemble_values(const_cast<feasm_pattern*>(p), fmt, s.ke[s.it % 2], s.values,
                                       FEASM_SCATTER_AUTO, s.main);
            if (rc != FEASM_OK) return rc;
            FEASM_HIP(hipEventRecord(s.done, s.main));
            s.issued = t;
            // the buffer of iteration it+1 was last read by iteration it-1, which
            // completed before this one was issued
            if (s.it + 1 <= q.n_reassembly) return generate(s, s.it + 1);
            return FEASM_OK;
        };

        std::deque<int64_t> pending;
        int64_t next_arrival = 0, finished = 0, in_use = 0, busy = 0;
        while (finished < n_requests) {
            double t = now_s();
            while (next_arrival < n_requests && requests[next_arrival].arrival_s <= t)
                pending.push_back(next_arrival++);
            bool progressed = false;
            for (Slot& s : slots) {
                if (s.req < 0) continue;
                const hipError_t q = hipEventQuery(s.done);
                if (q == hipErrorNotReady) continue;
                FEASM_HIP(q);
                progressed = true;
                t = now_s();
                feasm_request_result& res = results[s.req];
                const feasm_request& rq = requests[s.req];
                if (s.flushing) {
                    res.done_s = t;
                    in_use -= s.footprint;
                    s.req = -1;
                    s.flushing = false;
                    --busy;
                    ++finished;
                    continue;
                }
                if (s.it == 0)
                    res.assembled_s = t;
                else if (reassembly_latency)
                    reassembly_latency[re_off[s.req] + s.it - 1] = t - s.issued;
                if (s.it < rq.n_reassembly) {
                    ++s.it;
                    const int rc = issue(s, t);
                    if (rc != FEASM_OK) return rc;
                } else if (rq.keep_values) {
                    FEASM_HIP(hipMemcpyAsync(rq.keep_values, s.values,
                                             sizeof(double) * meshes[rq.mesh]->nnz,
                                             hipMemcpyDeviceToDevice, s.main));
                    FEASM_HIP(hipEventRecord(s.done, s.main));
                    s.flushing = true;
                } else {
                    res.done_s = t;
                    in_use -= s.footprint;
                    s.req = -1;
                    --busy;
                    ++finished;
                }
            }
            for (Slot& s : slots) {
                if (pending.empty()) break;
                if (s.req >= 0) continue;
                const int64_t r = pending.front();
                const int64_t fp = footprint(r);
                if (hbm_budget > 0 && in_use + fp > hbm_budget && busy > 0) break;
                pending.pop_front();
                t = now_s();
                results[r].admitted_s = t;
                s.req = r;
                s.it = 0;
                s.footprint = fp;
                s.flushing = false;
                in_use += fp;
                ++busy;
                int rc = generate(s, 0);
                if (rc == FEASM_OK) rc = issue(s, t);
                if (rc != FEASM_OK) return rc;
                progressed = true;
            }
            if (!progressed) {
                if (busy == 0 && pending.empty() && next_arrival < n_requests) {
                    const double wait = requests[next_arrival].arrival_s - now_s();
                    if (wait > 2e-4) std::this_thread::sleep_for(std::chrono::microseconds(100));
                } else {
                    std::this_thread::yield();
                }
            }
        }
        return FEASM_OK;
    });
}
