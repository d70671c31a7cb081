// Native serving engine: assembly + Newton-style re-assembly requests as
// they arrive, with continuous batching.
//
// One host thread runs the loop.  Requests arrive at given times; the FIFO
// head is admitted into a free slot once the HBM budget (sum of admitted
// footprints: the slot's element-matrix buffers plus one values buffer)
// allows.  Each slot has a stream for assembly and a side stream on which
// the next iteration's element matrices are generated (ping-pong buffers)
// while the current iteration assembles; a mesh may instead bring a pool of
// pre-generated element matrices, read in place.  A slot issues its next
// iteration as soon as it sees the previous one complete (a Newton loop with
// zero solver time), so the work of every admitted request overlaps on the
// device.
//
// Patterns: a mesh either comes with a resident handle of the caller, or the
// engine builds its pattern (pattern_build) on the first request that needs
// it and keeps it in a cache bounded in bytes, evicting the least recently
// used patterns that no admitted request is using.  A miss stalls the loop
// for the build (pattern_build and the first re-assembly synchronise).
//
// Times: admission is host time since the start; completion times and
// latencies come from timing events on the device, relative to an event
// recorded at the start.
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
    hipEvent_t issue = nullptr;  // before the wait for the element matrices
    hipEvent_t start = nullptr;  // the assembly starts
    hipEvent_t done = nullptr;
    hipEvent_t gen_begin[2] = {nullptr, nullptr};
    hipEvent_t gen[2] = {nullptr, nullptr};
    bool generated[2] = {false, false};
    double* ke[2] = {nullptr, nullptr};
    int64_t ke_cap = 0;  // doubles per element-matrix buffer
    double* values = nullptr;
    int64_t values_cap = 0;
    int64_t req = -1;
    int32_t it = 0;
    bool flushing = false;  // final copy-out in flight
    int64_t footprint = 0;
    const feasm_pattern* p = nullptr;
};

struct CacheEntry {
    feasm_pattern* p = nullptr;  // built by the engine
    int64_t bytes = 0;
    int64_t last = 0;
    int32_t in_use = 0;
};

int64_t pattern_bytes(const feasm_pattern* p) {
    const int64_t nn = p->n_nodes, ek = p->n_elem * p->k;
    int64_t b = ek * 4 * 4;                            // conn and three incidence arrays
    b += (nn + 1) * 8 * 3 + nn * 4 * 2 + p->node_nnz * 4;  // node pattern, runs, order
    b += (p->n_rows + 1) * 4;                         // row_ptr
    if (p->col_idx) b += p->nnz * 4;
    if (p->ca) b += (p->n_rows + 1) * 4 + p->n_ca * 4;
    if (p->owner_map) b += ek * p->k * 4;
    return b;
}

}  // namespace
}  // namespace feasm

extern "C" int serve_run(const feasm_serve_mesh* meshes, int64_t n_meshes,
                         const feasm_request* requests, int64_t n_requests,
                         const feasm_serve_config* cfg, feasm_request_result* results,
                         double* reassembly_latency, feasm_serve_stats* stats) {
    return feasm::guarded("serve_run", [&]() -> int {
        using namespace feasm;
        using clock = std::chrono::steady_clock;
        if (!meshes || !cfg || n_meshes <= 0 || (n_requests > 0 && (!requests || !results)))
            FEASM_FAIL(FEASM_EINVAL, "serve_run: null argument");
        const int fmt = cfg->fmt;
        const int32_t n_slots = cfg->slots;
        if (n_slots <= 0 || n_slots > 256) FEASM_FAIL(FEASM_EINVAL, "serve_run: slots must be in [1, 256]");
        if (fmt != FEASM_FMT_CSR && fmt != FEASM_FMT_CRAC)
            FEASM_FAIL(FEASM_EINVAL, "serve_run: fmt must be FEASM_FMT_CSR or FEASM_FMT_CRAC");
        const uint32_t fmt_flag = fmt == FEASM_FMT_CSR ? FEASM_BUILD_CSR : FEASM_BUILD_CRAC;
        int64_t max_gen = 0;
        for (int64_t m = 0; m < n_meshes; ++m) {
            const feasm_serve_mesh& M = meshes[m];
            if (M.pattern) {
                if (!(M.pattern->flags & fmt_flag))
                    FEASM_FAIL(FEASM_EINVAL, "serve_run: a mesh's pattern lacks the requested format");
                if (M.pattern->n_elem != M.n_elem || M.pattern->k != M.nodes_per_elem ||
                    M.pattern->d != M.dofs_per_node)
                    FEASM_FAIL(FEASM_EINVAL, "serve_run: a mesh's sizes differ from its pattern's");
            } else if (!M.conn) {
                FEASM_FAIL(FEASM_EINVAL, "serve_run: a mesh has neither a pattern nor a connectivity");
            }
            if (M.n_elem <= 0 || M.nodes_per_elem <= 0 || M.dofs_per_node <= 0 || M.n_nodes <= 0)
                FEASM_FAIL(FEASM_EINVAL, "serve_run: mesh sizes must be positive");
            const int64_t n = (int64_t)M.nodes_per_elem * M.dofs_per_node;
            if (M.ke_pool) {
                if (M.pool_size <= 0) FEASM_FAIL(FEASM_EINVAL, "serve_run: pool_size must be positive");
            } else {
                if (M.recipe != 0 && M.recipe != 1) FEASM_FAIL(FEASM_EINVAL, "serve_run: bad recipe");
                if (n * (n + 1) * 8 > 64 * 1024)
                    FEASM_FAIL(FEASM_ELIMIT, "serve_run: element matrices too large for the generator");
                max_gen = std::max(max_gen, M.n_elem * n * n);
            }
        }
        for (int64_t r = 0; r < n_requests; ++r) {
            if (requests[r].mesh < 0 || requests[r].mesh >= n_meshes || requests[r].n_reassembly < 0)
                FEASM_FAIL(FEASM_EINVAL, "serve_run: bad request " + std::to_string(r));
            if (r > 0 && requests[r].arrival_s < requests[r - 1].arrival_s)
                FEASM_FAIL(FEASM_EINVAL, "serve_run: requests must be sorted by arrival");
        }
        feasm_serve_stats st{};

        std::vector<Slot> slots(n_slots);
        std::vector<CacheEntry> cache(n_meshes);
        hipEvent_t t0_event = nullptr;
        const Allocator alloc = current_allocator();
        auto cleanup = [&]() {
            for (Slot& s : slots) {
                if (s.main) (void)hipStreamSynchronize(s.main);
                if (s.side) (void)hipStreamSynchronize(s.side);
            }
            for (Slot& s : slots) {
                for (double* q : {s.ke[0], s.ke[1], s.values}) dev_free(alloc, q, nullptr);
                for (hipEvent_t e : {s.issue, s.start, s.done, s.gen_begin[0], s.gen_begin[1], s.gen[0],
                                     s.gen[1]})
                    if (e) (void)hipEventDestroy(e);
                if (s.main) (void)hipStreamDestroy(s.main);
                if (s.side) (void)hipStreamDestroy(s.side);
            }
            for (CacheEntry& c : cache)
                if (c.p) {
                    release_pattern(c.p);
                    delete c.p;
                    c.p = nullptr;
                }
            if (t0_event) (void)hipEventDestroy(t0_event);
        };
        struct Guard {
            decltype(cleanup)& f;
            ~Guard() { f(); }
        } guard{cleanup};
        for (Slot& s : slots) {
            FEASM_HIP(hipStreamCreateWithFlags(&s.main, hipStreamNonBlocking));
            FEASM_HIP(hipStreamCreateWithFlags(&s.side, hipStreamNonBlocking));
            for (hipEvent_t* e : {&s.issue, &s.start, &s.done, &s.gen_begin[0], &s.gen_begin[1],
                                  &s.gen[0], &s.gen[1]})
                FEASM_HIP(hipEventCreate(e));
            if (max_gen > 0)
                for (int b = 0; b < 2; ++b) {
                    const int rc = dev_alloc_n(alloc, &s.ke[b], max_gen, nullptr, "serve_run");
                    if (rc != FEASM_OK) return rc;
                }
            s.ke_cap = max_gen;
        }
        FEASM_HIP(hipEventCreate(&t0_event));
        // re-assembly state of the caller's resident patterns, before the clock
        {
            Slot& s0 = slots[0];
            for (int64_t m = 0; m < n_meshes; ++m) {
                const feasm_pattern* p = meshes[m].pattern;
                if (!p) continue;
                if (s0.values_cap < p->nnz) {
                    dev_free(alloc, s0.values, nullptr);
                    s0.values = nullptr;
                    s0.values_cap = 0;
                    const int rc = dev_alloc_n(alloc, &s0.values, p->nnz, nullptr, "serve_run");
                    if (rc != FEASM_OK) return rc;
                    s0.values_cap = p->nnz;
                }
                const double* ke = meshes[m].ke_pool ? meshes[m].ke_pool : s0.ke[0];
                const int rc = reassemble_values(const_cast<feasm_pattern*>(p), fmt, ke, s0.values,
                                                 FEASM_SCATTER_AUTO, s0.main);
                if (rc != FEASM_OK) return rc;
            }
            FEASM_HIP(hipStreamSynchronize(s0.main));
        }
        std::vector<int64_t> re_off(n_requests + 1, 0);
        for (int64_t r = 0; r < n_requests; ++r) re_off[r + 1] = re_off[r] + requests[r].n_reassembly;

        const auto t0 = clock::now();
        FEASM_HIP(hipEventRecord(t0_event, slots[0].main));
        auto now_s = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
        auto since_start = [&](hipEvent_t e, double* out) -> int {
            float ms = 0.f;
            FEASM_HIP(hipEventElapsedTime(&ms, t0_event, e));
            *out = ms * 1e-3;
            return FEASM_OK;
        };
        int64_t tick = 0, cache_total = 0;
        // the pattern of mesh m for a slot: the caller's, or the cache's
        // (built on a miss, evicting least recently used idle patterns)
        auto acquire = [&](int64_t m, Slot& s) -> int {
            if (meshes[m].pattern) {
                s.p = meshes[m].pattern;
                return FEASM_OK;
            }
            CacheEntry& c = cache[m];
            c.last = ++tick;
            if (c.p) {
                ++st.pattern_hits;
                ++c.in_use;
                s.p = c.p;
                return FEASM_OK;
            }
            ++st.pattern_misses;
            const auto b0 = clock::now();
            const feasm_serve_mesh& M = meshes[m];
            feasm_pattern* p = nullptr;
            int rc = pattern_build(M.conn, M.n_elem, M.nodes_per_elem, M.dofs_per_node, M.n_nodes,
                                   fmt_flag, s.main, &p);
            if (rc != FEASM_OK) return rc;
            c.p = p;
            // room for the values, then the re-assembly record (synchronises)
            if (s.values_cap < p->nnz) {
                FEASM_HIP(hipStreamSynchronize(s.main));
                dev_free(alloc, s.values, nullptr);
                s.values = nullptr;
                s.values_cap = 0;
                rc = dev_alloc_n(alloc, &s.values, p->nnz, nullptr, "serve_run");
                if (rc != FEASM_OK) return rc;
                s.values_cap = p->nnz;
            }
            const double* ke = M.ke_pool ? M.ke_pool : s.ke[0];
            rc = reassemble_values(p, fmt, ke, s.values, FEASM_SCATTER_AUTO, s.main);
            if (rc != FEASM_OK) return rc;
            FEASM_HIP(hipStreamSynchronize(s.main));
            st.pattern_build_s += std::chrono::duration<double>(clock::now() - b0).count();
            c.bytes = pattern_bytes(p);
            cache_total += c.bytes;
            c.in_use = 1;
            s.p = p;
            while (cfg->pattern_cache_bytes > 0 && cache_total > cfg->pattern_cache_bytes) {
                int64_t victim = -1;
                for (int64_t o = 0; o < n_meshes; ++o)
                    if (cache[o].p && cache[o].in_use == 0 &&
                        (victim < 0 || cache[o].last < cache[victim].last))
                        victim = o;
                if (victim < 0) break;  // every resident pattern is in use
                // no queued work reads it: its requests have completed
                release_pattern(cache[victim].p);
                delete cache[victim].p;
                cache[victim].p = nullptr;
                cache_total -= cache[victim].bytes;
                ++st.pattern_evictions;
            }
            st.pattern_cache_peak_bytes = std::max(st.pattern_cache_peak_bytes, cache_total);
            return FEASM_OK;
        };
        auto release = [&](int64_t m) {
            if (!meshes[m].pattern && cache[m].in_use > 0) --cache[m].in_use;
        };
        auto footprint = [&](int64_t r) {
            const feasm_serve_mesh& M = meshes[requests[r].mesh];
            const int64_t n = (int64_t)M.nodes_per_elem * M.dofs_per_node;
            const int64_t ke = M.ke_pool ? 0 : 2 * M.n_elem * n * n * 8;
            // the values of a pattern not built yet are bounded by the element entries
            const feasm_pattern* p = M.pattern ? M.pattern : cache[requests[r].mesh].p;
            return ke + (p ? p->nnz : M.n_elem * n * n) * 8;
        };
        auto ke_of = [&](Slot& s, int32_t it) -> const double* {
            const feasm_request& q = requests[s.req];
            const feasm_serve_mesh& M = meshes[q.mesh];
            if (M.ke_pool) {
                const int64_t block = M.n_elem * s.p->n * s.p->n;
                return M.ke_pool + (int64_t)((q.seed + (uint64_t)it) % (uint64_t)M.pool_size) * block;
            }
            return s.ke[it % 2];
        };
        auto generate = [&](Slot& s, int32_t it) -> int {
            const feasm_request& q = requests[s.req];
            const feasm_serve_mesh& M = meshes[q.mesh];
            if (M.ke_pool) return FEASM_OK;
            FEASM_HIP(hipEventRecord(s.gen_begin[it % 2], s.side));
            const int rc = generate_ke(M.recipe, M.n_elem, s.p->n, iteration_seed(q.seed, it), 0,
                                       s.ke[it % 2], s.side);
            if (rc != FEASM_OK) return rc;
            FEASM_HIP(hipEventRecord(s.gen[it % 2], s.side));
            s.generated[it % 2] = true;
            st.generated_bytes += M.n_elem * s.p->n * s.p->n * 8;
            return FEASM_OK;
        };
        auto issue = [&](Slot& s) -> int {
            const feasm_request& q = requests[s.req];
            FEASM_HIP(hipEventRecord(s.issue, s.main));
            if (!meshes[q.mesh].ke_pool) FEASM_HIP(hipStreamWaitEvent(s.main, s.gen[s.it % 2], 0));
            FEASM_HIP(hipEventRecord(s.start, s.main));
            int rc;
            if (s.it == 0)
                rc = assemble_on_stream(s.p, fmt, ke_of(s, 0), s.values, FEASM_SCATTER_AUTO, s.main);
            else
                rc = reassemble_values(const_cast<feasm_pattern*>(s.p), fmt, ke_of(s, s.it), s.values,
                                       FEASM_SCATTER_AUTO, s.main);
            if (rc != FEASM_OK) return rc;
            FEASM_HIP(hipEventRecord(s.done, s.main));
            // the buffer of iteration it+1 was last read by iteration it-1, which
            // completed before this one was issued
            if (s.it + 1 <= q.n_reassembly) return generate(s, s.it + 1);
            return FEASM_OK;
        };
        // device times of a completed iteration
        auto account = [&](Slot& s) -> int {
            float ms = 0.f;
            FEASM_HIP(hipEventElapsedTime(&ms, s.start, s.done));
            st.assemble_ms += ms;
            const int b = s.it % 2;
            if (s.generated[b]) {
                FEASM_HIP(hipEventElapsedTime(&ms, s.gen_begin[b], s.gen[b]));
                st.generate_ms += ms;
                s.generated[b] = false;
            }
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
                feasm_request_result& res = results[s.req];
                const feasm_request& rq = requests[s.req];
                auto finish = [&]() -> int {
                    const int rc = since_start(s.done, &res.done_s);
                    if (rc != FEASM_OK) return rc;
                    in_use -= s.footprint;
                    release(rq.mesh);
                    s.req = -1;
                    s.flushing = false;
                    --busy;
                    ++finished;
                    return FEASM_OK;
                };
                if (s.flushing) {
                    const int rc = finish();
                    if (rc != FEASM_OK) return rc;
                    continue;
                }
                int rc = account(s);
                if (rc != FEASM_OK) return rc;
                if (s.it == 0) {
                    rc = since_start(s.done, &res.assembled_s);
                } else if (reassembly_latency) {
                    float ms = 0.f;
                    FEASM_HIP(hipEventElapsedTime(&ms, s.issue, s.done));
                    reassembly_latency[re_off[s.req] + s.it - 1] = ms * 1e-3;
                }
                if (rc != FEASM_OK) return rc;
                if (s.it < rq.n_reassembly) {
                    ++s.it;
                    rc = issue(s);
                } else if (rq.keep_values) {
                    FEASM_HIP(hipMemcpyAsync(rq.keep_values, s.values, sizeof(double) * s.p->nnz,
                                             hipMemcpyDeviceToDevice, s.main));
                    FEASM_HIP(hipEventRecord(s.done, s.main));
                    s.flushing = true;
                } else {
                    rc = finish();
                }
                if (rc != FEASM_OK) return rc;
            }
            for (Slot& s : slots) {
                if (pending.empty()) break;
                if (s.req >= 0) continue;
                const int64_t r = pending.front();
                const int64_t fp = footprint(r);
                if (cfg->hbm_budget > 0 && in_use + fp > cfg->hbm_budget && busy > 0) break;
                pending.pop_front();
                results[r].admitted_s = now_s();
                s.req = r;
                s.it = 0;
                s.footprint = fp;
                s.flushing = false;
                in_use += fp;
                ++busy;
                int rc = acquire(requests[r].mesh, s);
                if (rc == FEASM_OK && s.values_cap < s.p->nnz) {
                    // a larger mesh than this slot has served: grow its values buffer
                    FEASM_HIP(hipStreamSynchronize(s.main));
                    dev_free(alloc, s.values, nullptr);
                    s.values = nullptr;
                    s.values_cap = 0;
                    rc = dev_alloc_n(alloc, &s.values, s.p->nnz, nullptr, "serve_run");
                    if (rc == FEASM_OK) s.values_cap = s.p->nnz;
                }
                if (rc == FEASM_OK) rc = generate(s, 0);
                if (rc == FEASM_OK) rc = issue(s);
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
        for (Slot& s : slots) FEASM_HIP(hipStreamSynchronize(s.main));
        for (const CacheEntry& c : cache)
            if (c.p) ++st.patterns_resident_at_end;
        if (stats) *stats = st;
        return FEASM_OK;
    });
}
