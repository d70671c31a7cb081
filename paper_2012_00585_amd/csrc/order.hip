// Node order for the row-owned kernels: light nodes (at most kLightInc
// incident entries) first, then the others, each part in increasing node
// id.  Light rows then run with the single-batch kernel and the rest with
// the looping one, and within each part consecutive wavefronts still write
// neighbouring value rows (ordering the rows by element instead makes the
// value writes scattered, which measured slower).
//
// The order is a stable two-way partition: one exclusive scan of the light
// flags gives every light node its position, and a heavy node v goes to
// n_light + (v - light nodes before v).
#include <algorithm>

#include "internal.h"

namespace feasm {
namespace {

__global__ void k_light_flags(const int64_t* __restrict__ inc_ptr, int64_t n_nodes,
                              int32_t* __restrict__ light) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n_nodes;
         v += (int64_t)gridDim.x * blockDim.x)
        light[v] = inc_ptr[v + 1] - inc_ptr[v] <= kLightInc ? 1 : 0;
}

__global__ void k_partition(const int32_t* __restrict__ light, const int64_t* __restrict__ before,
                            int64_t n_nodes, int32_t* __restrict__ order) {
    const int64_t n_light = before[n_nodes];
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n_nodes;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pos = light[v] ? before[v] : n_light + (v - before[v]);
        order[pos] = (int32_t)v;
    }
}

}  // namespace

int build_node_order(feasm_pattern* p, hipStream_t s, int64_t* n_light_host) {
    const int64_t nn = p->n_nodes;
    if (nn <= 0) {
        *n_light_host = 0;
        return FEASM_OK;
    }
    if (nn >= (1ll << 31)) FEASM_FAIL(FEASM_EOVERFLOW, "pattern_build: too many nodes to order");
    const char* who = "pattern_build (node order)";
    int32_t* light = nullptr;
    int64_t *before = nullptr, *scratch = nullptr;
    int rc = dev_alloc_n(p->alloc, &light, nn, s, who);
    if (rc == FEASM_OK) rc = dev_alloc_n(p->alloc, &before, nn + 1, s, who);
    if (rc == FEASM_OK) rc = dev_alloc_n(p->alloc, &scratch, scan_scratch_elems(nn), s, who);
    if (rc == FEASM_OK) rc = dev_alloc_n(p->alloc, &p->node_order, nn, s, who);
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(nn, 256), 65536);
    hipError_t e = hipSuccess;
    if (rc == FEASM_OK) {
        k_light_flags<<<grid, 256, 0, s>>>(p->inc_ptr, nn, light);
        e = hipGetLastError();
    }
    if (rc == FEASM_OK && e == hipSuccess) rc = exclusive_scan<int32_t>(light, nn, before, scratch, s);
    if (rc == FEASM_OK && e == hipSuccess) {
        k_partition<<<grid, 256, 0, s>>>(light, before, nn, p->node_order);
        e = hipGetLastError();
    }
    if (rc == FEASM_OK && e == hipSuccess)
        e = hipMemcpyAsync(n_light_host, before + nn, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (rc == FEASM_OK && e == hipSuccess) e = hipStreamSynchronize(s);
    if (rc == FEASM_OK && e != hipSuccess) {
        set_error(std::string("build_node_order: ") + hipGetErrorString(e));
        rc = e == hipErrorOutOfMemory ? FEASM_ENOMEM : FEASM_EHIP;
    }
    if (rc != FEASM_OK) (void)hipStreamSynchronize(s);
    for (void* q : {(void*)light, (void*)before, (void*)scratch}) dev_free(p->alloc, q, s);
    return rc;
}

}  // namespace feasm
