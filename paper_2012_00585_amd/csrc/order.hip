// Node order for the row-owned kernels: light nodes (at most kLightInc
// incident entries) first, then the others, each part in increasing node
// id.  Light rows then run with the single-batch kernel and the rest with
// the looping one, and within each part consecutive wavefronts still write
// neighbouring value rows (ordering the rows by element instead makes the
// value writes scattered, which measured slower).
#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace feasm {
namespace {

__global__ void k_order_keys(const int64_t* __restrict__ inc_ptr, int64_t n_nodes,
                             uint64_t* __restrict__ keys) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n_nodes;
         v += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t heavy = inc_ptr[v + 1] - inc_ptr[v] > kLightInc ? 1 : 0;
        keys[v] = (heavy << 62) | (uint64_t)v;
    }
}

__global__ void k_order_extract(const uint64_t* __restrict__ keys, int64_t n_nodes,
                                int32_t* __restrict__ order, int64_t* __restrict__ n_light) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_nodes;
         i += (int64_t)gridDim.x * blockDim.x) {
        order[i] = (int32_t)(keys[i] & 0x7FFFFFFFull);
        const bool heavy = (keys[i] >> 62) != 0;
        const bool prev_light = i == 0 || (keys[i - 1] >> 62) == 0;
        if (heavy && prev_light) *n_light = i;  // the first heavy position
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
    uint64_t *keys = nullptr, *sorted = nullptr;
    int64_t* d_light = nullptr;
    void* temp = nullptr;
    size_t temp_bytes = 0;
    int rc = FEASM_OK;
    auto fail = [&](hipError_t e) {
        set_error(std::string("build_node_order: ") + hipGetErrorString(e));
        rc = e == hipErrorOutOfMemory ? FEASM_ENOMEM : FEASM_EHIP;
    };
    const char* who = "pattern_build (node order)";
    rc = dev_alloc_n(p->alloc, &keys, nn, s, who);
    if (rc == FEASM_OK) rc = dev_alloc_n(p->alloc, &sorted, nn, s, who);
    if (rc == FEASM_OK) rc = dev_alloc_n(p->alloc, &d_light, 1, s, who);
    if (rc == FEASM_OK) rc = dev_alloc_n(p->alloc, &p->node_order, nn, s, who);
    hipError_t e = hipSuccess;
    if (rc == FEASM_OK)
        e = hipcub::DeviceRadixSort::SortKeys(nullptr, temp_bytes, keys, sorted, (int)nn, 0, 63, s);
    if (rc == FEASM_OK && e == hipSuccess) rc = dev_alloc(p->alloc, &temp, temp_bytes, s, who);
    if (rc != FEASM_OK) e = hipErrorOutOfMemory;
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(nn, 256), 65536);
    if (e == hipSuccess) {
        *n_light_host = nn;
        e = hipMemcpyAsync(d_light, n_light_host, sizeof(int64_t), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) {
        k_order_keys<<<grid, 256, 0, s>>>(p->inc_ptr, nn, keys);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortKeys(temp, temp_bytes, keys, sorted, (int)nn, 0, 63, s);
    if (e == hipSuccess) {
        k_order_extract<<<grid, 256, 0, s>>>(sorted, nn, p->node_order, d_light);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(n_light_host, d_light, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess && rc == FEASM_OK) fail(e);
    if (e != hipSuccess) (void)hipStreamSynchronize(s);
    for (void* q : {(void*)keys, (void*)sorted, (void*)d_light, temp}) dev_free(p->alloc, q, s);
    return rc;
}

}  // namespace feasm
