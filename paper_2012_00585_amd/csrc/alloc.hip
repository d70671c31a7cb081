// Device memory of the library: hipMalloc / hipFree, or the allocator the
// caller installs with set_allocator.
#include <mutex>

#include "internal.h"

namespace feasm {

namespace {
std::mutex g_alloc_mutex;
Allocator g_alloc;
}  // namespace

Allocator current_allocator() {
    std::lock_guard<std::mutex> lock(g_alloc_mutex);
    return g_alloc;
}

int dev_alloc(const Allocator& a, void** ptr, size_t bytes, hipStream_t s, const char* who) {
    *ptr = nullptr;
    if (bytes == 0) bytes = 256;
    if (a.alloc) {
        void* q = a.alloc(bytes, s, a.ctx);
        if (!q) {
            set_error(std::string(who) + ": the installed allocator returned no memory for " +
                      std::to_string(bytes) + " bytes");
            return FEASM_ENOMEM;
        }
        *ptr = q;
        return FEASM_OK;
    }
    const hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        set_error(std::string(who) + ": hipMalloc(" + std::to_string(bytes) +
                  "): " + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FEASM_ENOMEM : FEASM_EHIP;
    }
    return FEASM_OK;
}

void dev_free(const Allocator& a, void* ptr, hipStream_t s) {
    if (!ptr) return;
    if (a.release)
        a.release(ptr, s, a.ctx);
    else
        (void)hipFree(ptr);
}

}  // namespace feasm

extern "C" int set_allocator(feasm_alloc_fn alloc, feasm_release_fn release, void* ctx) {
    return feasm::guarded("set_allocator", [&]() -> int {
        using namespace feasm;
        if ((alloc == nullptr) != (release == nullptr))
            FEASM_FAIL(FEASM_EINVAL, "set_allocator: give both alloc and release, or neither");
        std::lock_guard<std::mutex> lock(g_alloc_mutex);
        g_alloc.alloc = alloc;
        g_alloc.release = release;
        g_alloc.ctx = alloc ? ctx : nullptr;
        return FEASM_OK;
    });
}
