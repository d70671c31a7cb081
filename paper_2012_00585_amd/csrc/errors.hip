// Thread-local error message of the C ABI, and the guard that keeps C++
// exceptions inside the library.
#include "internal.h"

namespace feasm {

namespace {
thread_local std::string g_last_error;
// set when the message itself could not be stored (no host memory)
thread_local const char* g_fallback = nullptr;
}  // namespace

void set_error(const std::string& msg) noexcept {
    try {
        g_last_error = msg;
        g_fallback = nullptr;
    } catch (...) {
        g_fallback = "feasm: out of host memory while recording an error message";
    }
}

void set_error_for(const char* who, const char* what) noexcept {
    try {
        set_error(std::string(who) + ": " + what);
    } catch (...) {
        // `what` may belong to an exception object about to be destroyed
        g_fallback = "feasm: out of host memory while recording an error message";
    }
}

void set_error_literal(const char* msg) noexcept { g_fallback = msg; }

}  // namespace feasm

extern "C" const char* last_error(void) {
    return feasm::g_fallback ? feasm::g_fallback : feasm::g_last_error.c_str();
}
