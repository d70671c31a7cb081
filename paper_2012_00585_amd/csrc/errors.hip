// Thread-local error message of the C ABI.
#include "internal.h"

namespace feasm {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace feasm

extern "C" const char* last_error(void) { return feasm::g_last_error.c_str(); }
