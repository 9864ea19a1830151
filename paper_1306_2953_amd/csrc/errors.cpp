// Error reporting across the C ABI: a thread-local message per failing call.
#include <string>

#include "internal.hpp"

namespace {
thread_local std::string g_last_error;
}

namespace rs {

void set_error(const std::string &msg) { g_last_error = msg; }

rs_status fail(rs_status code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

rs_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return RS_EHIP;
}

}  // namespace rs

extern "C" const char *rs_last_error(void) { return g_last_error.c_str(); }

extern "C" int rs_version(void) { return 1; }
