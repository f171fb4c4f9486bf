// Error reporting and version query of the C ABI.
#include <stdarg.h>
#include <stdio.h>

#include "common.hpp"

namespace capvndf {

namespace {
thread_local char g_last_error[512] = "";
}

int32_t fail(int32_t code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return code;
}

int32_t check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return CAPVNDF_OK;
    return fail(CAPVNDF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int32_t check_launch(const char* what) { return check_hip(hipGetLastError(), what); }

int32_t check_array(const void* p, const char* name) {
    if (p == nullptr) return fail(CAPVNDF_ERR_NULL_PTR, "%s is NULL", name);
    if (!aligned_to(p, 4)) return fail(CAPVNDF_ERR_MISALIGNED, "%s is not 4-byte aligned", name);
    return CAPVNDF_OK;
}

}  // namespace capvndf

extern "C" int32_t capvndf_version(void) { return CAPVNDF_VERSION; }

extern "C" const char* capvndf_last_error(void) { return capvndf::g_last_error; }
