// Host-side error text, version and launch checking.
#include <cstdarg>
#include <cstdio>

#include "common.hpp"

namespace mimo {

static thread_local char g_err[512] = "";

int32_t fail(int32_t code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int32_t check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MIMO_ERR_HIP, "%s: launch failed: %s", what, hipGetErrorString(e));
    return MIMO_OK;
}

}  // namespace mimo

extern "C" const char* mimo_last_error(void) { return mimo::g_err; }

extern "C" int32_t mimo_version(void) { return 1; }
