// api.hip -- error reporting shared by every entry point of the C ABI.
#include <stdarg.h>
#include <stdio.h>

#include "common.hpp"

namespace n2v {

static thread_local char g_last_error[512] = "no error";

int set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return set_error(N2V_EDEVICE, "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
}

}  // namespace n2v

extern "C" const char *n2v_last_error(void) { return n2v::g_last_error; }

extern "C" int n2v_abi_version(void) { return N2V_ABI_VERSION; }
