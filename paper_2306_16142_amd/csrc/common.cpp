// Thread-local error message and version entry points of the C ABI.
#include <cstdarg>
#include <cstdio>
#include <string>

#include "common.hpp"

namespace ddf {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

}  // namespace ddf

extern "C" int32_t ddf_abi_version(void) { return DDF_ABI_VERSION; }
extern "C" const char *ddf_last_error(void) { return ddf::g_last_error.c_str(); }
