// Version and error reporting of the C ABI.
#include <stdarg.h>
#include <stdio.h>

#include "common.hpp"

namespace pgs {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

}  // namespace pgs

extern "C" const char* pgs_version(void) { return "pocketgs-gfx950 0.1"; }

extern "C" const char* pgs_last_error(void) { return pgs::g_err; }
