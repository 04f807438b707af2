// Error reporting and version of libabc.so.
#include <stdarg.h>
#include <stdio.h>

#include "common.hpp"

namespace abc {

static thread_local char g_last_error[512] = "";

abc_status set_error(abc_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return st;
}

}  // namespace abc

extern "C" const char* abc_last_error(void) { return abc::g_last_error; }

extern "C" const char* abc_version(void) { return "abc-mi355x 0.1 (gfx950)"; }
