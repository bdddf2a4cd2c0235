// Thread-local error message and version string of libdopinf.
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/dopinf.h"

namespace dopinf {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace dopinf

extern "C" const char* dopinf_last_error(void) { return dopinf::g_last_error.c_str(); }

extern "C" const char* dopinf_version(void) { return "dopinf 0.1 gfx950"; }
