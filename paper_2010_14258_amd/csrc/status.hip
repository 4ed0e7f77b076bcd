// Status strings and the thread-local error message of the C ABI.
#include <cstdarg>
#include <cstdio>
#include <string>

#include "common.h"

namespace ldbp {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

}  // namespace ldbp

extern "C" const char* ldbp_version(void) { return "ldbp-gfx950 0.1"; }

extern "C" const char* ldbp_last_error(void) { return ldbp::g_last_error.c_str(); }

extern "C" const char* ldbp_status_string(int status) {
  switch (status) {
    case LDBP_OK: return "ok";
    case LDBP_EINVAL: return "invalid argument";
    case LDBP_EWORKSPACE: return "workspace too small";
    case LDBP_EUNSUPPORTED: return "unsupported";
    case LDBP_EHIP: return "HIP runtime error";
    case LDBP_ENONFINITE: return "non-finite output";
    default: return "unknown status";
  }
}
