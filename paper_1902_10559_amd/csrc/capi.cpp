// Error reporting and version for the C interface.
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace {
thread_local char g_last_error[512] = "";
}

namespace ss {

ss_status fail(ss_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_last_error[0] = '\0'; }

}  // namespace ss

extern "C" const char* ss_last_error(void) { return g_last_error; }

extern "C" const char* ss_version(void) { return "ssart 0.1 gfx950"; }

extern "C" int64_t ss_stream_len(int64_t nnz) {
  return nnz <= 0 ? 0 : (nnz + SS_CHUNK - 1) / SS_CHUNK * SS_CHUNK + SS_CHUNK;
}
