// Internal helpers shared by the library's translation units.
#pragma once

#include <cstdarg>
#include <cstdint>

#include "ssart.h"

namespace ss {

// Records `code` and a formatted message as the calling thread's last error
// and returns `code`.
ss_status fail(ss_status code, const char* fmt, ...);

// Clears the calling thread's last error (called on entry to every API call).
void clear_error();

inline bool is_pos(int64_t v) { return v > 0; }

}  // namespace ss
