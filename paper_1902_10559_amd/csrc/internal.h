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

// Checks a system's line orders: row_lanes in {0, 8, 16, 32, 64} (a row is
// read by 64/rows_per_wave lanes, rows_per_wave <= 8), col_lanes in {0, 4,
// 8, 16, 32, 64}.
inline ss_status check_lanes(const ss_system* S, const char* fn) {
  auto ok = [](int v, int lo) { return v == 0 || (v >= lo && v <= 64 && (v & (v - 1)) == 0); };
  if (!ok(S->row_lanes, 8) || !ok(S->col_lanes, 4))
    return fail(SS_E_ARG, "%s: row_lanes must be 0, 8, 16, 32 or 64 and col_lanes 0, 4, 8, 16, 32 or 64", fn);
  return SS_OK;
}

// For the consumers that need each line's entries in ascending order.
inline ss_status check_ascending(const ss_system* S, const char* fn) {
  if (S->row_lanes || S->col_lanes)
    return fail(SS_E_ARG, "%s: needs lines in ascending order (row_lanes = col_lanes = 0)", fn);
  return SS_OK;
}

}  // namespace ss
