// Copies of line lists (CSR rows or CSC columns) in the interleaved order
// that line_dot_i reads (lines.h), for the solvers whose lines are stored in
// ascending order: one wavefront per line, each entry moved with its value
// bit for bit, so the copy holds the same entries (the line offsets do not
// change).
#pragma once

#include "device.h"
#include "internal.h"
#include "lines.h"

namespace ss {
namespace {

constexpr int kIlvWaves = 4;  // lines per block

// VB: value bytes per entry (4 or 8); L: lanes per line of the reading
// kernel.
template <int VB>
__global__ __launch_bounds__(kWave* kIlvWaves) void k_interleave(const int64_t* __restrict__ ptr, int64_t lines,
                                                                 const int32_t* __restrict__ idx,
                                                                 const void* __restrict__ val,
                                                                 int32_t* __restrict__ idx_out,
                                                                 void* __restrict__ val_out, int L) {
  const int64_t line = static_cast<int64_t>(blockIdx.x) * kIlvWaves + wave_id();
  if (line >= lines) return;
  const int64_t lo = gl(ptr)[line], n = gl(ptr)[line + 1] - lo;
  for (int64_t e = lane_id(); e < n; e += kWave) {
    const int64_t d = lo + interleaved_pos(e, n, L);
    glw(idx_out)[d] = gl(idx)[lo + e];
    if constexpr (VB == 8)
      glw(static_cast<uint64_t*>(val_out))[d] = gl(static_cast<const uint64_t*>(val))[lo + e];
    else
      glw(static_cast<uint32_t*>(val_out))[d] = gl(static_cast<const uint32_t*>(val))[lo + e];
  }
}

// The copy of `lines` lines (offsets ptr[0 .. lines]) for groups of L lanes;
// vb: value bytes per entry (4 or 8).
inline ss_status interleave_lines(const int64_t* ptr, int64_t lines, const int32_t* idx, const void* val,
                                  int32_t* idx_out, void* val_out, size_t vb, int L, hipStream_t st) {
  const int64_t blocks = (lines + kIlvWaves - 1) / kIlvWaves;
  if (blocks > INT32_MAX) return fail(SS_E_ARG, "too many lines to interleave");
  if (vb == 8)
    k_interleave<8><<<static_cast<uint32_t>(blocks), kWave * kIlvWaves, 0, st>>>(ptr, lines, idx, val, idx_out,
                                                                                   val_out, L);
  else
    k_interleave<4><<<static_cast<uint32_t>(blocks), kWave * kIlvWaves, 0, st>>>(ptr, lines, idx, val, idx_out,
                                                                                   val_out, L);
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

}  // namespace
}  // namespace ss
