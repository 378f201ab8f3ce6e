// Sparse line sums shared by the solvers: one row (column) of a CSR (CSC)
// matrix against a dense vector, by a group of L lanes of a 64-lane
// wavefront, for one system (NV = 1) or the interleaved folded pair (NV = 2).
#pragma once

#include "device.h"

namespace ss {

// Workgroups are dealt round-robin to the 8 XCDs; this gives XCD x the
// contiguous logical range [start(x), start(x) + count(x)).
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nblocks) {
  const uint32_t x = b & 7u, q = b >> 3;
  const uint32_t per = nblocks >> 3, rem = nblocks & 7u;
  return x * per + (x < rem ? x : rem) + q;
}

// Index and value streams are read once per launch.  Plain loads: on gfx950
// the non-temporal hint measured slower for these streams (batched workload,
// one box, same shapes: 1.58 -> 1.40 ms forward, 1.78 -> 1.41 ms back).
__device__ inline int32_t ld_stream(const int32_t* p) { return *gl(p); }

// Entry-wise form of line_dot: lane g of a group takes entries lo + g,
// lo + g + L, ...: U entries per lane in flight per pass.  Adjacent lanes
// hold adjacent entries, so where a line's entries touch nearby positions of
// x (a ray crossing consecutive voxels) one gather instruction touches few
// cache lines.  Slots past the end of the line re-read its last entry (same
// cache line) and are masked out of the sum: with no branch around them, all
// 2U stream loads of a pass are issued before the first wait.
template <int NV, int WT, int L, int U>
__device__ inline void line_dot_e(const int32_t* idx, const void* val, const float* x, int64_t lo, int64_t hi,
                                int glane, float* acc) {
  for (int64_t base = lo + glane; base < hi; base += U * L) {
    int32_t c[U];
    Vec<NV> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = base + u * L;
      const int64_t kk = k < hi ? k : hi - 1;
      c[u] = ld_stream(idx + kk);
      v[u] = load_vals<NV, WT>(val, kk);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const Vec<NV> xv = load_vec<NV>(x, c[u]);
      const bool in = base + u * L < hi;
#pragma unroll
      for (int h = 0; h < NV; ++h) {
        const float s = fmaf(v[u].v[h], xv.v[h], acc[h]);
        acc[h] = in ? s : acc[h];
      }
    }
  }
}

// Sum over one line (row or column): acc += sum_k val[k] * x[idx[k]] for k in
// [lo, hi), by the L lanes of a group.  Chunked form: lanes take aligned
// chunks of SS_CHUNK entries (U chunks per lane per pass), a quarter of the
// stream load instructions of the entry-wise form, at the price of gathers
// that each touch more cache lines; entries of a chunk outside
// [lo, hi) are masked out.  Slots past the line's last chunk re-read that
// chunk, so every pass issues all its loads without a branch and never
// leaves the line's chunks: the arrays' capacity of ss_stream_len(nnz)
// entries covers the last chunk of the last line.
template <int NV, int WT, int L, int U>
__device__ inline void line_dot_c(const int32_t* idx, const void* val, const float* x, int64_t lo, int64_t hi,
                                int glane, float* acc) {
  constexpr int64_t C = SS_CHUNK;
  const int64_t first = lo & ~(C - 1);
  const int64_t last = (hi - 1) & ~(C - 1);
  for (int64_t base = first + C * glane; base < hi; base += C * U * L) {
    u32x4 c[U];
    Vec<NV> v[U][SS_CHUNK];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k0 = base + C * u * L;
      const int64_t kk = k0 <= last ? k0 : last;
      c[u] = load_idx_chunk(idx, kk);
      load_val_chunk<NV, WT>(val, kk, v[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int j = 0; j < SS_CHUNK; ++j) {
        const int64_t k = base + C * u * L + j;
        const bool in = k >= lo && k < hi;
        const Vec<NV> xv = load_vec<NV>(x, in ? static_cast<int32_t>(c[u][j]) : 0);
#pragma unroll
        for (int h = 0; h < NV; ++h) {
          const float sum = fmaf(v[u][j].v[h], xv.v[h], acc[h]);
          acc[h] = in ? sum : acc[h];
        }
      }
    }
  }
}

// Interleaved stream form.  A line of n entries is cut into blocks of
// SS_CHUNK * L entries (the last one shorter, r entries).  Within a block,
// lane g of the group takes the entries g, g + L, g + 2L, ... of the block
// (q = r / L of them, one more if g < r mod L), and they are stored
// consecutively, lane after lane: entry e of the block (lane e mod L, slot
// e / L) sits at position g*q + min(g, r mod L) + e / L.  One load of
// SS_CHUNK entries per lane then streams a block, as in the chunked form,
// while a gather instruction still has adjacent lanes on adjacent entries of
// the line, as in the entry-wise form.  The permutation stays inside each
// line, so the line offsets do not change.
// L is a power of two (4 .. 64): shifts and masks, not divisions.
static_assert(SS_CHUNK == 4, "interleaved_pos takes blocks of 4 entries per lane");
__host__ __device__ inline int64_t interleaved_pos(int64_t e, int64_t n, int L) {
  const int lg = __builtin_ctz(static_cast<unsigned>(L));
  const int lgB = lg + 2;  // SS_CHUNK = 4 entries per lane and block
  const int64_t B = int64_t{1} << lgB;
  const int64_t base = (e >> lgB) << lgB;
  const int64_t s = e - base;
  const int64_t r = n - base < B ? n - base : B;
  const int64_t q = r >> lg, rem = r & (L - 1);
  const int64_t g = s & (L - 1);
  return base + g * q + (g < rem ? g : rem) + (s >> lg);
}

// P blocks per pass.  Idle slots (past a lane's share of a block, or blocks
// past the line's last) are masked out.  A lane's load of SS_CHUNK entries
// starts at most at the end of its block, so the loads reach at most
// SS_CHUNK entries past the line's end: the interleaved copy of a stream
// has room for nnz + SS_CHUNK entries.
template <int NV, int WT, int L, int P>
__device__ inline void line_dot_i(const int32_t* idx, const void* val, const float* x, int64_t lo, int64_t hi,
                                  int glane, float* acc) {
  constexpr int B = SS_CHUNK * L;
  const int n = static_cast<int>(hi - lo);
  const int nb = (n + B - 1) / B;
  for (int b0 = 0; b0 < nb; b0 += P) {
    u32x4 c[P];
    Vec<NV> v[P][SS_CHUNK];
    int cnt[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int b = b0 + u < nb ? b0 + u : nb - 1;
      const int r = n - b * B < B ? n - b * B : B;
      const int q = r / L, rem = r % L;
      cnt[u] = b0 + u < nb ? q + (glane < rem ? 1 : 0) : 0;
      const int64_t k = lo + b * B + glane * q + (glane < rem ? glane : rem);
      c[u] = load_idx_at(idx, k);
      load_val_at<NV, WT>(val, k, v[u]);
    }
#pragma unroll
    for (int u = 0; u < P; ++u) {
#pragma unroll
      for (int j = 0; j < SS_CHUNK; ++j) {
        const bool in = j < cnt[u];
        const Vec<NV> xv = load_vec<NV>(x, in ? static_cast<int32_t>(c[u][j]) : 0);
#pragma unroll
        for (int h = 0; h < NV; ++h) {
          const float sum = fmaf(v[u][j].v[h], xv.v[h], acc[h]);
          acc[h] = in ? sum : acc[h];
        }
      }
    }
  }
}

// U entries per lane in flight per pass, entry-wise or in chunks (CH).
template <int NV, int WT, int L, int U, bool CH>
__device__ inline void line_dot(const int32_t* idx, const void* val, const float* x, int64_t lo, int64_t hi,
                                int glane, float* acc) {
  if constexpr (CH) line_dot_c<NV, WT, L, U / SS_CHUNK>(idx, val, x, lo, hi, glane, acc);
  else line_dot_e<NV, WT, L, U>(idx, val, x, lo, hi, glane, acc);
}

// Projection of the updated image onto f >= 0.  One system: clamp.  The
// folded pair: voxels j and N-1-j are (f2 + f1) / 2 and (f2 - f1) / 2 by
// eq. (5); clamp both and map back, which keeps f2 >= |f1| (halving and
// doubling are exact in FP32).
template <int NV>
__device__ inline Vec<NV> project_nonneg(Vec<NV> f) {
  if constexpr (NV == 1) {
    f.v[0] = fmaxf(f.v[0], 0.0f);
  } else {
    const float a = fmaxf(0.5f * (f.v[1] + f.v[0]), 0.0f);
    const float b = fmaxf(0.5f * (f.v[1] - f.v[0]), 0.0f);
    f.v[0] = a - b;
    f.v[1] = a + b;
  }
  return f;
}

}  // namespace ss
