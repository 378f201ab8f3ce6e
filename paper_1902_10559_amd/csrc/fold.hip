// The fold of Section 2: A -> (A(1), A(2)) on one shared pattern, p -> (p1,
// p2), the SART normalisation sums, and the checks of eq. (2).
//
// Output row i (< m) of the pair is the union of two sorted index lists:
//   X = columns < n of row i of A,   Y = columns < n of row M-1-i of A,
// with v1 = a - b, v2 = a + b (a from X, b from Y, an absent term is +0.0).
// Output column j (< n) of the CSC copy is built column-locally from column j
// of A's CSC: X = its rows < m, Y = its rows >= m mapped to M-1-row (which
// reverses them into ascending order).  Both copies hold the same entries.
//
// A group of lanes (32 for a row pair, 8 for a column; a whole wavefront
// when the input is checked) merges one list pair, staged in shared memory.
// With dX[k] = 1 when X[k] is also in Y (dY likewise), and exclusive prefix
// counts of those flags taken with ballots (cut to the group's lanes):
//   union position of X[k]       = k + lower_bound(Y, X[k]) - prefix_dX[k]
//   union position of Y[l] not in X = lower_bound(X, Y[l]) + l - prefix_dY[l]
// (the union elements below a value are those of X and of Y below it, minus
// the common ones counted twice).  The union size is |X| + |Y| - #common.

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "device.h"
#include "internal.h"
#include "lines.h"

namespace ss {
namespace {

constexpr int kFoldWaves = 4;  // wavefronts per block; one list pair each

enum : uint32_t { kFlagAsym = 1u, kFlagShape = 2u, kFlagNonfinite = 4u };

struct FoldCheck {
  uint32_t flags;
  uint32_t pad;
  unsigned long long sum_csr, sum_csc;   // order-free checksums of entries
  unsigned long long cnt_csr, cnt_csc;   // union sizes from the two copies
};

// A sorted list of (index, value).  FLIP = true reads a stored ascending list
// backwards and maps each index t to base - t.
template <bool FLIP>
struct Seq {
  const int32_t* idx;
  const float* val;
  int64_t len;
  int32_t base;
  __device__ int32_t key(int64_t l) const {
    if constexpr (FLIP) return base - idx[len - 1 - l];
    else return idx[l];
  }
  __device__ float value(int64_t l) const {
    if constexpr (FLIP) return val[len - 1 - l];
    else return val[l];
  }
  // number of elements < k
  __device__ int64_t lower_bound(int32_t k) const {
    int64_t lo = 0, hi = len;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (key(mid) < k) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  }
};

__device__ inline int64_t lower_bound_idx(const int32_t* idx, int64_t len, int32_t k) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (idx[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The same list held in shared memory (address space 3, so that searches
// compile to LDS reads).
#define SS_LDS __attribute__((address_space(3)))
template <bool FLIP>
struct LSeq {
  const SS_LDS int32_t* idx;
  const SS_LDS float* val;
  int64_t len;
  int32_t base;
  __device__ int32_t key(int64_t l) const {
    if constexpr (FLIP) return base - idx[len - 1 - l];
    else return idx[l];
  }
  __device__ float value(int64_t l) const {
    if constexpr (FLIP) return val[len - 1 - l];
    else return val[l];
  }
  __device__ int64_t lower_bound(int32_t k) const {
    int64_t lo = 0, hi = len;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (key(mid) < k) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  }
};

// Lines are staged in shared memory by one coalesced pass, so that the
// per-element binary searches of the merge hit LDS instead of making
// dependent global loads: rows of up to kStageRow entries (two lists), columns
// of up to kStageCol entries; longer lines are merged from global memory.
// The buffers are sized for the lines of the workloads (rows up to ~400,
// columns up to ~80 entries in the batched workload) and small enough to
// keep 6 (rows: 768 entries per wavefront) or 8 (columns: 512) blocks per
// CU.
constexpr int kStageRow = 384;
constexpr int kStageCol = 256;

// The counting and filling passes can fold several lines per wavefront,
// each by a group of G lanes with its own part of the staging buffer: a
// short line (the batched workload's rows hold ~35 entries per list, its
// columns ~40 in all) would leave most of a wavefront idle behind the same
// chain of loads.  G is chosen per call from the mean line length (see
// pick_lanes): rows 32 or 64 lanes, columns 8, 16 or 64.  Measured on the
// batched workload (fold of 256 slices): 64 lanes per row and per column
// 20.3 ms, 32 per row and 16 per column 10.3 ms, 32 and 8 10.0 ms; 16 per
// row slowed the row fill (3.9 -> 5.8 ms).  On the polar grid (columns of
// ~420 entries) 8 lanes per column would stage nothing: whole wavefronts.
//
// Entries staged per group: columns 8 per lane (a whole column), rows 6 per
// lane and list; a wavefront per line (G = 64) keeps the larger buffers.
template <bool COLS, int G>
constexpr int stage_cap() {
  if constexpr (G == 64) return COLS ? kStageCol : kStageRow;
  else return COLS ? 8 * G : 6 * G;
}

// A sorted list of len (<= R * G) entries in registers, R per lane: all
// its loads are issued before the first is waited for, so a line pair costs
// one memory latency, not one per 64 entries.  VALS: also the values (the
// counting pass needs only the indices).
template <int R, bool VALS>
struct Staged {
  int32_t c[R];
  float v[R];
};

// A line is handled by a group of G lanes (G = 64: the whole wavefront;
// G < 64: the wavefront folds 64 / G lines at once).  Ballots are cut to
// the group's bits.
template <int G>
__device__ inline int group_lane() {
  return lane_id() & (G - 1);
}

template <int G>
__device__ inline uint64_t group_ballot(bool v) {
  const uint64_t b = __ballot(v);
  if constexpr (G == kWave) return b;
  else return (b >> (lane_id() & ~(G - 1))) & ((uint64_t{1} << G) - 1);
}

template <int G>
__device__ inline uint64_t group_lanemask_lt() {
  return (uint64_t{1} << group_lane<G>()) - 1;
}

template <int R, bool VALS, int G = kWave>
__device__ inline void stage_load(const int32_t* gi, const float* gv, int64_t len, Staged<R, VALS>& s) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t k = static_cast<int64_t>(r) * G + group_lane<G>();
    s.c[r] = INT32_MAX;
    if (k < len) {
      s.c[r] = gl(gi)[k];
      if constexpr (VALS) s.v[r] = gl(gv)[k];
    }
  }
}

// Writes the staged list to shared memory and returns how many of its
// indices are below `limit` (a prefix).
template <int G = kWave, int R, bool VALS>
__device__ inline int64_t stage_store(const Staged<R, VALS>& s, int64_t len, SS_LDS int32_t* si, SS_LDS float* sv,
                                      int32_t limit) {
  int64_t below = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t k = static_cast<int64_t>(r) * G + group_lane<G>();
    if (k < len) {
      si[k] = s.c[r];
      if constexpr (VALS) sv[k] = s.v[r];
    }
    below += __popcll(group_ballot<G>(s.c[r] < limit));
  }
  return below;
}

// Makes one wavefront's shared-memory writes visible to all its lanes.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Merges X and Y as described at the top of the file.  FILL writes every
// union entry at out_base + position: its index and the pair (a - b, a + b)
// in storage type WT.  With lanes > 0 the position within the line (of
// n_out entries) is permuted into the solver's interleaved order for groups
// of that many lanes.  Returns the union size (in every lane) and adds each
// entry's FP64 a + b to the lane's `sum`.
template <bool FILL, int WT, int G = kWave, class SX, class SY>
__device__ int64_t wave_merge(const SX& X, const SY& Y, int64_t out_base, int32_t* out_idx, void* out_val,
                              double& sum, int64_t n_out, int lanes) {
  const int lane = group_lane<G>();
  int64_t common = 0;
  for (int64_t base = 0; base < X.len; base += G) {
    const int64_t k = base + lane;
    const bool valid = k < X.len;
    int32_t x = 0;
    int64_t r = 0;
    bool dup = false;
    if (valid) {
      x = X.key(k);
      r = Y.lower_bound(x);
      dup = r < Y.len && Y.key(r) == x;
    }
    const uint64_t mask = group_ballot<G>(dup);
    if (FILL && valid) {
      const int64_t before = common + __popcll(mask & group_lanemask_lt<G>());
      const int64_t pos0 = k + r - before;
      const int64_t pos = lanes ? interleaved_pos(pos0, n_out, lanes) : pos0;
      const float a = X.value(k);
      const float b = dup ? Y.value(r) : 0.0f;
      out_idx[out_base + pos] = x;
      store_pair<WT>(out_val, out_base + pos, a - b, a + b);
      sum += static_cast<double>(a) + static_cast<double>(b);
    }
    common += __popcll(mask);
  }
  int64_t seen = 0;
  for (int64_t base = 0; base < Y.len; base += G) {
    const int64_t l = base + lane;
    const bool valid = l < Y.len;
    int32_t y = 0;
    int64_t s = 0;
    bool dup = false;
    if (valid) {
      y = Y.key(l);
      s = X.lower_bound(y);
      dup = s < X.len && X.key(s) == y;
    }
    const uint64_t mask = group_ballot<G>(dup);
    if (FILL && valid && !dup) {
      const int64_t before = seen + __popcll(mask & group_lanemask_lt<G>());
      const int64_t pos0 = s + l - before;
      const int64_t pos = lanes ? interleaved_pos(pos0, n_out, lanes) : pos0;
      const float b = Y.value(l);
      out_idx[out_base + pos] = y;
      store_pair<WT>(out_val, out_base + pos, 0.0f - b, 0.0f + b);
      sum += static_cast<double>(b);
    }
    seen += __popcll(mask);
  }
  return X.len + Y.len - common;
}

// The two lists of output row i (CSR side).
struct RowLists {
  Seq<false> X;
  Seq<false> Y;
};

__device__ inline RowLists row_lists(const ss_matrix_dev& A, int64_t i) {
  const int64_t n = A.N / 2;
  const int64_t rs = A.row_ptr[i], re = A.row_ptr[i + 1];
  const int64_t i2 = A.M - 1 - i;
  const int64_t ys = A.row_ptr[i2], ye = A.row_ptr[i2 + 1];
  RowLists L;
  L.X = {A.col_idx + rs, A.val + rs, lower_bound_idx(A.col_idx + rs, re - rs, static_cast<int32_t>(n)), 0};
  L.Y = {A.col_idx + ys, A.val + ys, lower_bound_idx(A.col_idx + ys, ye - ys, static_cast<int32_t>(n)), 0};
  return L;
}

// The two lists of output column j (CSC side).
struct ColLists {
  Seq<false> X;
  Seq<true> Y;
};

__device__ inline ColLists col_lists(const ss_matrix_dev& A, int64_t j) {
  const int64_t m = A.M / 2;
  const int64_t cs = A.col_ptr[j], ce = A.col_ptr[j + 1];
  const int64_t split = lower_bound_idx(A.row_idx + cs, ce - cs, static_cast<int32_t>(m));
  ColLists L;
  L.X = {A.row_idx + cs, A.val_t + cs, split, 0};
  L.Y = {A.row_idx + cs + split, A.val_t + cs + split, ce - cs - split, static_cast<int32_t>(A.M - 1)};
  return L;
}

// Per-wavefront staging buffers: two lists of kStageRow entries (the rows i
// and M-1-i), or one column of up to kStageCol entries.
struct StageBuf {
  SS_LDS int32_t* idx;
  SS_LDS float* val;
};

// Merges output line t (a row, or a column when COLS) into the union: its
// size, and with FILL the entries written at out_base.
// G: lanes per line (columns only may use 32: two columns per wavefront,
// each group with half of the wavefront's staging buffer).
template <bool COLS, bool FILL, int WT, int G = kWave>
__device__ int64_t fold_line(const ss_matrix_dev& A, int64_t t, int64_t out_base, int32_t* out_idx,
                             void* out_val, double& sum, StageBuf sb, int64_t n_out, int lanes) {
  if constexpr (COLS) {
    constexpr int cap = stage_cap<true, G>();
    const int64_t cs = gl(A.col_ptr)[t], ce = gl(A.col_ptr)[t + 1];
    const int64_t len = ce - cs;
    if (len <= cap) {
      Staged<cap / G, FILL> sl;
      stage_load<cap / G, FILL, G>(A.row_idx + cs, A.val_t + cs, len, sl);
      const int64_t split = stage_store<G>(sl, len, sb.idx, sb.val, static_cast<int32_t>(A.M / 2));
      wave_lds_sync();
      const LSeq<false> X{sb.idx, sb.val, split, 0};
      const LSeq<true> Y{sb.idx + split, sb.val + split, len - split, static_cast<int32_t>(A.M - 1)};
      return wave_merge<FILL, WT, G>(X, Y, out_base, out_idx, out_val, sum, n_out, lanes);
    }
    const ColLists L = col_lists(A, t);
    return wave_merge<FILL, WT, G>(L.X, L.Y, out_base, out_idx, out_val, sum, n_out, lanes);
  } else {
    constexpr int cap = stage_cap<false, G>();  // per list
    const int64_t t2 = A.M - 1 - t;
    const int64_t rs = gl(A.row_ptr)[t], re = gl(A.row_ptr)[t + 1];
    const int64_t ys = gl(A.row_ptr)[t2], ye = gl(A.row_ptr)[t2 + 1];
    if (re - rs <= cap && ye - ys <= cap) {
      const int32_t n = static_cast<int32_t>(A.N / 2);
      Staged<cap / G, FILL> sx, sy;
      stage_load<cap / G, FILL, G>(A.col_idx + rs, A.val + rs, re - rs, sx);
      stage_load<cap / G, FILL, G>(A.col_idx + ys, A.val + ys, ye - ys, sy);
      const int64_t xl = stage_store<G>(sx, re - rs, sb.idx, sb.val, n);
      const int64_t yl = stage_store<G>(sy, ye - ys, sb.idx + cap, sb.val + cap, n);
      wave_lds_sync();
      const LSeq<false> X{sb.idx, sb.val, xl, 0};
      const LSeq<false> Y{sb.idx + cap, sb.val + cap, yl, 0};
      return wave_merge<FILL, WT, G>(X, Y, out_base, out_idx, out_val, sum, n_out, lanes);
    }
    const RowLists L = row_lists(A, t);
    return wave_merge<FILL, WT, G>(L.X, L.Y, out_base, out_idx, out_val, sum, n_out, lanes);
  }
}

// This wavefront's staging buffers in the block's shared memory.
#define SS_STAGE_BUF(name)                                                        \
  constexpr int name##_cap = COLS ? std::max(kStageCol, 8 * kWave) : std::max(2 * kStageRow, 12 * kWave); \
  __shared__ int32_t name##_idx[kFoldWaves][name##_cap];                          \
  __shared__ float name##_val[kFoldWaves][name##_cap];                            \
  const StageBuf name{(SS_LDS int32_t*)(&name##_idx[wave_id()][0]), (SS_LDS float*)(&name##_val[wave_id()][0])}

// Group grp's part of the wavefront's staging buffer.
template <bool COLS, int G>
__device__ inline StageBuf group_buf(StageBuf sb, int grp) {
  constexpr int per = (COLS ? 1 : 2) * stage_cap<COLS, G>();
  if constexpr (G == kWave) return sb;
  else return StageBuf{sb.idx + grp * per, sb.val + grp * per};
}

__device__ inline unsigned long long mix64(unsigned long long z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__device__ inline unsigned long long entry_hash(int64_t i, int64_t j, float v) {
  return mix64((static_cast<unsigned long long>(i) << 32) ^ static_cast<unsigned long long>(j) ^
               mix64(__float_as_uint(v)));
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// One matrix of a fold and where its lines and scan tiles sit in the grids
// of the launches (a batch of matrices folds in one launch per phase).
struct FoldJob {
  ss_matrix_dev A;
  const float* p;
  ss_system out;
  int64_t rblk0, cblk0;    // first block of its rows / columns (line_blocks_for)
  int64_t rtile0, ctile0;  // first scan tile of its row / column offsets
};

// B = false: the job travels in the kernel arguments; B = true: a device
// table of `count` jobs ordered by their first blocks, and per grid (row
// lines, column lines, row scan tiles, column scan tiles) the job of each
// block, so that a block finds its job with one load.
struct JobArg {
  const FoldJob* table;
  int32_t count;
  const int32_t* b2j[4];
  FoldJob one;
};

// The job owning grid block b of the row (COLS false) or column lines, or of
// the scan tiles (TILES), and b's index within that job.
template <bool B, bool COLS, bool TILES>
__device__ inline const FoldJob& find_job(const JobArg& J, int64_t b, int64_t* local) {
  if constexpr (!B) {
    *local = b;
    return J.one;
  } else {
    auto first = [](const FoldJob& q) {
      return TILES ? (COLS ? q.ctile0 : q.rtile0) : (COLS ? q.cblk0 : q.rblk0);
    };
    const int k = __builtin_amdgcn_readfirstlane(gl(J.b2j[TILES ? (COLS ? 3 : 2) : (COLS ? 1 : 0)])[b]);
    *local = b - first(J.table[k]);
    return J.table[k];
  }
}

// Union size of every output line into ptr[t + 1]; ptr[0] = 0.
template <bool COLS, bool B, int G>
__global__ __launch_bounds__(kWave* kFoldWaves) void k_fold_count(JobArg J) {
  SS_STAGE_BUF(sb);
  int64_t lb;
  const FoldJob& jb = find_job<B, COLS, false>(J, blockIdx.x, &lb);
  const ss_matrix_dev& A = jb.A;
  const int64_t lines = COLS ? A.N / 2 : A.M / 2;
  const int grp = lane_id() / G;
  const int64_t t = (lb * kFoldWaves + wave_id()) * (kWave / G) + grp;
  if (t >= lines) return;
  double unused = 0.0;
  const int64_t cnt = fold_line<COLS, false, SS_F32, G>(A, t, 0, nullptr, nullptr, unused, group_buf<COLS, G>(sb, grp),
                                                       0, 0);
  int64_t* ptr = COLS ? jb.out.col_ptr : jb.out.row_ptr;
  if (group_lane<G>() == 0) {
    ptr[t + 1] = cnt;
    if (t == 0) ptr[0] = 0;
  }
}

// Per block of a check pass: the OR of its flags, the sum of its entry
// hashes and (rows) the sum of its union sizes.
struct CheckPart {
  uint32_t flags;
  uint32_t pad;
  unsigned long long hash;
  unsigned long long cnt;
};

// Checks of eq. (2) and of the arrays, one pair of mirrored lines (rows i
// and M-1-i, or columns j and N-1-j) per group of G lanes, with the lane
// groups and grids of the fold's counting pass: eq. (2) bitwise (equal
// lengths, mirrored indices, equal values), order, range and finiteness of
// both lines, an order-free checksum of the entries (the CSR and CSC copies
// must give the same), and for rows the size of the folded line (the same
// staged merge as the counting pass).  Each block writes one CheckPart; no
// atomics.
template <bool COLS, bool B, int G>
__global__ __launch_bounds__(kWave* kFoldWaves) void k_check_lines(JobArg J, CheckPart* parts) {
  SS_STAGE_BUF(sb);
  __shared__ CheckPart wp[kFoldWaves];
  int64_t lb;
  const FoldJob& jb = find_job<B, COLS, false>(J, blockIdx.x, &lb);
  const ss_matrix_dev& A = jb.A;
  const float* p = jb.p;
  const int64_t lines = COLS ? A.N : A.M;
  const int64_t other = COLS ? A.M : A.N;
  const int grp = lane_id() / G;
  const int lane = group_lane<G>();
  const int64_t t = (lb * kFoldWaves + wave_id()) * (kWave / G) + grp;
  const bool active = t < lines / 2;
  uint32_t flags = 0;
  unsigned long long h = 0;
  if (active) {
    const int64_t* ptr = COLS ? A.col_ptr : A.row_ptr;
    const int32_t* idx = COLS ? A.row_idx : A.col_idx;
    const float* val = COLS ? A.val_t : A.val;
    const int64_t t2 = lines - 1 - t;
    const int64_t as = gl(ptr)[t], ae = gl(ptr)[t + 1], bs = gl(ptr)[t2], be = gl(ptr)[t2 + 1];
    if (t == 0 && lane == 0 && (gl(ptr)[0] != 0 || gl(ptr)[lines] != A.nnz)) flags |= kFlagShape;
    const bool ranges_ok = as >= 0 && as <= ae && ae <= A.nnz && bs >= 0 && bs <= be && be <= A.nnz;
    if (!ranges_ok) {
      flags |= kFlagShape;
    } else {
      const int64_t la = ae - as, lbn = be - bs;
      if (la != lbn) flags |= kFlagAsym;
      for (int64_t k = lane; k < la; k += G) {
        const int32_t ca = gl(idx)[as + k];
        const float va = gl(val)[as + k];
        if (ca < 0 || ca >= other) flags |= kFlagShape;
        if (k + 1 < la && gl(idx)[as + k + 1] <= ca) flags |= kFlagShape;
        if (!isfinite(va)) flags |= kFlagNonfinite;
        h += COLS ? entry_hash(ca, t, va) : entry_hash(t, ca, va);
        if (la == lbn) {
          const int32_t cb = gl(idx)[bs + la - 1 - k];
          const float vb = gl(val)[bs + la - 1 - k];
          if (cb != other - 1 - ca || __float_as_uint(vb) != __float_as_uint(va)) flags |= kFlagAsym;
        }
      }
      for (int64_t k = lane; k < lbn; k += G) {
        const int32_t cb = gl(idx)[bs + k];
        const float vb = gl(val)[bs + k];
        if (cb < 0 || cb >= other) flags |= kFlagShape;
        if (k + 1 < lbn && gl(idx)[bs + k + 1] <= cb) flags |= kFlagShape;
        if (!isfinite(vb)) flags |= kFlagNonfinite;
        h += COLS ? entry_hash(cb, t2, vb) : entry_hash(t2, cb, vb);
      }
    }
    if (!COLS && p != nullptr && lane == 0 && (!isfinite(gl(p)[t]) || !isfinite(gl(p)[t2]))) flags |= kFlagNonfinite;
  }
  // the folded row's size, once the group's two rows are known to be sane
  unsigned long long cnt = 0;
  if constexpr (!COLS) {
    const bool sane = group_ballot<G>(active && (flags & kFlagShape) != 0) == 0;
    if (active && sane) {
      double unused = 0.0;
      const int64_t c = fold_line<false, false, SS_F32, G>(A, t, 0, nullptr, nullptr, unused,
                                                           group_buf<false, G>(sb, grp), 0, 0);
      if (lane == 0) cnt = static_cast<unsigned long long>(c);
    }
  }
  h = wave_sum_u64(h);
  cnt = wave_sum_u64(cnt);
  unsigned f = flags;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) f |= __shfl_xor(f, o, kWave);
  if (lane_id() == 0) wp[wave_id()] = CheckPart{f, 0u, h, cnt};
  __syncthreads();
  if (threadIdx.x == 0) {
    CheckPart r{0u, 0u, 0ull, 0ull};
    for (int w = 0; w < kFoldWaves; ++w) {
      r.flags |= wp[w].flags;
      r.hash += wp[w].hash;
      r.cnt += wp[w].cnt;
    }
    parts[blockIdx.x] = r;
  }
}

// Blocks of the counting, filling and check passes over `lines` line
// pairs or lines (kWave / G lines per wavefront).
__host__ __device__ inline int64_t line_blocks(int64_t lines, int G) {
  const int64_t per = kFoldWaves * (kWave / G);
  return (lines + per - 1) / per;
}

// One block per matrix: the check parts of both passes into its FoldCheck
// (integer sums and ORs: the order does not matter).  The size of the fold
// comes from the rows; the CSC copy is tied to the CSR by the checksums.
constexpr int kCheckFinThreads = 256;
template <bool B>
__global__ __launch_bounds__(kCheckFinThreads) void k_check_finish(JobArg J, const CheckPart* rparts,
                                                                   const CheckPart* cparts, int grow, int gcol,
                                                                   FoldCheck* out) {
  __shared__ uint32_t fl[kCheckFinThreads];
  __shared__ unsigned long long hr[kCheckFinThreads], hc[kCheckFinThreads], cr[kCheckFinThreads];
  const FoldJob& jb = B ? J.table[blockIdx.x] : J.one;
  const int64_t r0 = B ? jb.rblk0 : 0, c0 = B ? jb.cblk0 : 0;
  const int64_t rn = line_blocks(jb.A.M / 2, grow), cn = line_blocks(jb.A.N / 2, gcol);
  uint32_t f = 0;
  unsigned long long a = 0, c = 0, n = 0;
  for (int64_t b = threadIdx.x; b < rn; b += kCheckFinThreads) {
    f |= rparts[r0 + b].flags;
    a += rparts[r0 + b].hash;
    n += rparts[r0 + b].cnt;
  }
  for (int64_t b = threadIdx.x; b < cn; b += kCheckFinThreads) {
    f |= cparts[c0 + b].flags;
    c += cparts[c0 + b].hash;
  }
  fl[threadIdx.x] = f;
  hr[threadIdx.x] = a;
  hc[threadIdx.x] = c;
  cr[threadIdx.x] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    FoldCheck r{};
    for (int i = 0; i < kCheckFinThreads; ++i) {
      r.flags |= fl[i];
      r.sum_csr += hr[i];
      r.sum_csc += hc[i];
      r.cnt_csr += cr[i];
    }
    r.cnt_csc = r.cnt_csr;
    out[blockIdx.x] = r;
  }
}

// In-place inclusive scan of ptr[1..len] (ptr[0] = 0): ptr becomes the
// offsets array.  Two launches over tiles of kScanTile counts: each block
// first writes its tile's total; then each block adds the totals of the
// tiles before it (few: len / kScanTile) and scans its own tile in shared
// memory.  All loads are coalesced.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;

// Tiles of a job's offsets array: ptr[1..len], len = m (rows) or n (columns).
template <bool COLS>
__device__ inline void job_offsets(const FoldJob& jb, int64_t** ptr, int64_t* len) {
  *ptr = COLS ? jb.out.col_ptr : jb.out.row_ptr;
  *len = COLS ? jb.out.n : jb.out.m;
}

template <bool COLS, bool B>
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(JobArg J, int64_t* tile_sum) {
  int64_t lt;
  const FoldJob& jb = find_job<B, COLS, true>(J, blockIdx.x, &lt);
  int64_t* ptr;
  int64_t len;
  job_offsets<COLS>(jb, &ptr, &len);
  const int64_t base = 1 + lt * kScanTile;
  int64_t acc = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t i = base + threadIdx.x + static_cast<int64_t>(j) * kScanThreads;
    if (i <= len) acc += ptr[i];
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  __shared__ int64_t red[kScanThreads / kWave];
  if (lane_id() == 0) red[wave_id()] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) t += red[w];
    tile_sum[blockIdx.x] = t;
  }
}

// Each block adds the totals of its job's earlier tiles (few: len /
// kScanTile) and scans its own tile in shared memory.
template <bool COLS, bool B>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(JobArg J, const int64_t* tile_sum) {
  __shared__ int64_t vals[kScanTile];
  __shared__ int64_t tot[kScanThreads];
  __shared__ int64_t carry;
  int64_t lt;
  const FoldJob& jb = find_job<B, COLS, true>(J, blockIdx.x, &lt);
  int64_t* ptr;
  int64_t len;
  job_offsets<COLS>(jb, &ptr, &len);
  const int64_t base = 1 + lt * kScanTile;
  for (int j = 0; j < kScanPer; ++j) {
    const int t = threadIdx.x + j * kScanThreads;
    const int64_t i = base + t;
    vals[t] = i <= len ? ptr[i] : 0;
  }
  if (threadIdx.x == 0) {
    int64_t c = 0;
    for (int64_t b = static_cast<int64_t>(blockIdx.x) - lt; b < static_cast<int64_t>(blockIdx.x); ++b) c += tile_sum[b];
    carry = c;
  }
  __syncthreads();
  // each thread scans kScanPer consecutive counts
  int64_t run = 0;
  for (int j = 0; j < kScanPer; ++j) {
    run += vals[threadIdx.x * kScanPer + j];
    vals[threadIdx.x * kScanPer + j] = run;
  }
  tot[threadIdx.x] = run;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const int64_t v = threadIdx.x >= static_cast<unsigned>(o) ? tot[threadIdx.x - o] : 0;
    __syncthreads();
    tot[threadIdx.x] += v;
    __syncthreads();
  }
  const int64_t before = carry + (threadIdx.x > 0 ? tot[threadIdx.x - 1] : 0);
  for (int j = 0; j < kScanPer; ++j) vals[threadIdx.x * kScanPer + j] += before;
  __syncthreads();
  for (int j = 0; j < kScanPer; ++j) {
    const int t = threadIdx.x + j * kScanThreads;
    const int64_t i = base + t;
    if (i <= len) ptr[i] = vals[t];
  }
}

inline int64_t scan_tiles(int64_t len) { return (len + kScanTile - 1) / kScanTile; }

__device__ inline float recip_or_zero(double s) {
  return s != 0.0 ? static_cast<float>(1.0 / s) : 0.0f;
}

// Fills output rows (CSR side) or columns (CSC side) at the scanned offsets,
// with the FP32 reciprocal of the FP64 line sum of A (rows: W_i = sum over
// row i of A = sum of a + b over the union; columns: V_j likewise), and for
// rows also the folded p.
template <bool COLS, int WT, bool B, int G>
__global__ __launch_bounds__(kWave* kFoldWaves) void k_fold_fill(JobArg J) {
  SS_STAGE_BUF(sb);
  int64_t lb;
  const FoldJob& jb = find_job<B, COLS, false>(J, blockIdx.x, &lb);
  const ss_matrix_dev& A = jb.A;
  const ss_system& out = jb.out;
  const float* p = jb.p;
  const int64_t lines = COLS ? out.n : out.m;
  const int grp = lane_id() / G;
  const int64_t t = (lb * kFoldWaves + wave_id()) * (kWave / G) + grp;
  if (t >= lines) return;
  double sum = 0.0;
  if constexpr (COLS) {
    const int64_t o = out.col_ptr[t];
    fold_line<true, true, WT, G>(A, t, o, out.row_idx, out.val_t, sum, group_buf<COLS, G>(sb, grp),
                                 out.col_ptr[t + 1] - o, out.col_lanes);
  } else {
    const int64_t o = out.row_ptr[t];
    fold_line<false, true, WT, G>(A, t, o, out.col_idx, out.val, sum, group_buf<COLS, G>(sb, grp),
                                  out.row_ptr[t + 1] - o, out.row_lanes);
  }
  sum = group_sum<G>(sum);
  if (group_lane<G>() == 0) {
    if constexpr (COLS) {
      out.inv_col[t] = recip_or_zero(sum);
    } else {
      out.inv_row[t] = recip_or_zero(sum);
      const float a = p[t], b = p[A.M - 1 - t];
      reinterpret_cast<float2*>(out.p)[t] = make_float2(a - b, a + b);
    }
  }
}

// ---------------------------------------------------------------- unsplit
template <bool COLS>
__global__ __launch_bounds__(kWave* kFoldWaves) void k_line_recip(const int64_t* ptr, const float* val,
                                                                  int64_t lines, float* inv) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kFoldWaves + wave_id();
  if (t >= lines) return;
  double s = 0.0;
  for (int64_t k = ptr[t] + lane_id(); k < ptr[t + 1]; k += kWave) s += static_cast<double>(val[k]);
  s = group_sum<kWave>(s);
  if (lane_id() == 0) inv[t] = recip_or_zero(s);
}

template <int WT>
__global__ void k_convert(const float* src, int64_t count, void* dst) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < count) store_one<WT>(dst, k, src[k]);
}

__global__ void k_copy_f32(const float* src, int64_t count, float* dst) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < count) dst[k] = src[k];
}

inline unsigned blocks_for(int64_t lines) {
  return static_cast<unsigned>((lines + kFoldWaves - 1) / kFoldWaves);
}

// Blocks of the counting and filling passes (kWave / G lines per wavefront).
inline unsigned line_blocks_for(int64_t lines, int G) { return static_cast<unsigned>(line_blocks(lines, G)); }

// Lanes per line for one fold call, from the mean source-line lengths of all
// its matrices: a group is used where a mean row list fills half of its
// staging buffer, or a mean column three quarters of it, so that most lines
// are staged.
inline void pick_lanes(const ss_matrix_dev* A, int32_t count, int* grow, int* gcol) {
  double nnz = 0, M = 0, N = 0;
  for (int32_t k = 0; k < count; ++k) {
    nnz += static_cast<double>(A[k].nnz);
    M += static_cast<double>(A[k].M);
    N += static_cast<double>(A[k].N);
  }
  const double row = nnz / std::max(M, 1.0), col = nnz / std::max(N, 1.0);
  *grow = row <= 6.0 * 32 ? 32 : 64;  // a row pair: two lists of about row / 2
  *gcol = col <= 4.0 * 8 * 1.5 ? 8 : col <= 4.0 * 16 * 1.5 ? 16 : 64;
}

ss_status check_dev_matrix(const ss_matrix_dev* A, const char* fn) {
  if (!A || !A->row_ptr || !A->col_ptr) return fail(SS_E_ARG, "%s: NULL matrix array", fn);
  if (A->M <= 0 || A->N <= 0 || A->nnz < 0) return fail(SS_E_ARG, "%s: bad matrix size", fn);
  if (A->nnz > 0 && (!A->col_idx || !A->val || !A->row_idx || !A->val_t))
    return fail(SS_E_ARG, "%s: NULL matrix array", fn);
  if (A->M > INT32_MAX || A->N > INT32_MAX) return fail(SS_E_ARG, "%s: M and N must fit in int32", fn);
  return SS_OK;
}

// Jobs written into the device table from kernel arguments, kJobChunk per
// launch (no host-to-device copy of a pageable buffer).
constexpr int kJobChunk = 16;
struct JobChunk {
  FoldJob j[kJobChunk];
  int32_t count;
  int32_t first;
};

__global__ void k_put_jobs(JobChunk ch, FoldJob* table) {
  if (static_cast<int>(threadIdx.x) < ch.count) table[ch.first + threadIdx.x] = ch.j[threadIdx.x];
}

// The job of every block of the four batched grids (one block per job; the
// totals bound the last job's ranges).
__global__ void k_fill_b2j(const FoldJob* table, int32_t count, int64_t rblk, int64_t cblk, int64_t rtile,
                           int64_t ctile, int32_t* b_rows, int32_t* b_cols, int32_t* t_rows, int32_t* t_cols) {
  const int32_t k = static_cast<int32_t>(blockIdx.x);
  const FoldJob& q = table[k];
  const bool last = k + 1 == count;
  const int64_t r1 = last ? rblk : table[k + 1].rblk0, c1 = last ? cblk : table[k + 1].cblk0;
  const int64_t rt1 = last ? rtile : table[k + 1].rtile0, ct1 = last ? ctile : table[k + 1].ctile0;
  for (int64_t b = q.rblk0 + threadIdx.x; b < r1; b += blockDim.x) b_rows[b] = k;
  for (int64_t b = q.cblk0 + threadIdx.x; b < c1; b += blockDim.x) b_cols[b] = k;
  for (int64_t b = q.rtile0 + threadIdx.x; b < rt1; b += blockDim.x) t_rows[b] = k;
  for (int64_t b = q.ctile0 + threadIdx.x; b < ct1; b += blockDim.x) t_cols[b] = k;
}

// Grid sizes of one fold call: blocks of row and column lines, scan tiles.
struct FoldGrid {
  int64_t rblk = 0, cblk = 0, rtile = 0, ctile = 0;
  int grow = 64, gcol = 64;  // lanes per row pair / column
};

inline int64_t tiles_for(int64_t len) { return std::max<int64_t>(1, scan_tiles(len)); }

// count, scan and fill for rows, then for columns; tiles: scan scratch.
template <bool B>
void run_fold(const JobArg& J, const FoldGrid& g, int wt, int64_t* tiles, hipStream_t st) {
  const dim3 lb(kWave * kFoldWaves), sb(kScanThreads);
  const auto R = static_cast<unsigned>(g.rblk), Cb = static_cast<unsigned>(g.cblk);
  const auto RT = static_cast<unsigned>(g.rtile), CT = static_cast<unsigned>(g.ctile);
  auto count = [&](auto cols, auto g, unsigned blocks) {
    k_fold_count<decltype(cols)::value, B, decltype(g)::value><<<blocks, lb, 0, st>>>(J);
  };
  auto fill = [&](auto cols, auto g, unsigned blocks) {
    constexpr bool C = decltype(cols)::value;
    constexpr int G = decltype(g)::value;
    if (wt == SS_F32) k_fold_fill<C, SS_F32, B, G><<<blocks, lb, 0, st>>>(J);
    else if (wt == SS_BF16) k_fold_fill<C, SS_BF16, B, G><<<blocks, lb, 0, st>>>(J);
    else k_fold_fill<C, SS_F16, B, G><<<blocks, lb, 0, st>>>(J);
  };
  using Rows = std::false_type;
  using Cols = std::true_type;
  if (R > 0) {
    if (g.grow == 32) count(Rows{}, std::integral_constant<int, 32>{}, R);
    else count(Rows{}, std::integral_constant<int, 64>{}, R);
    k_scan_tiles<false, B><<<RT, sb, 0, st>>>(J, tiles);
    k_scan_apply<false, B><<<RT, sb, 0, st>>>(J, tiles);
    if (g.grow == 32) fill(Rows{}, std::integral_constant<int, 32>{}, R);
    else fill(Rows{}, std::integral_constant<int, 64>{}, R);
  }
  if (Cb > 0) {
    if (g.gcol == 8) count(Cols{}, std::integral_constant<int, 8>{}, Cb);
    else if (g.gcol == 16) count(Cols{}, std::integral_constant<int, 16>{}, Cb);
    else count(Cols{}, std::integral_constant<int, 64>{}, Cb);
    k_scan_tiles<true, B><<<CT, sb, 0, st>>>(J, tiles);
    k_scan_apply<true, B><<<CT, sb, 0, st>>>(J, tiles);
    if (g.gcol == 8) fill(Cols{}, std::integral_constant<int, 8>{}, Cb);
    else if (g.gcol == 16) fill(Cols{}, std::integral_constant<int, 16>{}, Cb);
    else fill(Cols{}, std::integral_constant<int, 64>{}, Cb);
  }
}

ss_status check_fold_out(const ss_matrix_dev* A, const float* p, const ss_system* out, const char* fn) {
  if (ss_status s = check_dev_matrix(A, fn)) return s;
  if (!p || !out) return fail(SS_E_ARG, "%s: NULL argument", fn);
  if (A->M % 2 || A->N % 2) return fail(SS_E_ODD, "%s: M and N must be even", fn);
  if (out->m != A->M / 2 || out->n != A->N / 2 || out->nvals != 2)
    return fail(SS_E_ARG, "%s: out must be m = M/2, n = N/2, nvals = 2", fn);
  if (out->wdtype != SS_F32 && out->wdtype != SS_BF16 && out->wdtype != SS_F16)
    return fail(SS_E_ARG, "%s: unknown wdtype %d", fn, out->wdtype);
  if (!out->row_ptr || !out->col_ptr || !out->p || !out->inv_row || !out->inv_col ||
      (out->nnz > 0 && (!out->col_idx || !out->val || !out->row_idx || !out->val_t)))
    return fail(SS_E_ARG, "%s: NULL output array", fn);
  if (ss_status s = check_lanes(out, fn)) return s;
  return SS_OK;
}

// Offsets of each job in the batched grids; returns the totals.
FoldGrid layout_jobs(const ss_matrix_dev* A, const float* const* p, const ss_system* out, int32_t count,
                     std::vector<FoldJob>* jobs) {
  FoldGrid g;
  pick_lanes(A, count, &g.grow, &g.gcol);
  for (int32_t k = 0; k < count; ++k) {
    FoldJob j{};
    j.A = A[k];
    j.p = p ? p[k] : nullptr;
    if (out) j.out = out[k];
    j.rblk0 = g.rblk;
    j.cblk0 = g.cblk;
    j.rtile0 = g.rtile;
    j.ctile0 = g.ctile;
    g.rblk += line_blocks_for(A[k].M / 2, g.grow);
    g.cblk += line_blocks_for(A[k].N / 2, g.gcol);
    g.rtile += tiles_for(A[k].M / 2);
    g.ctile += tiles_for(A[k].N / 2);
    if (jobs) jobs->push_back(j);
  }
  return g;
}

size_t batch_table_bytes(int32_t count) { return (sizeof(FoldJob) * static_cast<size_t>(count) + 255) & ~size_t{255}; }

inline size_t al256(size_t v) { return (v + 255) & ~size_t{255}; }

// The head of a batch's workspace: the job table, then the block -> job
// tables of the four grids.
size_t batch_head_bytes(int32_t count, const FoldGrid& g) {
  return batch_table_bytes(count) + al256(sizeof(int32_t) * static_cast<size_t>(g.rblk)) +
         al256(sizeof(int32_t) * static_cast<size_t>(g.cblk)) + al256(sizeof(int32_t) * static_cast<size_t>(g.rtile)) +
         al256(sizeof(int32_t) * static_cast<size_t>(g.ctile));
}

// Writes the job table and the block -> job tables into the workspace head
// and returns the kernels' argument.
JobArg put_batch(const std::vector<FoldJob>& jobs, const FoldGrid& g, char* ws, hipStream_t st) {
  const int32_t count = static_cast<int32_t>(jobs.size());
  FoldJob* table = reinterpret_cast<FoldJob*>(ws);
  for (int32_t k0 = 0; k0 < count; k0 += kJobChunk) {
    JobChunk ch{};
    ch.first = k0;
    ch.count = std::min(kJobChunk, count - k0);
    for (int i = 0; i < ch.count; ++i) ch.j[i] = jobs[k0 + i];
    k_put_jobs<<<1, kWave, 0, st>>>(ch, table);
  }
  JobArg J{};
  J.table = table;
  J.count = count;
  char* o = ws + batch_table_bytes(count);
  const int64_t sizes[4] = {g.rblk, g.cblk, g.rtile, g.ctile};
  int32_t* t[4];
  for (int k = 0; k < 4; ++k) {
    t[k] = reinterpret_cast<int32_t*>(o);
    J.b2j[k] = t[k];
    o += al256(sizeof(int32_t) * static_cast<size_t>(sizes[k]));
  }
  k_fill_b2j<<<static_cast<unsigned>(count), 256, 0, st>>>(table, count, g.rblk, g.cblk, g.rtile, g.ctile, t[0], t[1],
                                                           t[2], t[3]);
  return J;
}

// The checks of eq. (2) and of the arrays for every job: both passes over
// the line pairs with the fold's lane groups, then one block per job.
template <bool B>
void run_check(const JobArg& J, const FoldGrid& g, CheckPart* rparts, CheckPart* cparts, FoldCheck* out,
               int32_t count, hipStream_t st) {
  const dim3 lb(kWave * kFoldWaves);
  const auto R = static_cast<unsigned>(g.rblk), Cb = static_cast<unsigned>(g.cblk);
  if (g.grow == 32) k_check_lines<false, B, 32><<<R, lb, 0, st>>>(J, rparts);
  else k_check_lines<false, B, 64><<<R, lb, 0, st>>>(J, rparts);
  if (g.gcol == 8) k_check_lines<true, B, 8><<<Cb, lb, 0, st>>>(J, cparts);
  else if (g.gcol == 16) k_check_lines<true, B, 16><<<Cb, lb, 0, st>>>(J, cparts);
  else k_check_lines<true, B, 64><<<Cb, lb, 0, st>>>(J, cparts);
  k_check_finish<B><<<static_cast<unsigned>(count), kCheckFinThreads, 0, st>>>(J, rparts, cparts, g.grow, g.gcol, out);
}

// Turns one matrix's check record into a status and the fold's size.
ss_status check_verdict(const FoldCheck& h, const char* fn, int32_t k, int64_t* nnz_half) {
  if (h.flags & kFlagShape)
    return fail(SS_E_SHAPE, "%s: matrix %d: CSR/CSC offsets, order or index range invalid", fn, k);
  if (h.flags & kFlagNonfinite) return fail(SS_E_NONFINITE, "%s: matrix %d: NaN or Inf in A or p", fn, k);
  if (h.flags & kFlagAsym)
    return fail(SS_E_ASYM, "%s: matrix %d: A violates eq. (2), w[i,j] != w[M-1-i,N-1-j]", fn, k);
  if (h.sum_csr != h.sum_csc) return fail(SS_E_SHAPE, "%s: matrix %d: CSR and CSC hold different entries", fn, k);
  *nnz_half = static_cast<int64_t>(h.cnt_csr);
  return SS_OK;
}

// Check parts of the worst-case grids (a wavefront per line pair).
inline size_t check_parts_bytes(int64_t M, int64_t N) {
  return sizeof(CheckPart) * static_cast<size_t>(line_blocks(M / 2, kWave) + line_blocks(N / 2, kWave));
}

// ---------------------------------------------------- allocation-free fold
// ss_fold_noalloc keeps the scan's per-tile sums (its only scratch) in this
// file-scope array instead of a caller workspace.  Each device holds its own
// copy until the process ends.  In host code the name is only a stand-in for
// the symbol: kernels are given the device address that hipGetSymbolAddress
// returns for the current device, looked up once per device.
constexpr int64_t kNoallocTiles = 4096;  // 32 KiB: lines up to 4095 * kScanTile
static __device__ __align__(256) int64_t scratch[kNoallocTiles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int64_t* g_scratch_ptr[kMaxDevices] = {};

ss_status noalloc_scratch(int64_t** out) {
  int dev = 0;
  SS_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SS_E_ARG, "ss_fold_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SS_E_HIP, "ss_fold_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<int64_t*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return SS_OK;
}

}  // namespace
}  // namespace ss

using namespace ss;

extern "C" ss_status ss_fold_workspace_bytes(int64_t M, int64_t N, size_t* bytes) {
  clear_error();
  if (!bytes || M <= 0 || N <= 0) return fail(SS_E_ARG, "ss_fold_workspace_bytes: bad argument");
  const int64_t tiles = scan_tiles(std::max(M, N) / 2 + 1) + 1;
  *bytes = 512 + std::max(sizeof(int64_t) * static_cast<size_t>(tiles), check_parts_bytes(M, N));
  return SS_OK;
}

extern "C" ss_status ss_fold_size(const ss_matrix_dev* A, const float* p, void* workspace,
                                  size_t workspace_bytes, int64_t* nnz_half, void* stream) {
  clear_error();
  if (ss_status s = check_dev_matrix(A, "ss_fold_size")) return s;
  if (!nnz_half || !workspace) return fail(SS_E_ARG, "ss_fold_size: NULL argument");
  if (A->M % 2 || A->N % 2)
    return fail(SS_E_ODD, "ss_fold_size: M=%lld and N=%lld must be even", (long long)A->M, (long long)A->N);
  size_t need = 0;
  ss_fold_workspace_bytes(A->M, A->N, &need);
  if (workspace_bytes < need) return fail(SS_E_WORKSPACE, "ss_fold_size: workspace needs %zu bytes", need);
  hipStream_t st = static_cast<hipStream_t>(stream);
  FoldCheck* chk = static_cast<FoldCheck*>(workspace);
  CheckPart* rparts = reinterpret_cast<CheckPart*>(static_cast<char*>(workspace) + 512);
  JobArg J{};
  J.count = 1;
  J.one.A = *A;
  J.one.p = p;
  const FoldGrid g = layout_jobs(A, nullptr, nullptr, 1, nullptr);
  run_check<false>(J, g, rparts, rparts + g.rblk, chk, 1, st);
  SS_HIP_TRY(hipGetLastError());
  FoldCheck h{};
  SS_HIP_TRY(hipMemcpyAsync(&h, chk, sizeof h, hipMemcpyDeviceToHost, st));
  SS_HIP_TRY(hipStreamSynchronize(st));
  return check_verdict(h, "ss_fold_size", 0, nnz_half);
}

extern "C" ss_status ss_fold(const ss_matrix_dev* A, const float* p, ss_system* out, void* workspace,
                             size_t workspace_bytes, void* stream) {
  clear_error();
  if (ss_status s = check_fold_out(A, p, out, "ss_fold")) return s;
  size_t need = 0;
  ss_fold_workspace_bytes(A->M, A->N, &need);
  if (!workspace || workspace_bytes < need) return fail(SS_E_WORKSPACE, "ss_fold: workspace needs %zu bytes", need);
  int64_t* tiles = reinterpret_cast<int64_t*>(static_cast<char*>(workspace) + 512);
  JobArg J{};
  J.count = 1;
  J.one.A = *A;
  J.one.p = p;
  J.one.out = *out;
  const FoldGrid g = layout_jobs(A, nullptr, nullptr, 1, nullptr);
  run_fold<false>(J, g, out->wdtype, tiles, static_cast<hipStream_t>(stream));
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_fold_noalloc(const ss_matrix_dev* A, const float* p, ss_system* out, void* stream) {
  clear_error();
  if (ss_status s = check_fold_out(A, p, out, "ss_fold_noalloc")) return s;
  // every scan launch writes all the tile sums it reads: nothing to clear
  if (tiles_for(std::max(A->M, A->N) / 2 + 1) + 1 > kNoallocTiles)
    return fail(SS_E_ARG, "ss_fold_noalloc: M/2 and N/2 must be at most %lld (the scratch holds %lld tile sums)",
                (long long)((kNoallocTiles - 1) * kScanTile - 1), (long long)kNoallocTiles);
  int64_t* tiles = nullptr;
  if (ss_status s = noalloc_scratch(&tiles)) return s;
  JobArg J{};
  J.count = 1;
  J.one.A = *A;
  J.one.p = p;
  J.one.out = *out;
  const FoldGrid g = layout_jobs(A, nullptr, nullptr, 1, nullptr);
  run_fold<false>(J, g, out->wdtype, tiles, static_cast<hipStream_t>(stream));
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_fold_batch_workspace_bytes(const ss_matrix_dev* A, int32_t count, size_t* bytes) {
  clear_error();
  if (!A || count <= 0 || !bytes) return fail(SS_E_ARG, "ss_fold_batch_workspace_bytes: bad argument");
  for (int32_t k = 0; k < count; ++k)
    if (A[k].M <= 0 || A[k].N <= 0) return fail(SS_E_ARG, "ss_fold_batch_workspace_bytes: bad matrix %d", k);
  const FoldGrid g = layout_jobs(A, nullptr, nullptr, count, nullptr);
  const size_t scratch = std::max(sizeof(int64_t) * static_cast<size_t>(std::max(g.rtile, g.ctile)),
                                  sizeof(CheckPart) * static_cast<size_t>(g.rblk + g.cblk));
  *bytes = batch_head_bytes(count, g) + ((scratch + 255) & ~size_t{255}) + sizeof(FoldCheck) * static_cast<size_t>(count);
  return SS_OK;
}

extern "C" ss_status ss_fold_size_batch(const ss_matrix_dev* A, const float* const* p, int32_t count,
                                        void* workspace, size_t workspace_bytes, int64_t* nnz_half,
                                        void* stream) {
  clear_error();
  if (!A || count <= 0 || !nnz_half || !workspace) return fail(SS_E_ARG, "ss_fold_size_batch: bad argument");
  for (int32_t k = 0; k < count; ++k) {
    if (ss_status s = check_dev_matrix(&A[k], "ss_fold_size_batch")) return s;
    if (A[k].M % 2 || A[k].N % 2)
      return fail(SS_E_ODD, "ss_fold_size_batch: matrix %d: M=%lld and N=%lld must be even", k, (long long)A[k].M,
                  (long long)A[k].N);
  }
  size_t need = 0;
  if (ss_status s = ss_fold_batch_workspace_bytes(A, count, &need)) return s;
  if (workspace_bytes < need) return fail(SS_E_WORKSPACE, "ss_fold_size_batch: workspace needs %zu bytes", need);
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<FoldJob> jobs;
  const FoldGrid g = layout_jobs(A, p, nullptr, count, &jobs);
  char* ws = static_cast<char*>(workspace);
  CheckPart* rparts = reinterpret_cast<CheckPart*>(ws + batch_head_bytes(count, g));
  const size_t scratch = std::max(sizeof(int64_t) * static_cast<size_t>(std::max(g.rtile, g.ctile)),
                                  sizeof(CheckPart) * static_cast<size_t>(g.rblk + g.cblk));
  FoldCheck* chk = reinterpret_cast<FoldCheck*>(ws + batch_head_bytes(count, g) + ((scratch + 255) & ~size_t{255}));
  const JobArg J = put_batch(jobs, g, ws, st);
  run_check<true>(J, g, rparts, rparts + g.rblk, chk, count, st);
  SS_HIP_TRY(hipGetLastError());
  std::vector<FoldCheck> h(static_cast<size_t>(count));
  SS_HIP_TRY(hipMemcpyAsync(h.data(), chk, sizeof(FoldCheck) * h.size(), hipMemcpyDeviceToHost, st));
  SS_HIP_TRY(hipStreamSynchronize(st));
  std::vector<int64_t> sizes(static_cast<size_t>(count));
  for (int32_t k = 0; k < count; ++k)
    if (ss_status s = check_verdict(h[k], "ss_fold_size_batch", k, &sizes[k])) return s;
  for (int32_t k = 0; k < count; ++k) nnz_half[k] = sizes[k];
  return SS_OK;
}

extern "C" ss_status ss_fold_batch(const ss_matrix_dev* A, const float* const* p, ss_system* out, int32_t count,
                                   void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (!A || !p || !out || count <= 0) return fail(SS_E_ARG, "ss_fold_batch: bad argument");
  for (int32_t k = 0; k < count; ++k) {
    if (ss_status s = check_fold_out(&A[k], p[k], &out[k], "ss_fold_batch")) return s;
    if (out[k].wdtype != out[0].wdtype) return fail(SS_E_ARG, "ss_fold_batch: all outputs must share wdtype");
  }
  size_t need = 0;
  if (ss_status s = ss_fold_batch_workspace_bytes(A, count, &need)) return s;
  if (!workspace || workspace_bytes < need)
    return fail(SS_E_WORKSPACE, "ss_fold_batch: workspace needs %zu bytes", need);
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<FoldJob> jobs;
  const FoldGrid g = layout_jobs(A, p, out, count, &jobs);
  char* ws = static_cast<char*>(workspace);
  int64_t* tiles = reinterpret_cast<int64_t*>(ws + batch_head_bytes(count, g));
  const JobArg J = put_batch(jobs, g, ws, st);
  run_fold<true>(J, g, out[0].wdtype, tiles, st);
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_unsplit(const ss_matrix_dev* A, const float* p, ss_system* out, void* stream) {
  clear_error();
  if (ss_status s = check_dev_matrix(A, "ss_unsplit")) return s;
  if (!p || !out) return fail(SS_E_ARG, "ss_unsplit: NULL argument");
  if (out->m != A->M || out->n != A->N || out->nnz != A->nnz || out->nvals != 1)
    return fail(SS_E_ARG, "ss_unsplit: out must be m = M, n = N, nnz = nnz(A), nvals = 1");
  if (out->wdtype != SS_F32 && out->wdtype != SS_BF16 && out->wdtype != SS_F16)
    return fail(SS_E_ARG, "ss_unsplit: unknown wdtype %d", out->wdtype);
  if (!out->row_ptr || !out->col_ptr || !out->p || !out->inv_row || !out->inv_col ||
      (out->nnz > 0 && (!out->col_idx || !out->val || !out->row_idx || !out->val_t)))
    return fail(SS_E_ARG, "ss_unsplit: NULL output array");
  if (out->wdtype == SS_F32 && (out->val != A->val || out->val_t != A->val_t))
    return fail(SS_E_ARG, "ss_unsplit: FP32 values must alias A's arrays");
  if (ss_status s = check_ascending(out, "ss_unsplit")) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  k_line_recip<false><<<blocks_for(A->M), kWave * kFoldWaves, 0, st>>>(A->row_ptr, A->val, A->M, out->inv_row);
  k_line_recip<true><<<blocks_for(A->N), kWave * kFoldWaves, 0, st>>>(A->col_ptr, A->val_t, A->N, out->inv_col);
  const unsigned nbv = static_cast<unsigned>((A->nnz + 255) / 256);
  if (out->wdtype != SS_F32 && A->nnz > 0) {
    if (out->wdtype == SS_BF16) {
      k_convert<SS_BF16><<<nbv, 256, 0, st>>>(A->val, A->nnz, out->val);
      k_convert<SS_BF16><<<nbv, 256, 0, st>>>(A->val_t, A->nnz, out->val_t);
    } else {
      k_convert<SS_F16><<<nbv, 256, 0, st>>>(A->val, A->nnz, out->val);
      k_convert<SS_F16><<<nbv, 256, 0, st>>>(A->val_t, A->nnz, out->val_t);
    }
  }
  if (out->p != p)
    k_copy_f32<<<static_cast<unsigned>((A->M + 255) / 256), 256, 0, st>>>(p, A->M, out->p);
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}
