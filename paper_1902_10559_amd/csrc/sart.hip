// Simultaneous SART on one or many systems at once (the paper's solver,
// Section 1 and its refs. [001], [003]):
//     f <- f + lambda * V^-1 A^T W^-1 (p - A f)
// run on both halves of the folded pair (systems (3) and (4), interleaved
// values sharing one index array) or on a single system.
//
// One iteration is two kernels:
//   k_sart_fp  forward projection, residual and scaled residual: per row i,
//              q = A[i,:] f, r = p[i] - q, z[i] = r * inv_row[i]; one FP64
//              partial of |r|^2 per block.
//   k_sart_bp  back projection and update from the pre-transposed (CSC)
//              copy: per column j, b = A[:,j]^T z, f'[j] = f[j] + lambda *
//              inv_col[j] * b.  Every column is owned by one lane group, so
//              the update needs no atomics.  The first block of each system
//              also sums the forward partials in index order (the kernel
//              boundary has made them visible), records rel_res(f^k) and
//              decides whether the system stops.
// The iterate alternates between two buffers (the caller's image and one in
// the workspace): f^k lives in buffer k mod 2.  A stop decided during the
// back projection of iteration k therefore leaves f^k intact even if other
// blocks of that launch already wrote f^{k+1} into the other buffer; a final
// kernel copies f^k into the caller's image when k is odd.  No block ever
// waits for another, and no cross-XCD fence is needed inside a kernel.
// Rows (columns) are processed by groups of 64/RPW (64/CPW) lanes of a
// wavefront; lanes stride over the row's entries (coalesced loads of indices
// and values), partial sums are combined by a fixed butterfly, so results are
// bitwise reproducible run to run.  A block never straddles two systems; the
// blocks of all systems form one grid per kernel.
//
// Per-system state lives in the caller's workspace: k (index of the current
// iterate), stop and pending flags, ||p||^2.  k changes only in the first
// forward block (so it is constant during a back projection), stop only in
// the first back-projection block.  Kernels of a stopped system exit at once,
// so a replayed graph may overshoot the iteration count harmlessly.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include <hip/hip_ext.h>

#include "device.h"
#include "graph_cache.h"
#include "internal.h"
#include "interleave.h"
#include "lines.h"
#include "staged.h"

namespace ss {
namespace {

// ---- device code begin
constexpr int kWPB = 4;          // wavefronts per block
constexpr int kThreads = kWave * kWPB;

struct SysState {
  double pnorm2;     // ||p||^2 over all halves
  double last_res;   // rel_res of the latest evaluated iterate
  int32_t k;         // index of the current iterate f^k
  int32_t stop;      // 1: f^k is final (written once, 0 -> 1)
  int32_t pending;   // 1: the next forward pass moves on to f^{k+1}
  int32_t pad;
};

struct SysDesc {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const void* val;
  const int64_t* col_ptr;
  const int32_t* row_idx;
  const void* val_t;
  const float* p;
  const float* inv_row;
  const float* inv_col;
  float* f[2];       // [0] the caller's image, [1] the workspace buffer
  float* z;
  double* res_hist;
  double* partials;
  SysState* st;
  int64_t m, n;
  int64_t fp_block0, bp_block0;  // first block of this system in each grid
  int32_t fp_nblocks, bp_nblocks;
  // band-staged forward projection (see staged.h)
  uint16_t* fb_idx;   // band-major copy of the row streams: column - band start
  void* fb_val;
  int32_t* fb_off;    // band-major segment -> first entry ([nseg] = padded total)
  uint32_t* fb_bits;  // one bit per chunk: set where a segment starts
  int32_t* fb_slot;   // row partial slot -> its band-major segment
  uint32_t* fb_rseg;  // m+1: row i's partial slots [rseg[i], rseg[i+1])
  float* fb_part;     // NV floats per band-major segment
  uint64_t* fb_len;   // nb*m+1: (segments, padded entries) per (band, row), scanned
  int64_t cv_rblk0;   // first block of this system in the set-up row grid
  int64_t cv_t64_0, cv_t32_0;  // first scan tile of fb_len / fb_rseg
  int32_t fb_nb;      // bands
  int32_t fb_pair0;   // first (system, band) pair of this system
  // tile-staged back projection
  uint16_t* bt_idx;   // rank of each CSC entry's row among its tile's rows
  BtMeta* bt_meta;    // per tile
  int32_t* bt_runs;   // per tile kBtRunCap pairs (first row, first LDS slot)
};

struct Params {
  float lambda;
  int32_t max_iter;
  double tol;
  int32_t nonneg;
  int32_t band_lg;   // log2 of the forward bands' width (staged)
  int32_t tile_lg;   // log2 of the back-projection tiles' columns (staged)
  int32_t band_q;    // chunks per forward work tile (staged)
  // block -> system of the staged grids (one load instead of a search of
  // dependent loads at every block's start): 0 the residual's rows, 1 the
  // back-projection tiles, 2 the set-up's rows; unused for one system
  const int32_t* b2s[3];
};

struct SetupFlags {
  int32_t zero_start;
};

constexpr int kDescChunk = 16;
struct DescChunk {
  SysDesc d[kDescChunk];
  int32_t count;
  int32_t first;
};

// Grid of a launch over all systems: 0 forward, 1 back projection, 2 the
// set-up grid over rows.
template <int GRID>
__device__ inline int64_t block0_of(const SysDesc& d) {
  if constexpr (GRID == 0) return d.fp_block0;
  else if constexpr (GRID == 1) return d.bp_block0;
  else return d.cv_rblk0;
}

template <int GRID>
__device__ inline int find_sys(const SysDesc* t, int nsys, int64_t b) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = __builtin_amdgcn_readfirstlane((lo + hi + 1) >> 1);
    if (block0_of<GRID>(t[mid]) <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The system of block b of a staged grid, from the set-up's table.
template <int GRID>
__device__ inline int sys_of(const Params* prm, int nsys, int64_t b) {
  return nsys == 1 ? 0 : __builtin_amdgcn_readfirstlane(gl(prm->b2s[GRID])[b]);
}

// Fills the block -> system tables of the staged grids (one block per
// system; a NULL table is skipped).
__global__ void k_fill_b2s(const SysDesc* table, int32_t* fp, int32_t* bp, int32_t* cv, int cv_rows) {
  const SysDesc& d = table[blockIdx.x];
  const int32_t s = static_cast<int32_t>(blockIdx.x);
  if (fp)
    for (int64_t i = threadIdx.x; i < d.fp_nblocks; i += blockDim.x) fp[d.fp_block0 + i] = s;
  if (bp)
    for (int64_t i = threadIdx.x; i < d.bp_nblocks; i += blockDim.x) bp[d.bp_block0 + i] = s;
  if (cv)
    for (int64_t i = threadIdx.x; i < (d.m + cv_rows - 1) / cv_rows; i += blockDim.x) cv[d.cv_rblk0 + i] = s;
}

// Writes up to kDescChunk descriptors (from the kernel arguments) into the
// table, and the parameters with the first chunk.
__global__ void k_put_desc(DescChunk ch, SysDesc* table, Params prm_in, Params* prm) {
  const int t = static_cast<int>(threadIdx.x);
  if (t < ch.count) table[ch.first + t] = ch.d[t];
  if (ch.first == 0 && t == 0) *prm = prm_in;
}

// Resets each system's state, clears its image (zero_start) and reduces
// ||p||^2 in a fixed order: one block of kSetupWaves wavefronts per system
// (a single system is one block: the wider, the sooner it is done), all
// systems in one launch.
constexpr int kSetupWaves = 16;
template <int NV>
__global__ __launch_bounds__(kWave* kSetupWaves) void k_setup(const SysDesc* table, SetupFlags fl) {
  constexpr int T = kWave * kSetupWaves;
  const SysDesc& d = table[blockIdx.x];
  if (fl.zero_start)
    for (int64_t i = threadIdx.x; i < d.n * NV; i += T) d.f[0][i] = 0.0f;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < d.m * NV; i += T) {
    const double v = d.p[i];
    s += v * v;
  }
  __shared__ double red[kSetupWaves];
  s = block_sum<kSetupWaves>(s, red);
  if (threadIdx.x == 0) {
    d.st->pnorm2 = s;
    d.st->last_res = 0.0;
    d.st->k = 0;
    d.st->stop = 0;
    d.st->pending = 0;
  }
}

__device__ inline int load_flag(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void store_flag(int32_t* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// What a tile needs before its main loads: the system, the tile's index in
// it, this lane group's line and the line's offsets.  Loaded one tile ahead.
struct TileCtx {
  int s;
  int stop;
  int64_t local;
  int64_t line;
  int64_t lo, hi;
};

template <bool BP, int PW>
__device__ inline TileCtx tile_ctx(const SysDesc* table, int nsys, uint32_t t, uint32_t ntiles, int xcd) {
  TileCtx c;
  const uint32_t b = __builtin_amdgcn_readfirstlane(xcd ? xcd_remap(t, ntiles) : t);
  // uniform per block: keep the descriptor in scalar registers
  c.s = __builtin_amdgcn_readfirstlane(nsys == 1 ? 0 : find_sys<BP ? 1 : 0>(table, nsys, b));
  const SysDesc& S = table[c.s];
  c.stop = *gl(&S.st->stop);
  c.local = static_cast<int64_t>(b) - (BP ? S.bp_block0 : S.fp_block0);
  c.line = c.local * (PW * kWPB) + wave_id() * PW + lane_id() / (kWave / PW);
  // lines past the end read ptr[lines] twice: an empty line, with no branch
  const int64_t lines = BP ? S.n : S.m;
  const int64_t* ptr = BP ? S.col_ptr : S.row_ptr;
  c.lo = gl(ptr)[c.line < lines ? c.line : lines];
  c.hi = gl(ptr)[c.line + 1 < lines ? c.line + 1 : lines];
  return c;
}

// Forward projection and residual.  A grid-stride loop over tiles of
// RPW*kWPB rows.  Per tile: p and 1/W are requested first, then the row
// sums, then the next tile's context (so its loads overlap this tile's
// reduction), then the residual, z and the block's FP64 partial.
// Stream forms: 0 entry-wise, 1 aligned chunks, 2 interleaved (the line's
// entries read from the workspace copy that k_interleave writes).
template <int NV, int WT, int L, int U, int SF>
__device__ inline void line_sum(const int32_t* idx, const void* val, const float* x, int64_t lo, int64_t hi,
                                int glane, float* acc) {
  if constexpr (SF == 2) line_dot_i<NV, WT, L, U / SS_CHUNK>(idx, val, x, lo, hi, glane, acc);
  else line_dot<NV, WT, L, U, SF == 1>(idx, val, x, lo, hi, glane, acc);
}

template <int NV, int WT, int RPW, int U, int SF>
__global__ __launch_bounds__(kThreads) void k_sart_fp(const SysDesc* __restrict__ table, int nsys,
                                                      uint32_t ntiles, int xcd, int parity) {
  constexpr int L = kWave / RPW;
  __shared__ double red[kWPB];
  uint32_t t = blockIdx.x;
  if (t >= ntiles) return;
  const int glane = lane_id() % L;
  TileCtx cur = tile_ctx<false, RPW>(table, nsys, t, ntiles, xcd);
  for (;;) {
    const uint32_t tn = t + gridDim.x;
    const bool more = tn < ntiles;
    TileCtx nxt{};
    if (!cur.stop) {
      const SysDesc& S = table[cur.s];
      // every lane requests its line's p and 1/W (one request per group),
      // so no branch separates these loads from the row's stream loads
      const bool owner = glane == 0 && cur.line < S.m;
      const int64_t li = cur.line < S.m ? cur.line : S.m - 1;
      const Vec<NV> pv = load_vec<NV>(S.p, li);
      const float w = gl(S.inv_row)[li];
      float acc[NV];
#pragma unroll
      for (int h = 0; h < NV; ++h) acc[h] = 0.0f;
      line_sum<NV, WT, L, U, SF>(S.col_idx, S.val, S.f[parity], cur.lo, cur.hi, glane, acc);
      if (more) nxt = tile_ctx<false, RPW>(table, nsys, tn, ntiles, xcd);
#pragma unroll
      for (int h = 0; h < NV; ++h) acc[h] = group_sum<L>(acc[h]);
      double d = 0.0;
      if (owner) {
        Vec<NV> zv;
#pragma unroll
        for (int h = 0; h < NV; ++h) {
          const float r = pv.v[h] - acc[h];
          zv.v[h] = r * w;
          d += static_cast<double>(r) * static_cast<double>(r);
        }
        store_vec<NV>(S.z, cur.line, zv);
      }
      const double tot = block_sum<kWPB>(d, red);
      if (threadIdx.x == 0) {
        glw(S.partials)[cur.local] = tot;
        // the first tile of the system moves the iterate index on
        SysState* st = S.st;
        if (cur.local == 0 && *gl(&st->pending)) {
          glw(&st->k)[0] += 1;
          glw(&st->pending)[0] = 0;
        }
      }
      __syncthreads();  // red is reused by the next tile
    } else if (more) {
      nxt = tile_ctx<false, RPW>(table, nsys, tn, ntiles, xcd);
    }
    if (!more) break;
    cur = nxt;
    t = tn;
  }
}

// The first back-projection block of a system: rel_res(f^k) from the forward
// partials in index order, the history entry, and the stop decision.
template <int WPB>
__device__ void finalize_residual(const Params* prm, const SysDesc& S, double* red) {
  SysState* st = S.st;
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < S.fp_nblocks; t += WPB * kWave) acc += gl(S.partials)[t];
  const double rsum = block_sum<WPB>(acc, red);
  if (threadIdx.x == 0) {
    const double pn = *gl(&st->pnorm2);
    const double rel = pn > 0.0 ? sqrt(rsum / pn) : sqrt(rsum);
    const int k = *gl(&st->k);
    if (S.res_hist) glw(S.res_hist)[k] = rel;
    glw(&st->last_res)[0] = rel;
    if (rel <= prm->tol || k >= prm->max_iter) store_flag(&st->stop, 1);
    else glw(&st->pending)[0] = 1;
  }
}

// Back projection and update, with the residual finalisation in the first
// tile of each system.  Grid-stride over tiles of CPW*kWPB columns, with the
// same ordering as the forward kernel.
template <int NV, int WT, int CPW, int U, int SF>
__global__ __launch_bounds__(kThreads) void k_sart_bp(const Params* __restrict__ prm,
                                                      const SysDesc* __restrict__ table, int nsys,
                                                      uint32_t ntiles, int xcd, int parity) {
  constexpr int L = kWave / CPW;
  __shared__ double red[kWPB];
  uint32_t t = blockIdx.x;
  if (t >= ntiles) return;
  const int glane = lane_id() % L;
  TileCtx cur = tile_ctx<true, CPW>(table, nsys, t, ntiles, xcd);
  for (;;) {
    const uint32_t tn = t + gridDim.x;
    const bool more = tn < ntiles;
    TileCtx nxt{};
    bool prefetched = false;
    if (!cur.stop) {
      const SysDesc& S = table[cur.s];
      if (cur.local == 0) {
        finalize_residual<kWPB>(prm, S, red);
        __syncthreads();
      }
      // f^k with k = max_iter is final: its residual is all that was wanted
      if (*gl(&S.st->k) < prm->max_iter) {
        const bool owner = glane == 0 && cur.line < S.n;
        const int64_t li = cur.line < S.n ? cur.line : S.n - 1;
        Vec<NV> fv = load_vec<NV>(S.f[parity], li);
        const float tl = prm->lambda * gl(S.inv_col)[li];
        float acc[NV];
#pragma unroll
        for (int h = 0; h < NV; ++h) acc[h] = 0.0f;
        line_sum<NV, WT, L, U, SF>(S.row_idx, S.val_t, S.z, cur.lo, cur.hi, glane, acc);
        if (more) nxt = tile_ctx<true, CPW>(table, nsys, tn, ntiles, xcd);
        prefetched = true;
#pragma unroll
        for (int h = 0; h < NV; ++h) acc[h] = group_sum<L>(acc[h]);
        if (owner) {
#pragma unroll
          for (int h = 0; h < NV; ++h) fv.v[h] = fmaf(tl, acc[h], fv.v[h]);
          if (prm->nonneg) fv = project_nonneg<NV>(fv);
          store_vec<NV>(S.f[parity ^ 1], cur.line, fv);
        }
      }
    }
    if (!more) break;
    if (!prefetched) nxt = tile_ctx<true, CPW>(table, nsys, tn, ntiles, xcd);
    cur = nxt;
    t = tn;
  }
}

// Copies f^k into the caller's image when it sits in the workspace buffer.
template <int NV>
__global__ __launch_bounds__(kThreads) void k_finish(const SysDesc* table) {
  const SysDesc& S = table[blockIdx.x];
  if ((S.st->k & 1) == 0) return;
  const int64_t cnt = S.n * NV;
  for (int64_t i = threadIdx.x; i < cnt; i += kThreads) S.f[0][i] = S.f[1][i];
}

// ------------------------------------------- staged kernels (staged.h)
// Set-up grid over rows: kCvRows rows per block, kCvLanes lanes per row.
constexpr int kCvLanes = 16;
constexpr int kCvRows = kThreads / kCvLanes;

// A row's lanes load kRowWin windows of kCvLanes entries at once (a batch),
// so that a row costs fewer dependent load latencies than one or two per
// window; rows longer than a batch take several.  These kernels are bound by
// those latencies times the rows in flight: on the 256-slice batch, batches
// of 2, 4 and 8 windows filled in 4.31, 4.55 and 5.59 ms (the registers of
// larger batches cost residency).
constexpr int kRowWin = 2;
constexpr int kRowBatch = kRowWin * kCvLanes;

// The columns of one batch from `base`, and the column of the entry after
// it; positions past the row's end re-read its last entry (the row is not
// empty), so every load is inside the row.
struct RowBatch {
  int32_t c[kRowWin];
  int32_t after;
};

__device__ inline void row_batch_load(const int32_t* col, int64_t base, int64_t hi, int g, RowBatch& B) {
#pragma unroll
  for (int w = 0; w < kRowWin; ++w) {
    const int64_t k = base + w * kCvLanes + g;
    B.c[w] = gl(col)[k < hi ? k : hi - 1];
  }
  const int64_t ka = base + kRowBatch;
  B.after = gl(col)[ka < hi ? ka : hi - 1];
}

// The band runs of one window of a row (entries k = base + g, g < kCvLanes):
// per entry its band (-1 past the row's end), whether it starts a run and
// whether it ends one (the next entry is in another band, or there is
// none), and the first entry of its run.  `after` is the band of the entry
// after the window (-1 if none); `run0` and `band0` carry the previous
// window's last run start and band.  The lanes of a row call it together
// (the shuffles stay inside the row's lanes).
struct RunLane {
  int32_t band;
  bool valid, start, end;
  int64_t k, ks;
};

__device__ inline RunLane run_of(int32_t band, int32_t after, int64_t k, bool valid, int g, int64_t run0,
                                 int32_t band0) {
  RunLane r;
  r.k = k;
  r.valid = valid;
  r.band = band;
  int32_t bp = __shfl_up(band, 1, kCvLanes);
  if (g == 0) bp = band0;
  int32_t bn = __shfl_down(band, 1, kCvLanes);
  if (g == kCvLanes - 1) bn = after;
  r.start = valid && band != bp;
  r.end = valid && band != bn;
  int64_t ks = r.start ? k : int64_t{-1};
#pragma unroll
  for (int d = 1; d < kCvLanes; d <<= 1) {
    const int64_t t = __shfl_up(ks, d, kCvLanes);
    if (g >= d) ks = max(ks, t);
  }
  r.ks = ks >= 0 ? ks : run0;
  return r;
}

// The runs of window w of a loaded batch.
__device__ inline RunLane batch_run(const RowBatch& B, int w, int64_t base, int64_t hi, int lg, int g, int64_t run0,
                                    int32_t band0) {
  const int64_t k = base + w * kCvLanes + g;
  const bool valid = k < hi;
  const int32_t band = valid ? (B.c[w] >> lg) : -1;
  int32_t after;
  if (w + 1 < kRowWin) {  // lane 0 of the next window
    const int64_t kn = base + (w + 1) * kCvLanes;
    const int32_t cn = __shfl(B.c[w + 1], 0, kCvLanes);
    after = kn < hi ? (cn >> lg) : -1;
  } else {
    after = base + kRowBatch < hi ? (B.after >> lg) : -1;
  }
  return run_of(band, after, k, valid, g, run0, band0);
}

// Whether the entries of a loaded batch strictly ascend inside [0, n), each
// against the one before it (`prev`: the column before the batch, for a
// batch that does not start the row); every lane of the row gets the
// answer.  Returns the batch's last column in *last.
__device__ inline bool batch_ascends(const RowBatch& B, int64_t base, int64_t lo, int64_t hi, int64_t n,
                                     int32_t prev, int g, int32_t* last) {
  bool bad = false;
#pragma unroll
  for (int w = 0; w < kRowWin; ++w) {
    const int64_t k = base + w * kCvLanes + g;
    const int32_t c = B.c[w];
    int32_t p = __shfl_up(c, 1, kCvLanes);
    if (g == 0) p = w == 0 ? prev : __shfl(B.c[w - 1], kCvLanes - 1, kCvLanes);
    bad |= k < hi && (c < 0 || c >= n || (k > lo && p >= c));
  }
  *last = __shfl(B.c[kRowWin - 1], kCvLanes - 1, kCvLanes);
  int b = bad ? 1 : 0;
#pragma unroll
  for (int o = kCvLanes / 2; o > 0; o >>= 1) b |= __shfl_xor(b, o, kWave);
  return b == 0;
}

// Per row: the padded length of each band run (a segment) into
// fb_len[b*m + i] as (1 segment, entries rounded up to whole chunks), and
// the row's segment count into fb_rseg[i].  A row whose columns do not
// strictly ascend inside [0, n) gets no segments (the staged forward form
// then leaves it out).  The first batch is kept in registers between the
// check and the count.  One block per group of kCvRows rows: adjacent rows
// run together, so their band-major writes meet in the same cache lines
// (blocks that each walk a range of groups measured slower).
__global__ __launch_bounds__(kThreads) void k_fb_count(const SysDesc* table, int nsys, const Params* prm) {
  const int64_t vb = blockIdx.x;
  const SysDesc& S = table[sys_of<2>(prm, nsys, vb)];
  const int lg = prm->band_lg;
  const int64_t i = (vb - S.cv_rblk0) * kCvRows + threadIdx.x / kCvLanes;
  const int g = threadIdx.x % kCvLanes;
  if (i >= S.m) return;  // the row's lanes leave together
  const int64_t lo = gl(S.row_ptr)[i], hi = gl(S.row_ptr)[i + 1];
  if (hi <= lo) {
    if (g == 0) glw(S.fb_rseg)[i] = 0u;
    return;
  }
  RowBatch B0;
  row_batch_load(S.col_idx, lo, hi, g, B0);
  int32_t last;
  bool ok = batch_ascends(B0, lo, lo, hi, S.n, 0, g, &last);
  for (int64_t base = lo + kRowBatch; ok && base < hi; base += kRowBatch) {
    RowBatch B;
    row_batch_load(S.col_idx, base, hi, g, B);
    ok = batch_ascends(B, base, lo, hi, S.n, last, g, &last);
  }
  if (!ok) {
    if (g == 0) glw(S.fb_rseg)[i] = 0u;
    return;
  }
  int64_t run0 = lo;
  int32_t band0 = -1;
  uint32_t runs = 0;
  for (int64_t base = lo; base < hi; base += kRowBatch) {
    RowBatch B;
    if (base == lo) B = B0;
    else row_batch_load(S.col_idx, base, hi, g, B);
#pragma unroll
    for (int w = 0; w < kRowWin; ++w) {
      const RunLane r = batch_run(B, w, base, hi, lg, g, run0, band0);
      if (r.end)
        glw(S.fb_len)[static_cast<int64_t>(r.band) * S.m + i] =
            seg_pack(1u, static_cast<uint32_t>(pad_chunk(r.k + 1 - r.ks)));
      runs += r.start ? 1u : 0u;
      run0 = __shfl(r.ks, kCvLanes - 1, kCvLanes);
      band0 = __shfl(r.band, kCvLanes - 1, kCvLanes);
    }
  }
#pragma unroll
  for (int o = kCvLanes / 2; o > 0; o >>= 1) runs += __shfl_xor(runs, o, kWave);
  if (g == 0) glw(S.fb_rseg)[i] = runs;
}

// Per row, after both scans: each entry goes to its band-major position
// (16-bit column within the band, value copied bit for bit) and each
// segment's padding entries get value 0 and index 0; each run start records
// its segment's offset and its chunk's bit in fb_bits, and the row's slot
// for the run (the row's slots follow its bands in ascending order) records
// the segment.  A batch at a time: its columns and values, then every
// window's runs, then their (band, row) prefixes, then the stores.  VB:
// value bytes per entry.
template <int VB>
__global__ __launch_bounds__(kThreads) void k_fb_fill(const SysDesc* table, int nsys, const Params* prm) {
  const int64_t vb = blockIdx.x;
  const SysDesc& S = table[sys_of<2>(prm, nsys, vb)];
  using V = std::conditional_t<VB == 8, uint64_t, std::conditional_t<VB == 4, uint32_t, uint16_t>>;
  const int lg = prm->band_lg;
  const int64_t i = (vb - S.cv_rblk0) * kCvRows + threadIdx.x / kCvLanes;
  const int g = threadIdx.x % kCvLanes;
  if (i == 0 && g == 0) {
    const uint64_t tot = gl(S.fb_len)[static_cast<int64_t>(S.fb_nb) * S.m];
    glw(S.fb_off)[seg_count(tot)] = static_cast<int32_t>(seg_entries(tot));
  }
  if (i >= S.m) return;
  const uint32_t slot0 = gl(S.fb_rseg)[i];
  if (gl(S.fb_rseg)[i + 1] == slot0) return;  // an empty row, or one given no segments
  const int64_t lo = gl(S.row_ptr)[i], hi = gl(S.row_ptr)[i + 1];
  const V* val = static_cast<const V*>(S.val);
  V* fval = static_cast<V*>(S.fb_val);
  int64_t run0 = lo;
  int32_t band0 = -1;
  uint32_t ord = 0;  // the row's runs in earlier windows
  for (int64_t base = lo; base < hi; base += kRowBatch) {
    RowBatch B;
    row_batch_load(S.col_idx, base, hi, g, B);
    V v[kRowWin];
#pragma unroll
    for (int w = 0; w < kRowWin; ++w) {
      const int64_t k = base + w * kCvLanes + g;
      v[w] = gl(val)[k < hi ? k : hi - 1];
    }
    // every window's runs (per lane: its band, its run's first entry as an
    // offset from the batch, and its flags with its run's slot), then the
    // (band, row) prefixes of all windows, then the stores
    int32_t band[kRowWin], ksr[kRowWin];
    uint32_t fs[kRowWin];  // bit 0 valid, 1 start, 2 end; bits 8.. the run's slot in the row
#pragma unroll
    for (int w = 0; w < kRowWin; ++w) {
      const RunLane r = batch_run(B, w, base, hi, lg, g, run0, band0);
      uint32_t n = r.start ? 1u : 0u;  // runs started at or before this lane in the window
#pragma unroll
      for (int d = 1; d < kCvLanes; d <<= 1) {
        const uint32_t t = __shfl_up(n, d, kCvLanes);
        if (g >= d) n += t;
      }
      band[w] = r.band;
      ksr[w] = static_cast<int32_t>(r.ks - base);  // negative for a run from an earlier batch
      fs[w] = (r.valid ? 1u : 0u) | (r.start ? 2u : 0u) | (r.end ? 4u : 0u) | ((ord + n - 1u) << 8);
      ord += __shfl(n, kCvLanes - 1, kCvLanes);
      run0 = __shfl(r.ks, kCvLanes - 1, kCvLanes);
      band0 = __shfl(r.band, kCvLanes - 1, kCvLanes);
    }
    uint64_t pre[kRowWin];
    uint32_t e1[kRowWin];
#pragma unroll
    for (int w = 0; w < kRowWin; ++w) {
      const int64_t at = static_cast<int64_t>((fs[w] & 1u) ? band[w] : 0) * S.m + i;
      pre[w] = gl(S.fb_len)[at];
      e1[w] = seg_entries(gl(S.fb_len)[at + 1]);  // the prefix plus the padded length
    }
#pragma unroll
    for (int w = 0; w < kRowWin; ++w) {
      if (!(fs[w] & 1u)) continue;
      const int64_t e0 = seg_entries(pre[w]);
      const int64_t pos = e0 + (w * kCvLanes + g - ksr[w]);
      if (pos < e1[w]) {
        glw(S.fb_idx)[pos] = static_cast<uint16_t>(B.c[w] - (band[w] << lg));
        glw(fval)[pos] = v[w];
      }
      if (fs[w] & 4u) {
        for (int64_t q = pos + 1; q < e1[w]; ++q) {
          glw(S.fb_idx)[q] = 0;
          glw(fval)[q] = V{0};
        }
      }
      if (fs[w] & 2u) {
        const uint32_t sg = seg_count(pre[w]);
        glw(S.fb_off)[sg] = static_cast<int32_t>(e0);
        glw(S.fb_slot)[slot0 + (fs[w] >> 8)] = static_cast<int32_t>(sg);
        const int64_t c4 = e0 / SS_CHUNK;
        atomicOr(S.fb_bits + (c4 >> 5), 1u << (c4 & 31));
      }
    }
  }
}

// The scan pieces of the staged forward set-up: per system its (band, row)
// pairs (plus the total) and its rows (plus the total).
__global__ void k_make_pieces(const SysDesc* table, int nsys, ScanPiece<uint64_t>* p64, ScanPiece<uint32_t>* p32) {
  const int s = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (s >= nsys) return;
  const SysDesc& S = table[s];
  const int64_t l64 = static_cast<int64_t>(S.fb_nb) * S.m + 1, l32 = S.m + 1;
  p64[s] = ScanPiece<uint64_t>{S.fb_len, l64, S.cv_t64_0, (l64 + kPScanTile - 1) / kPScanTile, nullptr};
  p32[s] = ScanPiece<uint32_t>{S.fb_rseg, l32, S.cv_t32_0, (l32 + kPScanTile - 1) / kPScanTile, nullptr};
}

// The (system, band) pair q of all systems: its system and band.
__device__ inline void pair_of(const SysDesc* table, int nsys, int q, int* sys, int* band) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (table[mid].fb_pair0 <= q) lo = mid;
    else hi = mid - 1;
  }
  *sys = lo;
  *band = q - table[lo].fb_pair0;
}

// The work tiles per (system, band) pair: its chunks cut into ceil(chunks
// / q) tiles; their exclusive scan into pair_t0 (npairs + 1) and the total
// into ntiles[0].  One block; each thread takes a run of pairs.
constexpr int kTileThreads = 1024;
__global__ __launch_bounds__(kTileThreads) void k_band_pairs(const SysDesc* table, int nsys, int npairs, int q,
                                                             int32_t* pair_t0, int32_t* ntiles) {
  __shared__ int32_t tot[kTileThreads];
  const int chunk = (npairs + kTileThreads - 1) / kTileThreads;
  const int q0 = static_cast<int>(threadIdx.x) * chunk;
  const int q1 = min(npairs, q0 + chunk);
  auto tiles_of = [&](int p) {
    int sy, bd;
    pair_of(table, nsys, p, &sy, &bd);
    const SysDesc& S = table[sy];
    const int64_t e0 = seg_entries(gl(S.fb_len)[static_cast<int64_t>(bd) * S.m]);
    const int64_t e1 = seg_entries(gl(S.fb_len)[static_cast<int64_t>(bd + 1) * S.m]);
    return static_cast<int32_t>((e1 - e0) / SS_CHUNK + q - 1) / q;
  };
  int32_t mine = 0;
  for (int p = q0; p < q1; ++p) mine += tiles_of(p);
  tot[threadIdx.x] = mine;
  __syncthreads();
  for (int o = 1; o < kTileThreads; o <<= 1) {
    const int32_t v = threadIdx.x >= static_cast<unsigned>(o) ? tot[threadIdx.x - o] : 0;
    __syncthreads();
    tot[threadIdx.x] += v;
    __syncthreads();
  }
  int32_t t = tot[threadIdx.x] - mine;
  for (int p = q0; p < q1; ++p) {
    pair_t0[p] = t;
    t += tiles_of(p);
  }
  if (threadIdx.x == kTileThreads - 1) {
    pair_t0[npairs] = tot[kTileThreads - 1];
    ntiles[0] = tot[kTileThreads - 1];
  }
}

// First segment in [a, b) whose offset is >= e (offsets ascend).
__device__ inline int32_t seg_lower_bound(const int32_t* off, int32_t a, int32_t b, int64_t e) {
  while (a < b) {
    const int32_t mid = a + ((b - a) >> 1);
    if (gl(off)[mid] < e) a = mid + 1;
    else b = mid;
  }
  return a;
}

// One thread per work tile: tile j of its pair holds the segments that
// start in the pair's chunks [j q, (j + 1) q).
__global__ void k_band_tile_fill(const SysDesc* table, int nsys, int npairs, int q, const int32_t* pair_t0,
                                 const int32_t* ntiles, BandTile* tiles) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= gl(ntiles)[0]) return;
  int lo = 0, hi = npairs - 1;  // the last pair whose first tile is <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (gl(pair_t0)[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  int sy, bd;
  pair_of(table, nsys, lo, &sy, &bd);
  const SysDesc& S = table[sy];
  const uint64_t ba = gl(S.fb_len)[static_cast<int64_t>(bd) * S.m];
  const uint64_t bb = gl(S.fb_len)[static_cast<int64_t>(bd + 1) * S.m];
  const int32_t a = static_cast<int32_t>(seg_count(ba)), b = static_cast<int32_t>(seg_count(bb));
  const int64_t e0 = seg_entries(ba);
  const int64_t j = t - gl(pair_t0)[lo];
  const bool last = t + 1 == gl(pair_t0)[lo + 1];
  const int64_t qe = static_cast<int64_t>(q) * SS_CHUNK;
  const int32_t s0 = seg_lower_bound(S.fb_off, a, b, e0 + j * qe);
  const int32_t s1 = last ? b : seg_lower_bound(S.fb_off, a, b, e0 + (j + 1) * qe);
  BandTile T;
  T.sys = sy;
  T.band = bd;
  T.s0 = s0;
  T.s1 = s1;
  T.c0 = gl(S.fb_off)[s0] / SS_CHUNK;
  T.c1 = gl(S.fb_off)[s1] / SS_CHUNK;
  T.pad[0] = T.pad[1] = 0;
  int32_t* dst = reinterpret_cast<int32_t*>(tiles + t);
  const int32_t* src = reinterpret_cast<const int32_t*>(&T);
#pragma unroll
  for (int w = 0; w < 8; ++w) glw(dst)[w] = src[w];
}

// The loads of U windows of a band tile: per lane its chunk's indices,
// values and the word of start bits that holds its chunk's bit.
template <int NV, int U>
struct BandBatch {
  u32x2 ci[U];
  Vec<NV> v[U][SS_CHUNK];
  uint32_t bw[U];
};

// A wavefront's walk over one tile; the carried segment's state; the
// wavefront's LDS buffer of finished segment sums (kSegBuf segments from
// buf_base on), written to memory in contiguous runs.

template <int NV>
struct BandWalk {
  const uint16_t* tidx;
  const char* tval;
  const uint32_t* bits;
  float* buf;
  int64_t c0;
  int32_t nch;
  int32_t seg_base;  // the segment of the next window's first start
  int32_t carry_seg;
  int32_t buf_base;
  bool carry;        // a segment runs on from the previous window
  float carry_sum[NV];
};

// Writes the buffered sums of segments [buf_base, end) (the whole wavefront:
// 64 consecutive segments per store) and moves the buffer on to `end`.
template <int NV>
__device__ inline void band_flush(BandWalk<NV>& W, int32_t end, float* part, int lane) {
  __builtin_amdgcn_wave_barrier();
  float* dst = part + static_cast<int64_t>(W.buf_base) * NV;  // the run's first sum (uniform)
  const int32_t cnt = end - W.buf_base;  // at most kSegBuf
#pragma unroll
  for (int k = 0; k < kSegBuf / kWave; ++k) {
    const int32_t i = k * kWave + lane;
    if (i < cnt) store_vec<NV>(dst, i, lds_vec<NV>(W.buf, static_cast<uint32_t>(i)));
  }
  __builtin_amdgcn_wave_barrier();
  W.buf_base = end;
}

template <int NV>
__device__ inline void band_put(const BandWalk<NV>& W, int32_t seg, const float* v) {
#pragma unroll
  for (int h = 0; h < NV; ++h) W.buf[(seg - W.buf_base) * NV + h] = v[h];
}

template <int NV, int WT, int U>
__device__ inline void band_load(BandBatch<NV, U>& B, const BandWalk<NV>& W, int32_t wb, int lane) {
  constexpr uint32_t kChunkValBytes = SS_CHUNK * NV * (WT == SS_F32 ? 4 : 2);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int32_t c = wb + u * kWin + lane;
    // byte offsets in 32 bits: the loads keep the tile's bases in scalar registers
    const uint32_t cc = static_cast<uint32_t>(c < W.nch ? c : W.nch - 1);
    B.ci[u] = *gl(reinterpret_cast<const u32x2*>(reinterpret_cast<const char*>(W.tidx) + cc * 8u));
    load_val_chunk<NV, WT>(W.tval + cc * kChunkValBytes, 0, B.v[u]);
    B.bw[u] = gl(W.bits)[(static_cast<uint32_t>(W.c0 & 31) + cc) >> 5];
  }
}

// Per window: the chunk's products from the band in LDS, the start mask (a
// ballot of the chunks' start bits) and a segmented scan (the batch's
// windows independently, so their work overlaps).  Then in window order:
// the lane holding a segment's last chunk stores the segment's sum; the
// segment still open at the window's last lane is carried into the next
// window, whose lanes before its first start add to it, and is stored once a
// window starts a new segment or the tile ends.  The carried sum grows
// window by window, in order: results are reproducible.  Finished sums go to
// the wavefront's LDS buffer, which is written out once it holds at least
// kSegBuf - 64 of them (a window finishes at most 64 more) and after the
// wavefront's last tile of the band.
template <int NV, int U>
__device__ inline void band_windows(const BandBatch<NV, U>& B, BandWalk<NV>& W, int32_t wb, const float* xs,
                                    uint32_t xmask, float* part, int lane) {
  const uint64_t le_mask = ~uint64_t{0} >> (kWave - 1 - lane);
  float p[U][NV];
  uint64_t m[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int32_t c = wb + u * kWin + lane;
    const bool in = c < W.nch;
    m[u] = __ballot(in && ((B.bw[u] >> ((W.c0 + c) & 31)) & 1u) != 0);
    chunk_dot_lds<NV>(B.ci[u], B.v[u], xs, xmask, p[u]);
#pragma unroll
    for (int h = 0; h < NV; ++h) p[u][h] = in ? p[u][h] : 0.0f;
    seg_scan64<NV>(p[u], start_dist(m[u] & le_mask, lane));
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int32_t cw = wb + u * kWin;  // the window's first chunk
    if (cw >= W.nch) break;
    const int32_t c = cw + lane;
    const bool tile_ends = cw + kWin >= W.nch;  // the tile's last window
    if (W.carry) {
      // lanes before the first start (all valid lanes if none) continue it
      const int first = m[u] ? static_cast<int>(__builtin_ctzll(m[u])) : kWin;
      const int hl = min(first, W.nch - cw) - 1;
      if (hl >= 0) {
#pragma unroll
        for (int h = 0; h < NV; ++h)
          W.carry_sum[h] += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(p[u][h]), hl));
      }
      if (m[u] != 0 || tile_ends) {
        if (lane == 0) band_put<NV>(W, W.carry_seg, W.carry_sum);
        W.carry = false;
      }
    }
    // segments that start in this window: stored from their last lane,
    // except the one still open at lane 63, which is carried
    const uint64_t le = m[u] & le_mask;
    const bool next_starts = lane < kWave - 1 && ((m[u] >> (lane + 1)) & 1u) != 0;
    if (c < W.nch && le != 0 && (next_starts || c == W.nch - 1)) band_put<NV>(W, W.seg_base + __popcll(le) - 1, p[u]);
    if (m[u] != 0 && !tile_ends) {
      W.carry = true;
      W.carry_seg = W.seg_base + __popcll(m[u]) - 1;
#pragma unroll
      for (int h = 0; h < NV; ++h)
        W.carry_sum[h] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(p[u][h]), kWave - 1));
    }
    W.seg_base += __popcll(m[u]);
    const int32_t done = W.carry ? W.carry_seg : W.seg_base;  // segments below are finished
    if (done - W.buf_base >= kSegBuf - kWin) band_flush<NV>(W, done, part, lane);
  }
}

// One work tile of the band-staged forward projection, by one wavefront, in
// batches of U windows of 64 chunks (one chunk per lane): the next batch's
// loads are issued before the current batch is summed, so the wavefront
// always has loads in flight.  They are issued even past the tile's end (the
// clamped chunk is re-read): the compiler then counts them, and waits only
// for the batch it sums.  A tile ends with its last segment, so nothing is
// carried into the next tile, whose first segment follows this tile's last.
template <int NV, int WT, int U>
__device__ inline void band_tile(const SysDesc& S, const int32_t* tp, const float* xs, uint32_t xmask,
                                 BandWalk<NV>& W, int lane) {
  constexpr uint32_t kChunkValBytes = SS_CHUNK * NV * (WT == SS_F32 ? 4 : 2);
  constexpr int32_t kStep = kWin * U;
  W.seg_base = __builtin_amdgcn_readfirstlane(tp[2]);
  W.c0 = __builtin_amdgcn_readfirstlane(tp[4]);
  W.nch = __builtin_amdgcn_readfirstlane(tp[5]) - static_cast<int32_t>(W.c0);
  if (W.nch <= 0) return;
  W.tidx = S.fb_idx + W.c0 * SS_CHUNK;
  W.tval = static_cast<const char*>(S.fb_val) + W.c0 * kChunkValBytes;
  W.bits = S.fb_bits + (W.c0 >> 5);  // the word of the tile's first chunk
  W.carry = false;
  W.carry_seg = 0;
#pragma unroll
  for (int h = 0; h < NV; ++h) W.carry_sum[h] = 0.0f;
  BandBatch<NV, U> a, b;
  band_load<NV, WT, U>(a, W, 0, lane);
  // the scheduling barriers keep each batch's loads ahead of the other
  // batch's sums (the scheduler would otherwise hoist work that needs the
  // new loads, and the loads would then be waited for at once)
  for (int32_t wb = 0; wb < W.nch; wb += 2 * kStep) {
    band_load<NV, WT, U>(b, W, wb + kStep, lane);
    __builtin_amdgcn_sched_barrier(0);
    band_windows<NV, U>(a, W, wb, xs, xmask, S.fb_part, lane);
    if (wb + kStep >= W.nch) break;
    __builtin_amdgcn_sched_barrier(0);
    band_load<NV, WT, U>(a, W, wb + 2 * kStep, lane);
    __builtin_amdgcn_sched_barrier(0);
    band_windows<NV, U>(b, W, wb + kStep, xs, xmask, S.fb_part, lane);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Band-staged forward projection.  Block b takes the tiles [b T/G, (b+1)
// T/G) of the T tiles (G blocks), in runs of one band (tiles of a band are
// adjacent): per run the block loads the band of the image into LDS and its
// wavefronts take the run's tiles in turn, each tile whole (band_tile).  Only
// a change of band synchronises the block.  At most 64 registers (80 with
// batches of two windows), so that 8 (6) wavefronts per SIMD fit.
template <int NV, int WT, int U>
__global__ __launch_bounds__(kWave* kBandWaves) __attribute__((amdgpu_waves_per_eu(U > 1 ? 6 : 8))) void k_band_fp(
    const SysDesc* __restrict__ table, const BandTile* __restrict__ tiles, const int32_t* __restrict__ ntiles_p,
    const Params* __restrict__ prm, int parity) {
  extern __shared__ float xs[];
  constexpr int T = kWave * kBandWaves;
  const int lg = prm->band_lg;
  const uint32_t xmask = (1u << lg) - 1u;
  const int lane = lane_id();
  const int64_t nt = *gl(ntiles_p);
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * nt / gridDim.x;
  const int64_t t1 = static_cast<int64_t>(blockIdx.x + 1) * nt / gridDim.x;
  const int32_t* tw = reinterpret_cast<const int32_t*>(tiles);
  constexpr int kTw = sizeof(BandTile) / sizeof(int32_t);
  for (int64_t g0 = t0; g0 < t1;) {
    const int sys = __builtin_amdgcn_readfirstlane(tw[g0 * kTw]);
    const int band = __builtin_amdgcn_readfirstlane(tw[g0 * kTw + 1]);
    // the end of the run of tiles of this band (every wavefront finds it)
    int64_t g1 = g0 + 1;
    for (;;) {
      const int64_t tq = g1 + lane;
      const bool same = tq < t1 && tw[tq * kTw] == sys && tw[tq * kTw + 1] == band;
      const uint64_t diff = ~__ballot(same);
      const int run = diff ? static_cast<int>(__builtin_ctzll(diff)) : kWave;
      g1 += run;
      if (run < kWave) break;
    }
    const SysDesc& S = table[sys];
    if (!*gl(&S.st->stop)) {
      const int64_t j0 = static_cast<int64_t>(band) << lg;
      stage_contiguous<NV, T>(xs, S.f[parity] + j0 * NV, min(static_cast<int64_t>(1) << lg, S.n - j0));
      __syncthreads();
      // each wavefront takes a contiguous part of the run, so that its
      // segments follow on and its buffer is written out in long runs
      const int64_t a = g0 + (g1 - g0) * wave_id() / kBandWaves;
      const int64_t b = g0 + (g1 - g0) * (wave_id() + 1) / kBandWaves;
      if (a < b) {
        BandWalk<NV> W;
        W.buf = xs + (NV << lg) + wave_id() * (kSegBuf * NV);
        W.buf_base = __builtin_amdgcn_readfirstlane(tw[a * kTw + 2]);
        for (int64_t t = a; t < b; ++t) band_tile<NV, WT, U>(S, tw + t * kTw, xs, xmask, W, lane);
        band_flush<NV>(W, W.seg_base, S.fb_part, lane);
      }
      __syncthreads();  // the next run's band overwrites xs
    }
    g0 = g1;
  }
}

// The residual of the band-staged forward projection: per row, its
// segments' sums added in band order (through the row's slots), r = p - q, z = r / W, and the block's FP64
// partial of |r|^2; the first block of a system moves the iterate index on.
// One wavefront per block of kFinThreads rows, kFinRows rows per lane: the
// loads of a lane's rows (their slot ranges, then each row's first slot and
// partial, p and 1/W) are issued together, so a block waits for the chain
// offsets -> slot -> partial once rather than once per 64 rows (this kernel
// is bound by that chain's latencies, not by its bytes).
constexpr int kFinRows = kFinThreads / kWave;

template <int NV>
__global__ __launch_bounds__(kWave) void k_band_fin(const SysDesc* __restrict__ table, int nsys,
                                                    const Params* __restrict__ prm) {
  const int s = sys_of<0>(prm, nsys, blockIdx.x);
  const SysDesc& S = table[s];
  if (*gl(&S.st->stop)) return;
  const int64_t lb = static_cast<int64_t>(blockIdx.x) - S.fp_block0;
  const int lane = lane_id();
  // Every load below is unconditional, from a clamped index that is always
  // valid (row 0; slot and partial 0, which the layout always holds), and
  // its value is dropped at use where it does not apply: conditional loads
  // would make the compiler wait for them where the branches meet.
  int64_t ii[kFinRows], ic[kFinRows];
  uint32_t q0[kFinRows], q1[kFinRows];
#pragma unroll
  for (int rr = 0; rr < kFinRows; ++rr) {
    ii[rr] = lb * kFinThreads + rr * kWave + lane;
    ic[rr] = ii[rr] < S.m ? ii[rr] : 0;
    q0[rr] = gl(S.fb_rseg)[ic[rr]];
    q1[rr] = gl(S.fb_rseg)[ic[rr] + 1];
  }
  Vec<NV> pv[kFinRows], first[kFinRows];
  float w[kFinRows];
#pragma unroll
  for (int rr = 0; rr < kFinRows; ++rr) {
    pv[rr] = load_vec<NV>(S.p, ic[rr]);
    w[rr] = gl(S.inv_row)[ic[rr]];
  }
  int32_t sl[kFinRows];
#pragma unroll
  for (int rr = 0; rr < kFinRows; ++rr) sl[rr] = gl(S.fb_slot)[q0[rr] < q1[rr] ? q0[rr] : 0u];
#pragma unroll
  for (int rr = 0; rr < kFinRows; ++rr) first[rr] = load_vec<NV>(S.fb_part, q0[rr] < q1[rr] ? sl[rr] : 0);
  double d = 0.0;
#pragma unroll
  for (int rr = 0; rr < kFinRows; ++rr) {
    if (ii[rr] >= S.m) continue;
    // the row's segments' sums in slot order, from 0 as before
    float acc[NV];
#pragma unroll
    for (int h = 0; h < NV; ++h) acc[h] = 0.0f;
    if (q0[rr] < q1[rr]) {
#pragma unroll
      for (int h = 0; h < NV; ++h) acc[h] += first[rr].v[h];
    }
    for (uint32_t q = q0[rr] + 1; q < q1[rr]; ++q) {
      const Vec<NV> v = load_vec<NV>(S.fb_part, gl(S.fb_slot)[q]);
#pragma unroll
      for (int h = 0; h < NV; ++h) acc[h] += v.v[h];
    }
    Vec<NV> zv;
#pragma unroll
    for (int h = 0; h < NV; ++h) {
      const float r = pv[rr].v[h] - acc[h];
      zv.v[h] = r * w[rr];
      d += static_cast<double>(r) * static_cast<double>(r);
    }
    store_vec<NV>(S.z, ii[rr], zv);
  }
  const double tot = group_sum<kWave>(d);
  if (lane == 0) {
    glw(S.partials)[lb] = tot;
    SysState* st = S.st;
    if (lb == 0 && *gl(&st->pending)) {
      glw(&st->k)[0] += 1;
      glw(&st->pending)[0] = 0;
    }
  }
}

// Back-projection plan of one tile (one block per tile, all systems): a
// bitmap of the rows that the tile's columns touch, its runs of consecutive
// set bits (first row, first LDS slot), and each entry's rank among the
// set bits.  LDS: three arrays of ceil(m/32) words.
constexpr int kPlanAhead = 4;  // entries per thread whose loads are in flight together
__global__ __launch_bounds__(kStagedThreads) void k_bt_plan(const SysDesc* table, int nsys, const Params* prm) {
  extern __shared__ uint32_t bw[];
  constexpr int T = kStagedThreads;
  __shared__ uint32_t tsum[2][T];
  const int s = sys_of<1>(prm, nsys, blockIdx.x);
  const SysDesc& S = table[s];
  const int64_t lt = static_cast<int64_t>(blockIdx.x) - S.bp_block0;
  const int64_t j0 = lt << prm->tile_lg;
  const int64_t j1 = min(S.n, j0 + (int64_t{1} << prm->tile_lg));
  const int words = static_cast<int>((S.m + 31) / 32);
  uint32_t* bm = bw;
  uint32_t* pre = bw + words;
  uint32_t* rpre = bw + 2 * words;
  for (int w = threadIdx.x; w < words; w += T) bm[w] = 0u;
  __syncthreads();
  const int64_t k0 = gl(S.col_ptr)[j0], k1 = gl(S.col_ptr)[j1];
  // kPlanAhead entries per thread and pass, their loads issued together
  // (from clamped indices, values past the tile dropped): the tile's
  // entries cost a few memory latencies, not one per entry a thread takes
  for (int64_t kb = k0 + threadIdx.x; kb < k1; kb += static_cast<int64_t>(T) * kPlanAhead) {
    int32_t rv[kPlanAhead];
#pragma unroll
    for (int u = 0; u < kPlanAhead; ++u) {
      const int64_t k = kb + static_cast<int64_t>(u) * T;
      rv[u] = gl(S.row_idx)[k < k1 ? k : k1 - 1];
    }
#pragma unroll
    for (int u = 0; u < kPlanAhead; ++u) {
      const int32_t r = rv[u];
      if (kb + static_cast<int64_t>(u) * T < k1 && r >= 0 && r < S.m) atomicOr(&bm[r >> 5], 1u << (r & 31));
    }
  }
  __syncthreads();
  // counts of set bits and of run starts per word, scanned over the words
  // (each thread a contiguous chunk, then the chunk totals across threads)
  const int chunk = (words + T - 1) / T;
  const int w0 = static_cast<int>(threadIdx.x) * chunk, w1 = min(words, w0 + chunk);
  uint32_t cb = 0, cr = 0;
  for (int w = w0; w < w1; ++w) {
    const uint32_t v = bm[w];
    const uint32_t carry = w > 0 ? bm[w - 1] >> 31 : 0u;
    const uint32_t starts = v & ~((v << 1) | carry);
    pre[w] = cb;
    rpre[w] = cr;
    cb += __popc(v);
    cr += __popc(starts);
  }
  tsum[0][threadIdx.x] = cb;
  tsum[1][threadIdx.x] = cr;
  __syncthreads();
  for (int o = 1; o < T; o <<= 1) {
    const uint32_t a = threadIdx.x >= static_cast<unsigned>(o) ? tsum[0][threadIdx.x - o] : 0u;
    const uint32_t b = threadIdx.x >= static_cast<unsigned>(o) ? tsum[1][threadIdx.x - o] : 0u;
    __syncthreads();
    tsum[0][threadIdx.x] += a;
    tsum[1][threadIdx.x] += b;
    __syncthreads();
  }
  const uint32_t bb = tsum[0][threadIdx.x] - cb, rb = tsum[1][threadIdx.x] - cr;
  for (int w = w0; w < w1; ++w) {
    pre[w] += bb;
    rpre[w] += rb;
  }
  const uint32_t rows = tsum[0][T - 1], runs = tsum[1][T - 1];
  const bool ok = rows <= static_cast<uint32_t>(kBtMaxRows) && runs <= static_cast<uint32_t>(kBtRunCap);
  if (threadIdx.x == 0) {
    auto* mt = glw(reinterpret_cast<int32_t*>(S.bt_meta + lt));
    mt[0] = static_cast<int32_t>(rows);
    mt[1] = static_cast<int32_t>(runs);
    mt[2] = ok ? 1 : 0;
    mt[3] = 0;
  }
  __syncthreads();
  if (!ok) return;
  int32_t* runs_out = S.bt_runs + 2 * lt * kBtRunCap;
  for (int w = threadIdx.x; w < words; w += T) {
    const uint32_t v = bm[w];
    const uint32_t carry = w > 0 ? bm[w - 1] >> 31 : 0u;
    uint32_t starts = v & ~((v << 1) | carry);
    uint32_t ri = rpre[w];
    while (starts) {
      const int bit = __builtin_ctz(starts);
      starts &= starts - 1;
      const uint32_t slot = pre[w] + __popc(v & ((1u << bit) - 1u));
      glw(runs_out)[2 * ri] = w * 32 + bit;
      glw(runs_out)[2 * ri + 1] = static_cast<int32_t>(slot);
      ++ri;
    }
  }
  for (int64_t kb = k0 + threadIdx.x; kb < k1; kb += static_cast<int64_t>(T) * kPlanAhead) {
    int32_t rv[kPlanAhead];
#pragma unroll
    for (int u = 0; u < kPlanAhead; ++u) {
      const int64_t k = kb + static_cast<int64_t>(u) * T;
      rv[u] = gl(S.row_idx)[k < k1 ? k : k1 - 1];
    }
#pragma unroll
    for (int u = 0; u < kPlanAhead; ++u) {
      const int64_t k = kb + static_cast<int64_t>(u) * T;
      if (k >= k1) break;
      const int32_t r = rv[u];
      const int32_t rr = r >= 0 && r < S.m ? r : 0;
      const uint32_t rank = pre[rr >> 5] + __popc(bm[rr >> 5] & ((1u << (rr & 31)) - 1u));
      glw(S.bt_idx)[k] = static_cast<uint16_t>(rank < rows ? rank : 0u);
    }
  }
}

// Tile-staged back projection: one block per tile of 2^tile_lg columns.
// The tile's rows of z go into LDS (runs dealt to the wavefronts), then CPW
// columns per wavefront are summed from there and updated.  A tile whose
// rows did not fit keeps global gathers.  The first tile of a system also
// finalises the residual.
template <int NV, int WT, int CPW, int P>
__global__ __launch_bounds__(kStagedThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_tile_bp(const Params* __restrict__ prm,
                                                            const SysDesc* __restrict__ table, int nsys,
                                                            int parity) {
  extern __shared__ float zs[];
  __shared__ double red[kStagedWaves];
  constexpr int L = kWave / CPW;
  const int s = sys_of<1>(prm, nsys, blockIdx.x);
  const SysDesc& S = table[s];
  if (*gl(&S.st->stop)) return;
  const int64_t lt = static_cast<int64_t>(blockIdx.x) - S.bp_block0;
  if (lt == 0) {
    finalize_residual<kStagedWaves>(prm, S, red);
    __syncthreads();
  }
  if (*gl(&S.st->k) >= prm->max_iter) return;
  const int lg = prm->tile_lg;
  const int64_t j0 = lt << lg;
  const int64_t j1 = min(S.n, j0 + (int64_t{1} << lg));
  // the first pass's column offsets, before the tile's rows are staged
  int64_t j = j0 + wave_id() * CPW + lane_id() / L;
  int64_t jj = j < j1 ? j : j1 - 1;
  int64_t nlo = gl(S.col_ptr)[jj], nhi = gl(S.col_ptr)[jj + 1];
  const int32_t* mt = reinterpret_cast<const int32_t*>(S.bt_meta + lt);
  const int32_t nrows = gl(mt)[0], nruns = gl(mt)[1];
  const bool staged = gl(mt)[2] != 0;
  if (staged) {
    const int32_t* runs = S.bt_runs + 2 * lt * kBtRunCap;
    for (int r = wave_id(); r < nruns; r += kStagedWaves) {
      const int32_t first = gl(runs)[2 * r], slot = gl(runs)[2 * r + 1];
      const int32_t end = r + 1 < nruns ? gl(runs)[2 * r + 3] : nrows;
      for (int q = lane_id(); q < end - slot; q += kWave) {
        const Vec<NV> zv = load_vec<NV>(S.z, first + q);
#pragma unroll
        for (int h = 0; h < NV; ++h) zs[(slot + q) * NV + h] = zv.v[h];
      }
    }
    __syncthreads();
  }
  const int glane = lane_id() % L;
  const float* fin = S.f[parity];
  // each pass loads the next pass's column offsets before its own streams
  for (int64_t jb = j0; jb < j1; jb += kStagedWaves * CPW) {
    const int64_t jc = j, jjc = jj;
    const bool owner = glane == 0 && jc < j1;
    const int64_t lo = nlo, hi = jc < j1 ? nhi : nlo;
    j += kStagedWaves * CPW;
    jj = j < j1 ? j : j1 - 1;
    nlo = gl(S.col_ptr)[jj];
    nhi = gl(S.col_ptr)[jj + 1];
    Vec<NV> fv = load_vec<NV>(fin, jjc);
    const float tl = prm->lambda * gl(S.inv_col)[jjc];
    float acc[NV];
#pragma unroll
    for (int h = 0; h < NV; ++h) acc[h] = 0.0f;
    if (staged) line_dot_lds<NV, WT, L, P>(S.bt_idx, S.val_t, zs, lo, hi, glane, acc, kBtMaxRows - 1u);
    else line_dot_c<NV, WT, L, P>(S.row_idx, S.val_t, S.z, lo, hi, glane, acc);
#pragma unroll
    for (int h = 0; h < NV; ++h) acc[h] = group_sum<L>(acc[h]);
    if (owner) {
#pragma unroll
      for (int h = 0; h < NV; ++h) fv.v[h] = fmaf(tl, acc[h], fv.v[h]);
      if (prm->nonneg) fv = project_nonneg<NV>(fv);
      store_vec<NV>(S.f[parity ^ 1], jc, fv);
    }
  }
}

// Sizes of the staged forms (one thread): forward segments and work tiles,
// back-projection tiles, how many of them are staged and the rows they stage.
__global__ void k_staged_info(const SysDesc* table, int nsys, int stg, const int32_t* ntiles, int64_t* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t segs = 0, bt = 0, ok = 0, rows = 0;
  for (int s = 0; s < nsys; ++s) {
    const SysDesc& S = table[s];
    if (stg & 1) segs += seg_count(S.fb_len[static_cast<int64_t>(S.fb_nb) * S.m]);
    if (stg & 2) {
      for (int32_t t = 0; t < S.bp_nblocks; ++t) {
        const int32_t* mt = reinterpret_cast<const int32_t*>(S.bt_meta + t);
        ++bt;
        if (mt[2]) {
          ++ok;
          rows += mt[0];
        }
      }
    }
  }
  out[0] = segs;
  out[1] = (stg & 1) ? *ntiles : 0;
  out[2] = bt;
  out[3] = ok;
  out[4] = rows;
}

// ---- device code end

// ------------------------------------------------------------------ host
struct Layout {
  size_t params, table, states, z, partials, total;
  std::vector<size_t> z_off, part_off, f_off;
  // interleaved copies of the row (forward) and column (back) streams
  std::vector<size_t> fi_idx, fi_val, bi_idx, bi_val;
  // staged forms (per system) and their set-up scratch (shared)
  std::vector<size_t> fb_idx, fb_val, fb_len, fb_rseg, fb_off, fb_slot, fb_part, fb_bits, bt_idx, bt_meta, bt_runs;
  size_t fb_len_lo = 0, fb_len_hi = 0, fb_rseg_lo = 0, fb_rseg_hi = 0, fb_bits_lo = 0, fb_bits_hi = 0;
  size_t tiles = 0, ntiles = 0, pair_t0 = 0, pieces64 = 0, pieces32 = 0, tsum64 = 0, tsum32 = 0, info = 0;
  size_t b2s[3] = {0, 0, 0};  // block -> system tables of the staged grids (0: none)
  int64_t tile_cap = 0, t64 = 0, t32 = 0, npairs = 0;
};

// Stream form of each kernel from the chunked option: bit 2 (bit 3) selects
// the interleaved form for the forward (back) projection, else bit 0 (bit 1)
// the chunked one.
inline int fp_form(int ch) { return (ch & 4) ? 2 : (ch & 1); }
inline int bp_form(int ch) { return (ch & 8) ? 2 : ((ch >> 1) & 1); }

// Systems whose lines are stored interleaved (row_lanes / col_lanes) are
// read in place with the interleaved form; others get workspace copies.
inline int effective_chunked(const ss_system* sys, int ch) {
  return ch | (sys[0].row_lanes ? 4 : 0) | (sys[0].col_lanes ? 8 : 0);
}

inline size_t value_bytes(const ss_system& S) { return static_cast<size_t>(S.nvals) * (S.wdtype == SS_F32 ? 4 : 2); }

inline size_t align256(size_t v) { return (v + 255) & ~size_t{255}; }

// Staged-form sizes shared by the layout and the set-up.
inline int band_lg_of(const ss_sart_opts* o) { return o->band_width ? __builtin_ctz(o->band_width) : 12; }
inline int tile_lg_of(const ss_sart_opts* o) { return o->tile_cols ? __builtin_ctz(o->tile_cols) : 10; }
inline int band_q_of(const ss_sart_opts* o) { return (o->tile_entries ? o->tile_entries : 2048) / SS_CHUNK; }
inline int64_t bands_of(const ss_system& S, int lg) { return (S.n + (int64_t{1} << lg) - 1) >> lg; }
inline int64_t seg_bound(const ss_system& S, int lg) { return std::min<int64_t>(S.nnz, bands_of(S, lg) * S.m) + 1; }
// entries of the band-major copy at most: every segment padded by up to
// SS_CHUNK - 1 entries
inline int64_t padded_bound(const ss_system& S, int lg) {
  return S.nnz + (SS_CHUNK - 1) * (seg_bound(S, lg) - 1) + SS_CHUNK;
}
inline int64_t pscan_tiles(int64_t len) { return (len + kPScanTile - 1) / kPScanTile; }
inline size_t stream_cap(int64_t nnz) { return static_cast<size_t>(ss_stream_len(nnz) > 0 ? ss_stream_len(nnz) : 4); }

Layout make_layout(const ss_system* sys, int nsys, const ss_sart_opts* opt) {
  const int ch = effective_chunked(sys, opt->chunked);
  const int stg = opt->staged;
  Layout L;
  size_t o = 0;
  L.params = o;
  o += align256(sizeof(Params));
  L.table = o;
  o += align256(sizeof(SysDesc) * nsys);
  L.states = o;
  o += align256(sizeof(SysState) * nsys);
  L.z = o;
  for (int s = 0; s < nsys; ++s) {
    L.z_off.push_back(o);
    o += align256(sizeof(float) * static_cast<size_t>(sys[s].m * sys[s].nvals));
  }
  for (int s = 0; s < nsys; ++s) {
    L.f_off.push_back(o);
    o += align256(sizeof(float) * static_cast<size_t>(sys[s].n * sys[s].nvals));
  }
  L.partials = o;
  for (int s = 0; s < nsys; ++s) {
    L.part_off.push_back(o);
    // the most forward-projection blocks any configuration uses: 1 row per wave
    o += align256(sizeof(double) * static_cast<size_t>((sys[s].m + kWPB - 1) / kWPB));
  }
  for (int s = 0; s < nsys; ++s) {
    const size_t cap = static_cast<size_t>(sys[s].nnz) + SS_CHUNK;
    for (int which = 0; which < 2; ++which) {
      if (!(which ? bp_form(ch) == 2 && !sys[s].col_lanes && !(stg & 2)
                  : fp_form(ch) == 2 && !sys[s].row_lanes && !(stg & 1)))
        continue;
      (which ? L.bi_idx : L.fi_idx).push_back(o);
      o += align256(sizeof(int32_t) * cap);
      (which ? L.bi_val : L.fi_val).push_back(o);
      o += align256(value_bytes(sys[s]) * cap);
    }
  }
  if (stg & 1) {
    const int lg = band_lg_of(opt);
    const int q = band_q_of(opt);
    for (int s = 0; s < nsys; ++s) {
      const ss_system& S = sys[s];
      const int64_t nsb = seg_bound(S, lg);
      const int64_t pe = padded_bound(S, lg);
      L.fb_idx.push_back(o);
      o += align256(sizeof(uint16_t) * static_cast<size_t>(pe));
      L.fb_val.push_back(o);
      o += align256(value_bytes(S) * static_cast<size_t>(pe));
      L.fb_off.push_back(o);
      o += align256(sizeof(int32_t) * static_cast<size_t>(nsb + 1));
      L.fb_slot.push_back(o);
      o += align256(sizeof(int32_t) * static_cast<size_t>(nsb));
      L.fb_part.push_back(o);
      o += align256(sizeof(float) * S.nvals * static_cast<size_t>(nsb));
      L.tile_cap += bands_of(S, lg) + pe / SS_CHUNK / q + 1;
      L.npairs += bands_of(S, lg);
      L.t64 += pscan_tiles(bands_of(S, lg) * S.m + 1);
      L.t32 += pscan_tiles(S.m + 1);
    }
    // the arrays the set-up clears, each kind in one contiguous range
    L.fb_len_lo = o;
    for (int s = 0; s < nsys; ++s) {
      L.fb_len.push_back(o);
      o += align256(sizeof(uint64_t) * static_cast<size_t>(bands_of(sys[s], lg) * sys[s].m + 1));
    }
    L.fb_len_hi = o;
    L.fb_rseg_lo = o;
    for (int s = 0; s < nsys; ++s) {
      L.fb_rseg.push_back(o);
      o += align256(sizeof(uint32_t) * static_cast<size_t>(sys[s].m + 1));
    }
    L.fb_rseg_hi = o;
    L.fb_bits_lo = o;
    for (int s = 0; s < nsys; ++s) {
      L.fb_bits.push_back(o);
      // one bit per chunk, plus the words a window's mask reads past the last
      o += align256(sizeof(uint32_t) * static_cast<size_t>(padded_bound(sys[s], lg) / SS_CHUNK / 32 + 3));
    }
    L.fb_bits_hi = o;
    L.pair_t0 = o;
    o += align256(sizeof(int32_t) * static_cast<size_t>(L.npairs + 1));
    L.tiles = o;
    o += align256(sizeof(BandTile) * static_cast<size_t>(L.tile_cap + 1));
    L.ntiles = o;
    o += 256;
    L.pieces64 = o;
    o += align256(sizeof(ScanPiece<uint64_t>) * nsys);
    L.pieces32 = o;
    o += align256(sizeof(ScanPiece<uint32_t>) * nsys);
    L.tsum64 = o;
    o += align256(sizeof(uint64_t) * static_cast<size_t>(L.t64));
    L.tsum32 = o;
    o += align256(sizeof(uint32_t) * static_cast<size_t>(L.t32));
  }
  if (stg) {
    L.info = o;
    o += 256;
  }
  if (stg && nsys > 1) {
    const int lg = tile_lg_of(opt);
    int64_t nb[3] = {0, 0, 0};
    for (int s = 0; s < nsys; ++s) {
      nb[0] += (sys[s].m + kFinThreads - 1) / kFinThreads;
      nb[1] += (sys[s].n + (int64_t{1} << lg) - 1) >> lg;
      nb[2] += (sys[s].m + kCvRows - 1) / kCvRows;
    }
    for (int k = 0; k < 3; ++k) {
      if (k == 0 && !(stg & 1)) continue;
      if (k == 1 && !(stg & 2)) continue;
      if (k == 2 && !(stg & 1)) continue;
      L.b2s[k] = o;
      o += align256(sizeof(int32_t) * static_cast<size_t>(nb[k]));
    }
  }
  if (stg & 2) {
    const int lg = tile_lg_of(opt);
    for (int s = 0; s < nsys; ++s) {
      const ss_system& S = sys[s];
      const size_t nt = static_cast<size_t>((S.n + (int64_t{1} << lg) - 1) >> lg);
      L.bt_idx.push_back(o);
      o += align256(sizeof(uint16_t) * stream_cap(S.nnz));
      L.bt_meta.push_back(o);
      o += align256(sizeof(BtMeta) * nt);
      L.bt_runs.push_back(o);
      o += align256(2 * sizeof(int32_t) * kBtRunCap * nt);
    }
  }
  L.total = o;
  return L;
}

struct Cfg {
  int nv, wt, rpw, cpw, xcd, u, pers, ch;
  int stg, blg, tlg, bq;  // staged forms: bits, log2 band width, log2 tile columns, chunks per forward tile
};

ss_status validate(const ss_system* sys, int nsys, const ss_sart_opts* o, const char* fn) {
  if (!sys || nsys <= 0 || !o) return fail(SS_E_ARG, "%s: NULL systems or options", fn);
  for (int s = 0; s < nsys; ++s) {
    const ss_system& S = sys[s];
    if (S.m <= 0 || S.n <= 0 || S.nnz < 0) return fail(SS_E_ARG, "%s: system %d has a bad size", fn, s);
    if (S.nvals != sys[0].nvals || S.wdtype != sys[0].wdtype)
      return fail(SS_E_ARG, "%s: all systems of one call must share nvals and wdtype", fn);
    if (S.nvals != 1 && S.nvals != 2) return fail(SS_E_ARG, "%s: nvals must be 1 or 2", fn);
    if (S.wdtype != SS_F32 && S.wdtype != SS_BF16 && S.wdtype != SS_F16)
      return fail(SS_E_ARG, "%s: unknown wdtype", fn);
    if (!S.row_ptr || !S.col_ptr || !S.p || !S.inv_row || !S.inv_col ||
        (S.nnz > 0 && (!S.col_idx || !S.val || !S.row_idx || !S.val_t)))
      return fail(SS_E_ARG, "%s: system %d has a NULL array", fn, s);
    auto aligned = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    if (S.nnz > 0 && !(aligned(S.col_idx) && aligned(S.val) && aligned(S.row_idx) && aligned(S.val_t)))
      return fail(SS_E_ARG, "%s: system %d: index and value arrays must be 16-byte aligned", fn, s);
    if (S.m > INT32_MAX || S.n > INT32_MAX) return fail(SS_E_ARG, "%s: system %d too large", fn, s);
    if (ss_status e = check_lanes(&S, fn)) return e;
    if (S.row_lanes != sys[0].row_lanes || S.col_lanes != sys[0].col_lanes)
      return fail(SS_E_ARG, "%s: all systems of one call must share row_lanes and col_lanes", fn);
  }
  if (sys[0].row_lanes && o->rows_per_wave && o->rows_per_wave != kWave / sys[0].row_lanes)
    return fail(SS_E_ARG, "%s: rows stored for %d lanes need rows_per_wave %d (or 0)", fn, sys[0].row_lanes,
                kWave / sys[0].row_lanes);
  if (sys[0].col_lanes && o->cols_per_wave && o->cols_per_wave != kWave / sys[0].col_lanes)
    return fail(SS_E_ARG, "%s: columns stored for %d lanes need cols_per_wave %d (or 0)", fn, sys[0].col_lanes,
                kWave / sys[0].col_lanes);
  if (!(o->lambda > 0.0f && o->lambda < 2.0f)) return fail(SS_E_ARG, "%s: lambda must be in (0, 2)", fn);
  if (o->max_iter < 0 || o->max_iter > (1 << 30)) return fail(SS_E_ARG, "%s: bad max_iter", fn);
  if (o->tol > 0.0 && o->check_every <= 0) return fail(SS_E_ARG, "%s: check_every must be > 0", fn);
  auto ok_pw = [](int v, int maxv) { return v == 0 || (v > 0 && v <= maxv && (v & (v - 1)) == 0); };
  if (!ok_pw(o->rows_per_wave, 8)) return fail(SS_E_ARG, "%s: rows_per_wave must be 0,1,2,4,8", fn);
  if (!ok_pw(o->cols_per_wave, 16)) return fail(SS_E_ARG, "%s: cols_per_wave must be 0,1,2,4,8,16", fn);
  if (o->unroll != 0 && o->unroll != 4 && o->unroll != 8) return fail(SS_E_ARG, "%s: unroll must be 0, 4 or 8", fn);
  if (o->chunked < 0 || o->chunked > 15) return fail(SS_E_ARG, "%s: chunked must be 0..15", fn);
  if ((effective_chunked(sys, o->chunked) & 12) && sys[0].nvals == 1 && sys[0].wdtype != SS_F32)
    return fail(SS_E_ARG, "%s: the interleaved stream form needs entries of at least 4 bytes", fn);
  if (o->nonneg != 0 && o->nonneg != 1) return fail(SS_E_ARG, "%s: nonneg must be 0 or 1", fn);
  if (o->staged < 0 || o->staged > 3) return fail(SS_E_ARG, "%s: staged must be 0..3", fn);
  if (o->residual_every > 1) return fail(SS_E_ARG, "%s: residual_every is for ordered subsets (0 or 1 here)", fn);
  auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
  if (o->band_width && (!pow2(o->band_width) || o->band_width < 1024 || o->band_width > 16384))
    return fail(SS_E_ARG, "%s: band_width must be a power of two in 1024..16384", fn);
  if (o->tile_cols && (!pow2(o->tile_cols) || o->tile_cols < 64 || o->tile_cols > 8192))
    return fail(SS_E_ARG, "%s: tile_cols must be a power of two in 64..8192", fn);
  if (o->tile_entries && (o->tile_entries % 256 != 0 || o->tile_entries < 1024 || o->tile_entries > 65536))
    return fail(SS_E_ARG, "%s: tile_entries must be a multiple of 256 in 1024..65536", fn);
  if ((o->staged & 1) && band_lds_bytes(sys[0].nvals, band_lg_of(o)) > 65536)
    return fail(SS_E_ARG, "%s: the staged forward projection needs band_width*nvals*4 + 16384*nvals <= 65536", fn);
  if (o->staged) {
    for (int s = 0; s < nsys; ++s) {
      const ss_system& S = sys[s];
      if (((o->staged & 1) && S.row_lanes) || ((o->staged & 2) && S.col_lanes))
        return fail(SS_E_ARG, "%s: the staged forms need lines in ascending order (row_lanes/col_lanes 0)", fn);
      if (S.nnz >= INT32_MAX) return fail(SS_E_ARG, "%s: the staged forms need nnz < 2^31", fn);
      if ((o->staged & 1) && padded_bound(S, band_lg_of(o)) >= INT32_MAX)
        return fail(SS_E_ARG, "%s: system %d: the padded band-major copy needs fewer than 2^31 entries", fn, s);
      if ((o->staged & 1) && bands_of(S, band_lg_of(o)) * S.m + 1 >= INT32_MAX)
        return fail(SS_E_ARG, "%s: system %d has too many (band, row) pairs for the staged forward form", fn, s);
      if ((o->staged & 2) && S.m > (int64_t{1} << 17))
        return fail(SS_E_ARG, "%s: the staged back projection needs m <= 2^17", fn);
    }
  }
  return SS_OK;
}

// The band-staged forward kernel loads the image in 16-byte pieces.
ss_status check_images(const ss_system* sys, int nsys, float* const* f, const ss_sart_opts* o, const char* fn) {
  if (!f) return fail(SS_E_ARG, "%s: NULL images", fn);
  for (int s = 0; s < nsys; ++s) {
    if (!f[s]) return fail(SS_E_ARG, "%s: NULL image %d", fn, s);
    if ((o->staged & 1) && (reinterpret_cast<uintptr_t>(f[s]) & 15u))
      return fail(SS_E_ARG, "%s: the staged forward projection needs 16-byte aligned images (image %d)", fn, s);
  }
  (void)sys;
  return SS_OK;
}

int pick_per_wave(double mean_len, int maxv) {
  int v = 1;
  while (v < maxv && mean_len * v < 48.0) v <<= 1;
  return v;
}

Cfg choose_cfg(const ss_system* sys, int nsys, const ss_sart_opts* o) {
  double nnz = 0, m = 0, n = 0;
  for (int s = 0; s < nsys; ++s) {
    nnz += static_cast<double>(sys[s].nnz);
    m += static_cast<double>(sys[s].m);
    n += static_cast<double>(sys[s].n);
  }
  Cfg c;
  c.nv = sys[0].nvals;
  c.wt = sys[0].wdtype;
  c.rpw = sys[0].row_lanes ? kWave / sys[0].row_lanes
         : o->rows_per_wave ? o->rows_per_wave : pick_per_wave(nnz / m, 8);
  c.cpw = sys[0].col_lanes ? kWave / sys[0].col_lanes
         : o->cols_per_wave ? o->cols_per_wave : pick_per_wave(nnz / n, 16);
  c.xcd = o->xcd_remap ? 1 : 0;
  c.u = o->unroll ? o->unroll : 4;
  c.ch = effective_chunked(sys, o->chunked);
  c.pers = o->persistent ? 1 : 0;
  c.stg = o->staged;
  c.blg = band_lg_of(o);
  c.tlg = tile_lg_of(o);
  c.bq = band_q_of(o);
  if (c.stg & 1) c.rpw = o->rows_per_wave ? o->rows_per_wave : 4;
  if (c.stg & 2) c.cpw = o->cols_per_wave ? o->cols_per_wave : 8;
  return c;
}

struct Grids {
  uint32_t fp_blocks, bp_blocks;
  uint32_t band_blocks;  // grid of the band-staged forward kernel
  uint32_t cv_blocks;    // set-up grid over rows
};

// Grid of the band-staged forward kernel: the blocks that fit on the device
// at once (its LDS decides), at most one per possible tile; each block then
// takes a contiguous run of the tiles.
uint32_t band_grid(const Cfg& c, const Layout& L) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int>, uint32_t> cap;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const size_t lds = band_lds_bytes(c.nv, c.blg);
  uint32_t resident;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_tuple(dev, c.nv, c.blg, c.bq);
    auto it = cap.find(key);
    if (it == cap.end()) {
      int cus = 0, per = 0;
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      const void* k = c.nv == 2 ? reinterpret_cast<const void*>(k_band_fp<2, SS_F32, 1>)
                                : reinterpret_cast<const void*>(k_band_fp<1, SS_F32, 1>);
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, kWave * kBandWaves, lds);
      it = cap.emplace(key, static_cast<uint32_t>(std::max(1, cus) * std::max(1, per))).first;
    }
    resident = it->second;
  }
  const int64_t tiles = std::max<int64_t>(1, L.tile_cap);
  return static_cast<uint32_t>(std::min<int64_t>(tiles, resident));
}

// Builds the staged forms of every system in the workspace (see staged.h):
// for the forward projection the band-major streams, segment offsets and
// slots and the work tiles; for the back projection the tiles' row plans and
// ranks.  All systems in one launch per phase.
ss_status build_staged(const ss_system* sys, int nsys, const Cfg& c, const Layout& L, char* ws, const Grids& g,
                       hipStream_t st) {
  const SysDesc* table = reinterpret_cast<const SysDesc*>(ws + L.table);
  const Params* dprm = reinterpret_cast<const Params*>(ws + L.params);
  if (c.stg & 1) {
    const int64_t n64 = static_cast<int64_t>((L.fb_len_hi - L.fb_len_lo) / sizeof(uint64_t));
    const int64_t n32 = static_cast<int64_t>((L.fb_rseg_hi - L.fb_rseg_lo) / sizeof(uint32_t));
    k_fill_zero<uint64_t><<<2048, 256, 0, st>>>(reinterpret_cast<uint64_t*>(ws + L.fb_len_lo), n64);
    k_fill_zero<uint32_t><<<512, 256, 0, st>>>(reinterpret_cast<uint32_t*>(ws + L.fb_rseg_lo), n32);
    const int64_t nbits = static_cast<int64_t>((L.fb_bits_hi - L.fb_bits_lo) / sizeof(uint32_t));
    k_fill_zero<uint32_t><<<512, 256, 0, st>>>(reinterpret_cast<uint32_t*>(ws + L.fb_bits_lo), nbits);
    k_fb_count<<<g.cv_blocks, kThreads, 0, st>>>(table, nsys, dprm);
    auto* p64 = reinterpret_cast<ScanPiece<uint64_t>*>(ws + L.pieces64);
    auto* p32 = reinterpret_cast<ScanPiece<uint32_t>*>(ws + L.pieces32);
    auto* t64 = reinterpret_cast<uint64_t*>(ws + L.tsum64);
    auto* t32 = reinterpret_cast<uint32_t*>(ws + L.tsum32);
    const unsigned pb = static_cast<unsigned>((nsys + 63) / 64);
    k_make_pieces<<<pb, 64, 0, st>>>(table, nsys, p64, p32);
    k_pscan_tiles<uint64_t><<<static_cast<unsigned>(L.t64), kPScanThreads, 0, st>>>(p64, nsys, t64);
    k_pscan_bases<uint64_t><<<pb, 64, 0, st>>>(p64, nsys, t64);
    k_pscan_apply<uint64_t><<<static_cast<unsigned>(L.t64), kPScanThreads, 0, st>>>(p64, nsys, t64);
    k_pscan_tiles<uint32_t><<<static_cast<unsigned>(L.t32), kPScanThreads, 0, st>>>(p32, nsys, t32);
    k_pscan_bases<uint32_t><<<pb, 64, 0, st>>>(p32, nsys, t32);
    k_pscan_apply<uint32_t><<<static_cast<unsigned>(L.t32), kPScanThreads, 0, st>>>(p32, nsys, t32);
    const size_t vb = value_bytes(sys[0]);
    if (vb == 8) k_fb_fill<8><<<g.cv_blocks, kThreads, 0, st>>>(table, nsys, dprm);
    else if (vb == 4) k_fb_fill<4><<<g.cv_blocks, kThreads, 0, st>>>(table, nsys, dprm);
    else k_fb_fill<2><<<g.cv_blocks, kThreads, 0, st>>>(table, nsys, dprm);
    const int npairs = static_cast<int>(L.npairs);
    auto* pt0 = reinterpret_cast<int32_t*>(ws + L.pair_t0);
    auto* nt = reinterpret_cast<int32_t*>(ws + L.ntiles);
    k_band_pairs<<<1, kTileThreads, 0, st>>>(table, nsys, npairs, c.bq, pt0, nt);
    const unsigned tb = static_cast<unsigned>((L.tile_cap + 255) / 256);
    k_band_tile_fill<<<tb, 256, 0, st>>>(table, nsys, npairs, c.bq, pt0, nt, reinterpret_cast<BandTile*>(ws + L.tiles));
  }
  if (c.stg & 2) {
    int64_t words = 1;
    for (int s = 0; s < nsys; ++s) words = std::max<int64_t>(words, (sys[s].m + 31) / 32);
    k_bt_plan<<<g.bp_blocks, kStagedThreads, static_cast<size_t>(3 * words * sizeof(uint32_t)), st>>>(table, nsys,
                                                                                                     dprm);
  }
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

// Writes the descriptor table and resets states (stream-ordered kernels);
// writes the interleaved stream copies where a kernel reads them, and the
// staged forms.
ss_status setup(const ss_system* sys, int nsys, float* const* f, double* const* res_hist,
                Params prm, const Cfg& c, const Layout& L, char* ws, Grids* g,
                int zero_start, hipStream_t st) {
  int64_t fb = 0, bb = 0, cv = 0, t64 = 0, t32 = 0;
  int32_t pairs = 0;
  prm.band_lg = c.blg;
  prm.tile_lg = c.tlg;
  prm.band_q = c.bq;
  for (int k = 0; k < 3; ++k) prm.b2s[k] = L.b2s[k] ? reinterpret_cast<const int32_t*>(ws + L.b2s[k]) : nullptr;
  const int64_t rpb = (c.stg & 1) ? kFinThreads : static_cast<int64_t>(c.rpw) * kWPB;
  const int64_t cpb = (c.stg & 2) ? (int64_t{1} << c.tlg) : static_cast<int64_t>(c.cpw) * kWPB;
  DescChunk ch{};
  SysDesc* table = reinterpret_cast<SysDesc*>(ws + L.table);
  Params* dprm = reinterpret_cast<Params*>(ws + L.params);
  for (int s = 0; s < nsys; ++s) {
    const ss_system& S = sys[s];
    SysDesc d{};
    d.row_ptr = S.row_ptr;
    d.col_idx = S.col_idx;
    d.val = S.val;
    d.col_ptr = S.col_ptr;
    d.row_idx = S.row_idx;
    d.val_t = S.val_t;
    d.p = S.p;
    d.inv_row = S.inv_row;
    d.inv_col = S.inv_col;
    d.f[0] = f[s];
    d.f[1] = reinterpret_cast<float*>(ws + L.f_off[s]);
    d.z = reinterpret_cast<float*>(ws + L.z_off[s]);
    d.res_hist = res_hist ? res_hist[s] : nullptr;
    d.partials = reinterpret_cast<double*>(ws + L.part_off[s]);
    d.st = reinterpret_cast<SysState*>(ws + L.states) + s;
    d.m = S.m;
    d.n = S.n;
    d.fp_nblocks = static_cast<int32_t>((S.m + rpb - 1) / rpb);
    d.bp_nblocks = static_cast<int32_t>((S.n + cpb - 1) / cpb);
    d.fp_block0 = fb;
    d.bp_block0 = bb;
    if (S.nnz > 0 && fp_form(c.ch) == 2 && !S.row_lanes && !(c.stg & 1)) {
      d.col_idx = reinterpret_cast<int32_t*>(ws + L.fi_idx[s]);
      d.val = ws + L.fi_val[s];
      if (ss_status e = interleave_lines(S.row_ptr, S.m, S.col_idx, S.val, const_cast<int32_t*>(d.col_idx),
                                         const_cast<void*>(d.val), value_bytes(S), kWave / c.rpw, st))
        return e;
    }
    if (S.nnz > 0 && bp_form(c.ch) == 2 && !S.col_lanes && !(c.stg & 2)) {
      d.row_idx = reinterpret_cast<int32_t*>(ws + L.bi_idx[s]);
      d.val_t = ws + L.bi_val[s];
      if (ss_status e = interleave_lines(S.col_ptr, S.n, S.row_idx, S.val_t, const_cast<int32_t*>(d.row_idx),
                                         const_cast<void*>(d.val_t), value_bytes(S), kWave / c.cpw, st))
        return e;
    }
    if (c.stg & 1) {
      d.fb_idx = reinterpret_cast<uint16_t*>(ws + L.fb_idx[s]);
      d.fb_val = ws + L.fb_val[s];
      d.fb_off = reinterpret_cast<int32_t*>(ws + L.fb_off[s]);
      d.fb_bits = reinterpret_cast<uint32_t*>(ws + L.fb_bits[s]);
      d.fb_slot = reinterpret_cast<int32_t*>(ws + L.fb_slot[s]);
      d.fb_rseg = reinterpret_cast<uint32_t*>(ws + L.fb_rseg[s]);
      d.fb_part = reinterpret_cast<float*>(ws + L.fb_part[s]);
      d.fb_len = reinterpret_cast<uint64_t*>(ws + L.fb_len[s]);
      d.fb_nb = static_cast<int32_t>(bands_of(S, c.blg));
      d.fb_pair0 = pairs;
      d.cv_rblk0 = cv;
      d.cv_t64_0 = t64;
      d.cv_t32_0 = t32;
      pairs += d.fb_nb;
      cv += (S.m + kCvRows - 1) / kCvRows;
      t64 += pscan_tiles(static_cast<int64_t>(d.fb_nb) * S.m + 1);
      t32 += pscan_tiles(S.m + 1);
    }
    if (c.stg & 2) {
      d.bt_idx = reinterpret_cast<uint16_t*>(ws + L.bt_idx[s]);
      d.bt_meta = reinterpret_cast<BtMeta*>(ws + L.bt_meta[s]);
      d.bt_runs = reinterpret_cast<int32_t*>(ws + L.bt_runs[s]);
    }
    fb += d.fp_nblocks;
    bb += d.bp_nblocks;
    ch.d[ch.count++] = d;
    if (ch.count == kDescChunk || s == nsys - 1) {
      k_put_desc<<<1, kWave, 0, st>>>(ch, table, prm, dprm);
      ch.first = s + 1;
      ch.count = 0;
    }
  }
  const SetupFlags fl{zero_start};
  if (c.nv == 2) k_setup<2><<<static_cast<unsigned>(nsys), kWave * kSetupWaves, 0, st>>>(table, fl);
  else k_setup<1><<<static_cast<unsigned>(nsys), kWave * kSetupWaves, 0, st>>>(table, fl);
  if (fb > UINT32_MAX || bb > UINT32_MAX || cv > UINT32_MAX) return fail(SS_E_ARG, "SART: grid too large");
  if (L.b2s[0] || L.b2s[1] || L.b2s[2])
    k_fill_b2s<<<static_cast<unsigned>(nsys), 256, 0, st>>>(
        table, L.b2s[0] ? reinterpret_cast<int32_t*>(ws + L.b2s[0]) : nullptr,
        L.b2s[1] ? reinterpret_cast<int32_t*>(ws + L.b2s[1]) : nullptr,
        L.b2s[2] ? reinterpret_cast<int32_t*>(ws + L.b2s[2]) : nullptr, kCvRows);
  g->fp_blocks = static_cast<uint32_t>(fb);
  g->bp_blocks = static_cast<uint32_t>(bb);
  g->cv_blocks = static_cast<uint32_t>(cv);
  g->band_blocks = (c.stg & 1) ? band_grid(c, L) : 0;
  SS_HIP_TRY(hipGetLastError());
  if (c.stg) return build_staged(sys, nsys, c, L, ws, *g, st);
  return SS_OK;
}

// Launches go through hipExtLaunchKernelGGL so that, when timing, the start
// and stop events are stamped by the kernel's own dispatch (no marker
// packets between kernels); with null events it is an ordinary launch.
struct Stamp {
  hipEvent_t start = nullptr, stop = nullptr;
  // a forward projection of two launches (band-staged): the first one's
  // stop and the second one's start
  hipEvent_t mid0 = nullptr, mid1 = nullptr;
};

// Grid for a grid-stride kernel: one block per tile, unless `persistent`
// and there are more tiles than resident blocks: then the resident capacity
// rounded down to a multiple of 8 (so tile t always runs on XCD t mod 8).
uint32_t grid_for(const void* kern, uint32_t ntiles, int persistent) {
  if (!persistent) return ntiles;
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, uint32_t> cap;
  int dev = 0;
  (void)hipGetDevice(&dev);
  uint32_t resident;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cap.find({kern, dev});
    if (it == cap.end()) {
      int cus = 0, per = 0;
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kThreads, 0);
      const uint32_t r = static_cast<uint32_t>(std::max(1, cus) * std::max(1, per));
      it = cap.emplace(std::make_pair(kern, dev), std::max<uint32_t>(8, r & ~7u)).first;
    }
    resident = it->second;
  }
  return ntiles <= resident ? ntiles : resident;
}

template <typename K, typename... Args>
void go(K kern, uint32_t ntiles, int persistent, hipStream_t st, Stamp e, Args... args) {
  const uint32_t grid = grid_for(reinterpret_cast<const void*>(kern), ntiles, persistent);
  hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, st, e.start, e.stop, 0, args...);
}

template <int NV, int WT, int U, int SF>
void launch_fp_u(int rpw, int pers, const SysDesc* t, int nsys, uint32_t nb, int xcd, int par, hipStream_t st,
                 Stamp e) {
  switch (rpw) {
    case 1: go(k_sart_fp<NV, WT, 1, U, SF>, nb, pers, st, e, t, nsys, nb, xcd, par); break;
    case 2: go(k_sart_fp<NV, WT, 2, U, SF>, nb, pers, st, e, t, nsys, nb, xcd, par); break;
    case 4: go(k_sart_fp<NV, WT, 4, U, SF>, nb, pers, st, e, t, nsys, nb, xcd, par); break;
    default: go(k_sart_fp<NV, WT, 8, U, SF>, nb, pers, st, e, t, nsys, nb, xcd, par); break;
  }
}

template <int NV, int WT, int U, int SF>
void launch_bp_u(int cpw, int pers, const Params* prm, const SysDesc* t, int nsys, uint32_t nb, int xcd, int par,
                 hipStream_t st, Stamp e) {
  switch (cpw) {
    case 1: go(k_sart_bp<NV, WT, 1, U, SF>, nb, pers, st, e, prm, t, nsys, nb, xcd, par); break;
    case 2: go(k_sart_bp<NV, WT, 2, U, SF>, nb, pers, st, e, prm, t, nsys, nb, xcd, par); break;
    case 4: go(k_sart_bp<NV, WT, 4, U, SF>, nb, pers, st, e, prm, t, nsys, nb, xcd, par); break;
    case 8: go(k_sart_bp<NV, WT, 8, U, SF>, nb, pers, st, e, prm, t, nsys, nb, xcd, par); break;
    default: go(k_sart_bp<NV, WT, 16, U, SF>, nb, pers, st, e, prm, t, nsys, nb, xcd, par); break;
  }
}

// Staged kernels: the forward pair (band kernel, then the residual kernel)
// and the tile-staged back projection.  The band kernel loads batches of one
// window per wavefront (unroll 4) or two (unroll 8); the back projection
// takes two chunks per lane and pass when a lane group is 8 lanes or fewer
// (8 or more columns per wavefront: a pass then still covers a column of 64
// entries), else one.
template <int NV, int WT, int P>
void launch_band(const Cfg& c, const char* ws, const Layout& L, int nsys, const Grids& g, int par, hipStream_t st,
                 Stamp e) {
  const Params* prm = reinterpret_cast<const Params*>(ws + L.params);
  const SysDesc* t = reinterpret_cast<const SysDesc*>(ws + L.table);
  const BandTile* tiles = reinterpret_cast<const BandTile*>(ws + L.tiles);
  const int32_t* nt = reinterpret_cast<const int32_t*>(ws + L.ntiles);
  const size_t lds = band_lds_bytes(NV, c.blg);
  hipExtLaunchKernelGGL(k_band_fp<NV, WT, P>, dim3(g.band_blocks), dim3(kWave * kBandWaves), lds, st, e.start,
                        e.mid0, 0, t, tiles, nt, prm, par);
  hipExtLaunchKernelGGL(k_band_fin<NV>, dim3(g.fp_blocks), dim3(kWave), 0, st, e.mid1, e.stop, 0, t, nsys, prm);
}

template <int NV, int WT, int P>
void launch_tile_bp(const Cfg& c, const char* ws, const Layout& L, int nsys, const Grids& g, int par, hipStream_t st,
                    Stamp e) {
  const Params* prm = reinterpret_cast<const Params*>(ws + L.params);
  const SysDesc* t = reinterpret_cast<const SysDesc*>(ws + L.table);
  const size_t lds = sizeof(float) * NV * kBtMaxRows;
  const dim3 grid(g.bp_blocks), blk(kStagedThreads);
  switch (c.cpw) {
    case 4: hipExtLaunchKernelGGL(k_tile_bp<NV, WT, 4, P>, grid, blk, lds, st, e.start, e.stop, 0, prm, t, nsys, par); break;
    case 16: hipExtLaunchKernelGGL(k_tile_bp<NV, WT, 16, P>, grid, blk, lds, st, e.start, e.stop, 0, prm, t, nsys, par); break;
    default: hipExtLaunchKernelGGL(k_tile_bp<NV, WT, 8, P>, grid, blk, lds, st, e.start, e.stop, 0, prm, t, nsys, par); break;
  }
}

template <bool BP>
void launch_kernel(const Cfg& c, const char* ws, const Layout& L, int nsys, const Grids& g, int par,
                   hipStream_t st, Stamp e = {}) {
  if ((c.stg & (BP ? 2 : 1)) != 0) {
#define SS_STAGED(NV, WT)                                                                            \
  if (c.nv == NV && c.wt == WT) {                                                                    \
    if (BP) {                                                                                        \
      if (c.cpw >= 8) launch_tile_bp<NV, WT, 2>(c, ws, L, nsys, g, par, st, e);                      \
      else launch_tile_bp<NV, WT, 1>(c, ws, L, nsys, g, par, st, e);                                 \
    } else {                                                                                         \
      if (c.u == 8) launch_band<NV, WT, 2>(c, ws, L, nsys, g, par, st, e);                           \
      else launch_band<NV, WT, 1>(c, ws, L, nsys, g, par, st, e);                                    \
    }                                                                                                \
    return;                                                                                          \
  }
    SS_STAGED(2, SS_F32)
    SS_STAGED(2, SS_BF16)
    SS_STAGED(2, SS_F16)
    SS_STAGED(1, SS_F32)
    SS_STAGED(1, SS_BF16)
    SS_STAGED(1, SS_F16)
#undef SS_STAGED
    return;
  }
  const Params* prm = reinterpret_cast<const Params*>(ws + L.params);
  const SysDesc* t = reinterpret_cast<const SysDesc*>(ws + L.table);
// single 16-bit values are rejected for the interleaved form by validate()
#define SF2(NV, WT) ((NV) == 2 || (WT) == SS_F32 ? 2 : 0)
#define SS_DISPATCH(NV, WT, U)                                                                      \
  if (c.nv == NV && c.wt == WT && c.u == U) {                                                       \
    if (BP) {                                                                                       \
      const int sf = bp_form(c.ch);                                                                 \
      if (sf == 2) launch_bp_u<NV, WT, U, SF2(NV, WT)>(c.cpw, c.pers, prm, t, nsys, g.bp_blocks, c.xcd, par, st, e); \
      else if (sf == 1) launch_bp_u<NV, WT, U, 1>(c.cpw, c.pers, prm, t, nsys, g.bp_blocks, c.xcd, par, st, e); \
      else launch_bp_u<NV, WT, U, 0>(c.cpw, c.pers, prm, t, nsys, g.bp_blocks, c.xcd, par, st, e);      \
    } else {                                                                                        \
      const int sf = fp_form(c.ch);                                                                 \
      if (sf == 2) launch_fp_u<NV, WT, U, SF2(NV, WT)>(c.rpw, c.pers, t, nsys, g.fp_blocks, c.xcd, par, st, e); \
      else if (sf == 1) launch_fp_u<NV, WT, U, 1>(c.rpw, c.pers, t, nsys, g.fp_blocks, c.xcd, par, st, e); \
      else launch_fp_u<NV, WT, U, 0>(c.rpw, c.pers, t, nsys, g.fp_blocks, c.xcd, par, st, e);       \
    }                                                                                               \
    return;                                                                                         \
  }
  SS_DISPATCH(2, SS_F32, 4)
  SS_DISPATCH(2, SS_BF16, 4)
  SS_DISPATCH(2, SS_F16, 4)
  SS_DISPATCH(1, SS_F32, 4)
  SS_DISPATCH(1, SS_BF16, 4)
  SS_DISPATCH(1, SS_F16, 4)
  SS_DISPATCH(2, SS_F32, 8)
  SS_DISPATCH(2, SS_BF16, 8)
  SS_DISPATCH(2, SS_F16, 8)
  SS_DISPATCH(1, SS_F32, 8)
  SS_DISPATCH(1, SS_BF16, 8)
  SS_DISPATCH(1, SS_F16, 8)
#undef SS_DISPATCH
#undef SF2
}

// `count` iterations; iteration i reads buffer (first + i) mod 2.
void launch_iterations(const Cfg& c, const char* ws, const Layout& L, int nsys, const Grids& g, int64_t first,
                       int count, hipStream_t st) {
  for (int i = 0; i < count; ++i) {
    const int par = static_cast<int>((first + i) & 1);
    launch_kernel<false>(c, ws, L, nsys, g, par, st);
    launch_kernel<true>(c, ws, L, nsys, g, par, st);
  }
}

void launch_finish(const Cfg& c, const char* ws, const Layout& L, int nsys, hipStream_t st) {
  const SysDesc* t = reinterpret_cast<const SysDesc*>(ws + L.table);
  if (c.nv == 2) k_finish<2><<<nsys, kThreads, 0, st>>>(t);
  else k_finish<1><<<nsys, kThreads, 0, st>>>(t);
}

// ----------------------------------------------------------- graph cache
struct GraphKey {
  int device;
  const void* ws;
  int nsys;
  uint32_t fpb, bpb;
  int nv, wt, rpw, cpw, xcd, u, pers, ch, count;
  int stg, blg, tlg, bq;
  uint32_t bandb;
  bool operator<(const GraphKey& o) const {
    return std::tie(device, ws, nsys, fpb, bpb, nv, wt, rpw, cpw, xcd, u, pers, ch, count, stg, blg, tlg, bq, bandb) <
           std::tie(o.device, o.ws, o.nsys, o.fpb, o.bpb, o.nv, o.wt, o.rpw, o.cpw, o.xcd, o.u, o.pers, o.ch,
                    o.count, o.stg, o.blg, o.tlg, o.bq, o.bandb);
  }
};

GraphCache<GraphKey>& graph_cache() {
  static auto* c = new GraphCache<GraphKey>(32);  // lives until process exit
  return *c;
}

ss_status read_states(const char* ws, const Layout& L, int nsys, std::vector<SysState>* h, hipStream_t st) {
  h->resize(nsys);
  SS_HIP_TRY(hipMemcpyAsync(h->data(), ws + L.states, sizeof(SysState) * nsys, hipMemcpyDeviceToHost, st));
  SS_HIP_TRY(hipStreamSynchronize(st));
  return SS_OK;
}

}  // namespace
}  // namespace ss

using namespace ss;

extern "C" ss_status ss_sart_workspace_bytes(const ss_system* sys, int32_t nsys, const ss_sart_opts* opts,
                                             size_t* bytes) {
  clear_error();
  if (!bytes) return fail(SS_E_ARG, "ss_sart_workspace_bytes: NULL bytes");
  if (ss_status s = validate(sys, nsys, opts, "ss_sart_workspace_bytes")) return s;
  *bytes = make_layout(sys, nsys, opts).total;
  return SS_OK;
}

extern "C" ss_status ss_sart_solve(const ss_system* sys, int32_t nsys, float* const* f, double* const* res_hist,
                                   const ss_sart_opts* opts, int32_t* iters, void* workspace,
                                   size_t workspace_bytes, void* stream) {
  clear_error();
  if (ss_status s = validate(sys, nsys, opts, "ss_sart_solve")) return s;
  if (!f || !workspace) return fail(SS_E_ARG, "ss_sart_solve: NULL images or workspace");
  for (int s = 0; s < nsys; ++s)
    if (!f[s] || (res_hist && !res_hist[s])) return fail(SS_E_ARG, "ss_sart_solve: NULL image %d", s);
  if (ss_status s = check_images(sys, nsys, f, opts, "ss_sart_solve")) return s;
  const Layout L = make_layout(sys, nsys, opts);
  if (workspace_bytes < L.total) return fail(SS_E_WORKSPACE, "ss_sart_solve: workspace needs %zu bytes", L.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const Cfg c = choose_cfg(sys, nsys, opts);
  Params prm{opts->lambda, opts->max_iter, opts->tol, opts->nonneg};
  Grids g{};
  if (ss_status s = setup(sys, nsys, f, res_hist, prm, c, L, ws, &g, opts->zero_start, st)) return s;
  const int64_t total = static_cast<int64_t>(opts->max_iter) + 1;  // forward passes incl. the final residual
  // an even chunk keeps the buffer parity of every replay aligned
  int chunk = opts->tol > 0.0 ? static_cast<int>(std::min<int64_t>(opts->check_every, total))
                              : static_cast<int>(std::min<int64_t>(total, 256));
  chunk += chunk & 1;
  GraphEntry* graph = nullptr;
  if (opts->use_graph) {
    int dev = 0;
    SS_HIP_TRY(hipGetDevice(&dev));
    const GraphKey key{dev, workspace, nsys, g.fp_blocks, g.bp_blocks, c.nv, c.wt, c.rpw, c.cpw, c.xcd, c.u, c.pers, c.ch,
                       chunk, c.stg, c.blg, c.tlg, c.bq, g.band_blocks};
    auto capture = [&](hipStream_t cs) { launch_iterations(c, ws, L, nsys, g, 0, chunk, cs); };
    if (ss_status s = graph_cache().acquire(key, dev, capture, &graph)) return s;
  }
  std::vector<SysState> hs;
  ss_status loop = SS_OK;
  for (int64_t done = 0; done < total && loop == SS_OK; done += chunk) {
    if (graph) {
      const hipError_t e = hipGraphLaunch(graph->exec, st);
      if (e != hipSuccess) loop = fail(SS_E_HIP, "hipGraphLaunch failed: %s", hipGetErrorString(e));
    } else {
      launch_iterations(c, ws, L, nsys, g, done, static_cast<int>(std::min<int64_t>(chunk, total - done)), st);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) loop = fail(SS_E_HIP, "SART launch failed: %s", hipGetErrorString(e));
    }
    if (loop == SS_OK && opts->tol > 0.0 && done + chunk < total) {
      loop = read_states(ws, L, nsys, &hs, st);
      bool all = true;
      for (const auto& x : hs) all = all && x.stop;
      if (loop == SS_OK && all) break;
    }
  }
  if (graph) graph_cache().release(graph, st);
  if (loop != SS_OK) return loop;
  launch_finish(c, ws, L, nsys, st);
  SS_HIP_TRY(hipGetLastError());
  if (!iters && opts->tol <= 0.0) return SS_OK;
  if (ss_status s = read_states(ws, L, nsys, &hs, st)) return s;
  ss_status result = SS_OK;
  for (int s = 0; s < nsys; ++s) {
    if (iters) iters[s] = hs[s].k;
    if (opts->tol > 0.0 && !(hs[s].last_res <= opts->tol)) result = SS_NOT_CONVERGED;
  }
  return result;
}

extern "C" ss_status ss_sart_time_phases(const ss_system* sys, int32_t nsys, float* const* f,
                                         const ss_sart_opts* opts, int32_t reps, double* ms, void* workspace,
                                         size_t workspace_bytes, void* stream) {
  clear_error();
  if (ss_status s = validate(sys, nsys, opts, "ss_sart_time_phases")) return s;
  if (!f || !workspace || !ms || reps <= 0) return fail(SS_E_ARG, "ss_sart_time_phases: bad argument");
  if (ss_status s = check_images(sys, nsys, f, opts, "ss_sart_time_phases")) return s;
  const Layout L = make_layout(sys, nsys, opts);
  if (workspace_bytes < L.total) return fail(SS_E_WORKSPACE, "ss_sart_time_phases: workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const Cfg c = choose_cfg(sys, nsys, opts);
  Params prm{opts->lambda, (1 << 30), -1.0, opts->nonneg};
  Grids g{};
  if (ss_status s = setup(sys, nsys, f, nullptr, prm, c, L, ws, &g, 0, st)) return s;
  const bool two = (c.stg & 1) != 0;
  std::vector<hipEvent_t> ev(6 * static_cast<size_t>(reps));
  for (auto& e : ev) SS_HIP_TRY(hipEventCreate(&e));
  launch_kernel<false>(c, ws, L, nsys, g, 0, st);  // warm caches and code
  launch_kernel<true>(c, ws, L, nsys, g, 0, st);
  for (int r = 0; r < reps; ++r) {
    const int par = (r + 1) & 1;
    hipEvent_t* e = &ev[6 * static_cast<size_t>(r)];
    launch_kernel<false>(c, ws, L, nsys, g, par, st, two ? Stamp{e[0], e[3], e[1], e[2]} : Stamp{e[0], e[1]});
    launch_kernel<true>(c, ws, L, nsys, g, par, st, Stamp{e[4], e[5]});
  }
  (void)hipEventSynchronize(ev.back());
  double t[3] = {0.0, 0.0, 0.0};
  for (int r = 0; r < reps; ++r) {
    hipEvent_t* e = &ev[6 * static_cast<size_t>(r)];
    float a = 0.f, b = 0.f, cc = 0.f;
    (void)hipEventElapsedTime(&a, e[0], e[1]);
    if (two) (void)hipEventElapsedTime(&b, e[2], e[3]);
    (void)hipEventElapsedTime(&cc, e[4], e[5]);
    t[0] += a;
    t[1] += b;
    t[2] += cc;
  }
  const hipError_t err = hipGetLastError();
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (err != hipSuccess) return fail(SS_E_HIP, "ss_sart_time_phases: %s", hipGetErrorString(err));
  for (int k = 0; k < 3; ++k) ms[k] = t[k] / reps;
  return SS_OK;
}

extern "C" ss_status ss_sart_staged_info(const ss_system* sys, int32_t nsys, float* const* f,
                                         const ss_sart_opts* opts, int64_t* info, void* workspace,
                                         size_t workspace_bytes, void* stream) {
  clear_error();
  if (ss_status s = validate(sys, nsys, opts, "ss_sart_staged_info")) return s;
  if (!info || !workspace || !opts->staged) return fail(SS_E_ARG, "ss_sart_staged_info: bad argument");
  if (ss_status s = check_images(sys, nsys, f, opts, "ss_sart_staged_info")) return s;
  const Layout L = make_layout(sys, nsys, opts);
  if (workspace_bytes < L.total) return fail(SS_E_WORKSPACE, "ss_sart_staged_info: workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const Cfg c = choose_cfg(sys, nsys, opts);
  Params prm{opts->lambda, 0, -1.0, opts->nonneg};
  Grids g{};
  if (ss_status s = setup(sys, nsys, f, nullptr, prm, c, L, ws, &g, 0, st)) return s;
  int64_t* dinfo = reinterpret_cast<int64_t*>(ws + L.info);
  k_staged_info<<<1, 64, 0, st>>>(reinterpret_cast<const SysDesc*>(ws + L.table), nsys, c.stg,
                                  reinterpret_cast<const int32_t*>(ws + L.ntiles), dinfo);
  SS_HIP_TRY(hipGetLastError());
  SS_HIP_TRY(hipMemcpyAsync(info, dinfo, 5 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SS_HIP_TRY(hipStreamSynchronize(st));
  return SS_OK;
}

extern "C" ss_status ss_sart_time_kernels(const ss_system* sys, int32_t nsys, float* const* f,
                                          const ss_sart_opts* opts, int32_t reps, double* fp_ms, double* bp_ms,
                                          void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (ss_status s = validate(sys, nsys, opts, "ss_sart_time_kernels")) return s;
  if (!f || !workspace || !fp_ms || !bp_ms || reps <= 0)
    return fail(SS_E_ARG, "ss_sart_time_kernels: bad argument");
  if (ss_status s = check_images(sys, nsys, f, opts, "ss_sart_time_kernels")) return s;
  const Layout L = make_layout(sys, nsys, opts);
  if (workspace_bytes < L.total) return fail(SS_E_WORKSPACE, "ss_sart_time_kernels: workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const Cfg c = choose_cfg(sys, nsys, opts);
  Params prm{opts->lambda, (1 << 30), -1.0, opts->nonneg};
  Grids g{};
  if (ss_status s = setup(sys, nsys, f, nullptr, prm, c, L, ws, &g, 0, st)) return s;
  // the kernels are timed where they run in a solve, forward and back
  // projection alternating; each launch carries its own start/stop events
  std::vector<hipEvent_t> ev(4 * static_cast<size_t>(reps));
  for (auto& e : ev) SS_HIP_TRY(hipEventCreate(&e));
  launch_kernel<false>(c, ws, L, nsys, g, 0, st);  // warm caches and code
  launch_kernel<true>(c, ws, L, nsys, g, 0, st);
  for (int r = 0; r < reps; ++r) {
    const int par = (r + 1) & 1;
    launch_kernel<false>(c, ws, L, nsys, g, par, st, Stamp{ev[4 * r], ev[4 * r + 1]});
    launch_kernel<true>(c, ws, L, nsys, g, par, st, Stamp{ev[4 * r + 2], ev[4 * r + 3]});
  }
  (void)hipEventSynchronize(ev.back());
  double t_fp = 0.0, t_bp = 0.0;
  for (int r = 0; r < reps; ++r) {
    float a = 0.f, b = 0.f;
    (void)hipEventElapsedTime(&a, ev[4 * r], ev[4 * r + 1]);
    (void)hipEventElapsedTime(&b, ev[4 * r + 2], ev[4 * r + 3]);
    t_fp += a;
    t_bp += b;
  }
  const hipError_t err = hipGetLastError();
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (err != hipSuccess) return fail(SS_E_HIP, "ss_sart_time_kernels: %s", hipGetErrorString(err));
  *fp_ms = t_fp / reps;
  *bp_ms = t_bp / reps;
  return SS_OK;
}

namespace {
// Time of the per-solve copies of the interleaved form, rows and columns
// (setup with the copies minus setup without them; best of 3).
ss_status time_copies(const ss_system* sys, int nsys, float* const* f, const ss_sart_opts* opts, void* workspace,
                      size_t workspace_bytes, hipStream_t st, double* rows_ms, double* cols_ms) {
  hipEvent_t e0, e1;
  SS_HIP_TRY(hipEventCreate(&e0));
  SS_HIP_TRY(hipEventCreate(&e1));
  double best[3] = {1e30, 1e30, 1e30};
  const int forms[3] = {0, 4, 8};
  ss_status result = SS_OK;
  for (int r = 0; r < 3 && result == SS_OK; ++r) {
    for (int k = 0; k < 3 && result == SS_OK; ++k) {
      ss_sart_opts o = *opts;
      o.chunked = forms[k];
      const Layout L = make_layout(sys, nsys, &o);
      if (L.total > workspace_bytes) {
        result = fail(SS_E_WORKSPACE, "ss_sart_autotune: workspace too small");
        break;
      }
      const Cfg c = choose_cfg(sys, nsys, &o);
      const Params prm{o.lambda, 1, -1.0, o.nonneg};
      Grids g{};
      (void)hipEventRecord(e0, st);
      result = setup(sys, nsys, f, nullptr, prm, c, L, static_cast<char*>(workspace), &g, 0, st);
      (void)hipEventRecord(e1, st);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      best[k] = std::min(best[k], static_cast<double>(ms));
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *rows_ms = std::max(0.0, best[1] - best[0]);
  *cols_ms = std::max(0.0, best[2] - best[0]);
  return result;
}

struct TuneKey {
  int nv, wt, nsys, row_lanes, col_lanes;
  int64_t m_bucket, row_bucket, col_bucket;
  bool operator<(const TuneKey& o) const {
    return std::tie(nv, wt, nsys, row_lanes, col_lanes, m_bucket, row_bucket, col_bucket) <
           std::tie(o.nv, o.wt, o.nsys, o.row_lanes, o.col_lanes, o.m_bucket, o.row_bucket, o.col_bucket);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::tuple<int, int, int, int, int, int>> g_tune;
}  // namespace

extern "C" ss_status ss_sart_autotune(const ss_system* sys, int32_t nsys, float* const* f, ss_sart_opts* opts,
                                      void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (ss_status s = validate(sys, nsys, opts, "ss_sart_autotune")) return s;
  double nnz = 0, m = 0, n = 0;
  for (int s = 0; s < nsys; ++s) {
    nnz += static_cast<double>(sys[s].nnz);
    m += static_cast<double>(sys[s].m);
    n += static_cast<double>(sys[s].n);
  }
  const TuneKey key{sys[0].nvals, sys[0].wdtype, nsys, sys[0].row_lanes, sys[0].col_lanes, static_cast<int64_t>(std::log2(m)),
                    static_cast<int64_t>(std::log2(1.0 + nnz / m) * 4), static_cast<int64_t>(std::log2(1.0 + nnz / n) * 4)};
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      std::tie(opts->rows_per_wave, opts->cols_per_wave, opts->xcd_remap, opts->unroll, opts->persistent,
               opts->chunked) = it->second;
      return SS_OK;
    }
  }
  // every candidate is timed in the alternating forward/back sequence; a
  // candidate replaces the statistics-based default only when it is more
  // than 3 % faster, so that timing noise does not flip the choice
  const int reps = 20;
  const Cfg dflt = choose_cfg(sys, nsys, opts);
  struct Best {
    double t = 1e30;
    int pw = 1, u = 4, xcd = 0, pers = 0, ch = 0;
  } bf, bb, df, db;
  Best bestf[2][2][2], bestb[2][2][2];  // per (persistent, xcd_remap, unroll == 8)
  // stream forms: entry-wise, chunked, and interleaved where the workspace
  // holds the interleaved copies
  std::vector<int> forms{0, 3};
  double copy_rows = 0.0, copy_cols = 0.0;
  const int fixed_rows = sys[0].row_lanes ? kWave / sys[0].row_lanes : 0;
  const int fixed_cols = sys[0].col_lanes ? kWave / sys[0].col_lanes : 0;
  if (fixed_rows && fixed_cols) {
    forms = {0};  // both kernels read the stored order in place
  } else {
    ss_sart_opts o = *opts;
    o.chunked = 12;
    if (validate(sys, nsys, &o, "ss_sart_autotune") == SS_OK && make_layout(sys, nsys, &o).total <= workspace_bytes) {
      forms.push_back(12);
      // the copies are made once per solve: spread over its iterations
      if (ss_status s = time_copies(sys, nsys, f, opts, workspace, workspace_bytes, static_cast<hipStream_t>(stream),
                                    &copy_rows, &copy_cols))
        return s;
      const double iters = std::max(1, opts->max_iter);
      copy_rows /= iters;
      copy_cols /= iters;
    }
    clear_error();
  }
  for (int pers = 0; pers <= 1; ++pers) {
    for (int xcd = 0; xcd <= 1; ++xcd) {
      for (int u = 4; u <= 8; u += 4) {
        for (int ch : forms) {
          for (int pw = 1; pw <= 16; pw <<= 1) {
            ss_sart_opts o = *opts;
            o.persistent = pers;
            o.xcd_remap = xcd;
            o.unroll = u;
            o.chunked = ch;
            if (fixed_rows && fixed_cols && pw > 1) continue;
            o.rows_per_wave = fixed_rows ? fixed_rows : (pw <= 8 ? pw : 8);
            o.cols_per_wave = fixed_cols ? fixed_cols : pw;
            double tf = 0, tb = 0;
            if (ss_status s = ss_sart_time_kernels(sys, nsys, f, &o, reps, &tf, &tb, workspace, workspace_bytes,
                                                   stream))
              return s;
            if (fp_form(ch) == 2) tf += copy_rows;
            if (bp_form(ch) == 2) tb += copy_cols;
            const bool base = xcd == dflt.xcd && u == dflt.u && pers == dflt.pers;
            if (base && fp_form(ch) == fp_form(dflt.ch) && o.rows_per_wave == dflt.rpw && tf < df.t)
              df = {tf, dflt.rpw, u, xcd, pers, ch};
            if (base && bp_form(ch) == bp_form(dflt.ch) && o.cols_per_wave == dflt.cpw && tb < db.t)
              db = {tb, dflt.cpw, u, xcd, pers, ch};
            Best& cf = bestf[pers][xcd][u / 8];
            Best& cb = bestb[pers][xcd][u / 8];
            if (pw <= 8 && tf < cf.t) cf = {tf, o.rows_per_wave, u, xcd, pers, ch};
            if (tb < cb.t) cb = {tb, o.cols_per_wave, u, xcd, pers, ch};
          }
        }
      }
    }
  }
  // one remap flag, unroll depth and grid mode serve both kernels: the
  // combination with the least forward + back time, each kernel with its
  // own lanes per line and stream form under it; the default is kept unless
  // that is more than 3 % faster
  for (int pers = 0; pers <= 1; ++pers)
    for (int xcd = 0; xcd <= 1; ++xcd)
      for (int u8 = 0; u8 <= 1; ++u8)
        if (bestf[pers][xcd][u8].t + bestb[pers][xcd][u8].t < bf.t + bb.t) {
          bf = bestf[pers][xcd][u8];
          bb = bestb[pers][xcd][u8];
        }
  if (df.t + db.t <= 1.03 * (bf.t + bb.t)) {
    bf = df;
    bb = db;
  }
  opts->rows_per_wave = bf.pw;
  opts->cols_per_wave = bb.pw;
  opts->xcd_remap = bf.xcd;
  opts->unroll = bf.u;
  opts->persistent = bf.pers;
  opts->chunked = (bf.ch & 5) | (bb.ch & 10);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[key] = std::make_tuple(opts->rows_per_wave, opts->cols_per_wave, opts->xcd_remap, opts->unroll,
                                opts->persistent, opts->chunked);
  return SS_OK;
}
