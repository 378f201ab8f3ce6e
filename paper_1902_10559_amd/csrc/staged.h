// Staged solver kernels: the SART products with the gathered vector held in
// shared memory (LDS) instead of being gathered from L2 entry by entry.
//
// Forward projection, band-staged.  The columns (voxels) are cut into bands
// of W consecutive indices; with the vertical-snake numbering a band is a
// run of whole voxel columns of the slice, a compact region of the image.
// Each row's entries in one band form a segment (the columns of a row
// ascend, so a segment is a contiguous part of the row).  A copy of the row
// streams is laid out band-major: band 0's segments (rows ascending), then
// band 1's, ..., with 16-bit column indices relative to the band's start,
// and every segment padded with zero entries to whole chunks of SS_CHUNK
// entries, so that no chunk holds two segments; a bitmap marks the chunks
// that start a segment.  A band's chunks are cut into work tiles of about
// the same number of chunks (whole segments each).  The tiles are dealt to
// the blocks in contiguous runs; a block loads the band of the image into
// LDS when its band changes, and each tile is streamed flat by one
// wavefront, one chunk per lane and 64 consecutive chunks (a window) at a
// time, with no lane left idle at a segment's end.  Per window a segmented
// scan across the lanes forms each segment's sum; a segment that runs past
// its window is carried in registers into the next one.
// Each segment's sum is stored by segment; a second kernel adds each row's
// segments in band order (a fixed order: results are reproducible), forms
// the residual, z and the FP64 residual partials.
//
// Back projection, tile-staged.  A tile is a run of Tv consecutive columns
// (a compact region of whole voxel columns again); the rays that cross it
// are a few runs of consecutive rows per view.  A set-up pass marks, per
// tile, the distinct rows of its columns in a bitmap, records them as runs
// and rewrites each entry's row as its rank among them (16 bits).  The back
// projection block copies those rows of z into LDS and gathers from there.
// Tiles whose distinct rows exceed the LDS budget keep global gathers.
#pragma once

#include "device.h"
#include "lines.h"

namespace ss {

constexpr int kStagedWaves = 8;                    // wavefronts per staged block
constexpr int kStagedThreads = kWave * kStagedWaves;
constexpr int kFinThreads = 256;                   // rows per residual block
constexpr int kBtRunCap = 128;                     // runs of staged rows per tile
constexpr int kBtMaxRows = 4096;                   // staged rows per tile (LDS)

// Per back-projection tile: distinct rows, runs, and whether it is staged.
struct BtMeta {
  int32_t rows;
  int32_t runs;
  int32_t ok;
  int32_t pad;
};

// One work tile of the band-staged forward projection: segments [s0, s1)
// of one band of one system, stored as its padded chunks [c0, c1).
struct BandTile {
  int32_t sys;
  int32_t band;
  int32_t s0, s1;
  int32_t c0, c1;
  int32_t pad[2];
};

constexpr int kBandWaves = 8;  // wavefronts per band-kernel block
constexpr int kWin = kWave;    // chunks per window: one per lane

constexpr int kSegBuf = 512;  // finished segment sums a band wavefront buffers

// Bytes of the band kernel's LDS: the band's NV floats per voxel, then per
// wavefront its buffer of segment sums.
__host__ __device__ inline size_t band_lds_bytes(int nv, int lg) {
  return (sizeof(float) * nv << lg) + sizeof(float) * nv * kSegBuf * kBandWaves;
}

// ------------------------------------------------------------ loads
// Four 16-bit indices of entries k0 .. k0+3 (k0 a multiple of 4).
__device__ inline u32x2 load_idx16_chunk(const uint16_t* idx, int64_t k0) {
  return gl(reinterpret_cast<const u32x2*>(idx))[k0 >> 2];
}

__device__ inline uint32_t idx16_at(const u32x2& c, int j) {
  const uint32_t w = j < 2 ? c.x : c.y;
  return (j & 1) ? (w >> 16) : (w & 0xffffu);
}

template <int NV>
__device__ inline Vec<NV> lds_vec(const float* x, uint32_t i) {
  Vec<NV> r;
  if constexpr (NV == 2) {
    const float2 v = reinterpret_cast<const float2*>(x)[i];
    r.v[0] = v.x;
    r.v[1] = v.y;
  } else {
    r.v[0] = x[i];
  }
  return r;
}

// p = sum over the chunk's SS_CHUNK entries of val * xs[idx] (xs in LDS),
// in entry order from 0.  Padding entries hold value 0 and index 0.  Every
// index is cut to `mask` (the band's capacity minus one): no read leaves
// the band.
template <int NV>
__device__ inline void chunk_dot_lds(const u32x2& ci, const Vec<NV>* v, const float* xs, uint32_t mask, float* p) {
  Vec<NV> x[SS_CHUNK];
#pragma unroll
  for (int j = 0; j < SS_CHUNK; ++j) x[j] = lds_vec<NV>(xs, idx16_at(ci, j) & mask);
#pragma unroll
  for (int h = 0; h < NV; ++h) {
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < SS_CHUNK; ++j) s = fmaf(v[j].v[h], x[j].v[h], s);
    p[h] = s;
  }
}

// One step of the segmented scan: v += the value CTRL brings from a lower
// lane, where `take`.
template <int NV, int CTRL, int ROWS>
__device__ inline void seg_scan_step(float* v, bool take) {
#pragma unroll
  for (int h = 0; h < NV; ++h) {
    const float t = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[h]), CTRL, ROWS, 0xf, false));
    v[h] = take ? v[h] + t : v[h];
  }
}

// Segmented inclusive scan over the 64 lanes of a wavefront: lane l ends
// with the sum of lanes a..l, a the last lane <= l that starts a segment,
// or lane 0 if none does.  `dist` is l - a (l + 1 if no lane <= l starts
// one).  Steps of 1, 2, 4, 8 lanes within rows of 16 (DPP row shifts), then
// the ends of rows 0 and 2 into rows 1 and 3 and the end of row 1 into rows
// 2 and 3 (DPP row broadcasts); a lane adds what a step brings only when no
// segment starts in the lanes that step spans.  The pattern of additions is
// fixed: results are reproducible.
template <int NV>
__device__ inline void seg_scan64(float* v, int dist) {
  const int l = lane_id();
  const int r = l & 15;
  seg_scan_step<NV, 0x111, 0xf>(v, r >= 1 && dist >= 1);
  seg_scan_step<NV, 0x112, 0xf>(v, r >= 2 && dist >= 2);
  seg_scan_step<NV, 0x114, 0xf>(v, r >= 4 && dist >= 4);
  seg_scan_step<NV, 0x118, 0xf>(v, r >= 8 && dist >= 8);
  seg_scan_step<NV, 0x142, 0xa>(v, (l & 16) != 0 && dist > r);
  seg_scan_step<NV, 0x143, 0xc>(v, l >= 32 && dist > l - 32);
}

// l - (the last lane <= l whose bit is set in `le`, the mask cut to lanes
// <= l), or l + 1 if none is.
__device__ inline int start_dist(uint64_t le, int l) {
  return le ? l - (63 - static_cast<int>(__builtin_clzll(le))) : l + 1;
}

// acc += sum over entries [lo, hi) of val[k] * xs[idx[k]], xs in LDS, by the
// L lanes of a group: aligned chunks of SS_CHUNK entries, P chunks per lane
// in flight per pass.  Entries of a chunk outside [lo, hi) are masked (their
// index is replaced by 0, always a valid LDS position); slots past the
// line's last chunk re-read it, so a pass issues all its loads without a
// branch.  Every index is cut to `mask` (the LDS vector's power-of-two
// capacity minus one), so no read can leave the allocation.
template <int NV, int WT, int L, int P>
__device__ inline void line_dot_lds(const uint16_t* idx, const void* val, const float* xs, int64_t lo, int64_t hi,
                                    int glane, float* acc, uint32_t mask) {
  constexpr int64_t C = SS_CHUNK;
  const int64_t first = lo & ~(C - 1);
  const int64_t last = (hi - 1) & ~(C - 1);
  for (int64_t base = first + C * glane; base < hi; base += C * P * L) {
    u32x2 c[P];
    Vec<NV> v[P][SS_CHUNK];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int64_t k0 = base + C * u * L;
      const int64_t kk = k0 <= last ? k0 : last;
      c[u] = load_idx16_chunk(idx, kk);
      load_val_chunk<NV, WT>(val, kk, v[u]);
    }
    // all of the pass's gathers first, then the products: the reads are in
    // flight together instead of each waiting before the next is issued
    Vec<NV> xv[P][SS_CHUNK];
#pragma unroll
    for (int u = 0; u < P; ++u) {
#pragma unroll
      for (int j = 0; j < SS_CHUNK; ++j) {
        const int64_t k = base + C * u * L + j;
        const bool in = k >= lo && k < hi;
        xv[u][j] = lds_vec<NV>(xs, in ? idx16_at(c[u], j) & mask : 0u);
      }
    }
#pragma unroll
    for (int u = 0; u < P; ++u) {
#pragma unroll
      for (int j = 0; j < SS_CHUNK; ++j) {
        const int64_t k = base + C * u * L + j;
        const bool in = k >= lo && k < hi;
#pragma unroll
        for (int h = 0; h < NV; ++h) {
          const float s = fmaf(v[u][j].v[h], xv[u][j].v[h], acc[h]);
          acc[h] = in ? s : acc[h];
        }
      }
    }
  }
}

// Copies `count` vectors of NV floats from global memory into LDS with
// 16-byte loads where the source allows (all threads of the block).
template <int NV, int T>
__device__ inline void stage_contiguous(float* dst, const float* src, int64_t count) {
  const int64_t nf = count * NV;
  const int64_t n4 = nf >> 2;
  const SS_GLOBAL u32x4* s4 = gl(reinterpret_cast<const u32x4*>(src));
  u32x4* d4 = reinterpret_cast<u32x4*>(dst);
  for (int64_t q = threadIdx.x; q < n4; q += T) d4[q] = s4[q];
  const int64_t rest = n4 << 2;
  if (static_cast<int64_t>(threadIdx.x) < nf - rest) dst[rest + threadIdx.x] = gl(src)[rest + threadIdx.x];
}

// ------------------------------------------------ scans for the set-up
// Exclusive scans of many independent pieces (one per system) in one
// launch sequence: per-tile sums, per-piece bases, then each tile scanned
// in LDS.  A piece of len elements occupies tiles [tile0, tile0 + tiles).
constexpr int kPScanThreads = 256;
constexpr int kPScanPer = 16;
constexpr int kPScanTile = kPScanThreads * kPScanPer;

template <typename T>
struct ScanPiece {
  T* ptr;
  int64_t len;
  int64_t tile0;
  int64_t tiles;
  T* total;  // receives the piece's sum (may be null)
};

template <typename T>
__device__ inline int find_piece(const ScanPiece<T>* pc, int npc, int64_t tile) {
  int lo = 0, hi = npc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pc[mid].tile0 <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__global__ __launch_bounds__(kPScanThreads) void k_pscan_tiles(const ScanPiece<T>* pc, int npc, T* tsum) {
  __shared__ T red[kPScanThreads / kWave];
  const int p = find_piece(pc, npc, blockIdx.x);
  const ScanPiece<T>& P = pc[p];
  const int64_t base = (static_cast<int64_t>(blockIdx.x) - P.tile0) * kPScanTile;
  T s = 0;
  for (int j = 0; j < kPScanPer; ++j) {
    const int64_t i = base + threadIdx.x + j * kPScanThreads;
    if (i < P.len) s += P.ptr[i];
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    T t = 0;
    for (int w = 0; w < kPScanThreads / kWave; ++w) t += red[w];
    tsum[blockIdx.x] = t;
  }
}

// One thread per piece turns its tile sums into exclusive tile bases.
template <typename T>
__global__ void k_pscan_bases(const ScanPiece<T>* pc, int npc, T* tsum) {
  const int p = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= npc) return;
  const ScanPiece<T>& P = pc[p];
  T run = 0;
  for (int64_t t = 0; t < P.tiles; ++t) {
    const T v = tsum[P.tile0 + t];
    tsum[P.tile0 + t] = run;
    run += v;
  }
  if (P.total) *P.total = run;
}

template <typename T>
__global__ __launch_bounds__(kPScanThreads) void k_pscan_apply(const ScanPiece<T>* pc, int npc, const T* tbase) {
  __shared__ T vals[kPScanTile];
  __shared__ T tot[kPScanThreads];
  const int p = find_piece(pc, npc, blockIdx.x);
  const ScanPiece<T>& P = pc[p];
  const int64_t base = (static_cast<int64_t>(blockIdx.x) - P.tile0) * kPScanTile;
  for (int j = 0; j < kPScanPer; ++j) {
    const int t = threadIdx.x + j * kPScanThreads;
    vals[t] = base + t < P.len ? P.ptr[base + t] : T(0);
  }
  __syncthreads();
  T run = 0;
  for (int j = 0; j < kPScanPer; ++j) {
    const T v = vals[threadIdx.x * kPScanPer + j];
    vals[threadIdx.x * kPScanPer + j] = run;  // exclusive within the thread's run
    run += v;
  }
  tot[threadIdx.x] = run;
  __syncthreads();
  for (int o = 1; o < kPScanThreads; o <<= 1) {
    const T v = threadIdx.x >= static_cast<unsigned>(o) ? tot[threadIdx.x - o] : T(0);
    __syncthreads();
    tot[threadIdx.x] += v;
    __syncthreads();
  }
  const T before = tbase[blockIdx.x] + (threadIdx.x > 0 ? tot[threadIdx.x - 1] : T(0));
  for (int j = 0; j < kPScanPer; ++j) vals[threadIdx.x * kPScanPer + j] += before;
  __syncthreads();
  for (int j = 0; j < kPScanPer; ++j) {
    const int t = threadIdx.x + j * kPScanThreads;
    if (base + t < P.len) P.ptr[base + t] = vals[t];
  }
}

// Fills n elements with zero (all systems' set-up arrays: one launch each).
template <typename T>
__global__ void k_fill_zero(T* p, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = T(0);
}

// Packed (segments, entries) pair: segments in the high 32 bits, entries in
// the low ones; per system both stay below 2^31, so sums never carry.
__host__ __device__ inline uint64_t seg_pack(uint32_t segs, uint32_t entries) {
  return (static_cast<uint64_t>(segs) << 32) | entries;
}
__host__ __device__ inline uint32_t seg_count(uint64_t v) { return static_cast<uint32_t>(v >> 32); }
__host__ __device__ inline uint32_t seg_entries(uint64_t v) { return static_cast<uint32_t>(v); }

// Entries of a segment padded to whole chunks.
__host__ __device__ inline int64_t pad_chunk(int64_t n) { return (n + SS_CHUNK - 1) & ~int64_t{SS_CHUNK - 1}; }

// First position in [lo, hi) whose column is >= key (columns ascend).
__device__ inline int64_t col_lower_bound(const int32_t* col, int64_t lo, int64_t hi, int32_t key) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (gl(col)[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

}  // namespace ss
