// Ordered-subset SART on the folded pair: the paper's ref. [004] (ordered
// subsets of projection data) applied to SART (ref. [001]), with subsets
// that the fold of Section 2 preserves.
//
// A subset is closed under the ray mirror i -> M-1-i (the rays of sources k
// and K-1-k of the symmetric scan); the fold maps it onto a block of rows of
// the folded system.  With rays ordered source-major, subset s of S is the
// folded rows [s R, (s+1) R), R = m / S.  One pass applies, for s = 0 .. S-1,
//     f <- f + lambda * V_s^-1 A_s^T W_s^-1 (p_s - A_s f)
// to both halves, with W the row sums of A(2) and V_s the column sums of
// A(2) over the rows of subset s (equal to A's over the mirror-closed
// subset), so that the recombined iterates are those of ordered-subset SART
// on A itself.
//
// Launches per pass: the residual of the current image (forward projection
// of every row, FP64 partials per block), its finalisation (history entry,
// stop decision, pass counter), then for each subset a forward kernel over
// its rows (z = W^-1 (p - A f)) and a back projection over every column,
// reading only the column's entries in that subset from a subset-major copy
// of the CSC (all columns' entries of subset s are contiguous, so a launch
// streams 1/S of the entries instead of touching every column's cache lines
// S times per pass), and updating f in place: each column
// belongs to one lane group, and the next subset's kernel starts after this
// one has ended.  A stop decided by the finalisation is read by every later
// kernel of the pass, so a stopped system's image is f^k exactly.

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "device.h"
#include "graph_cache.h"
#include "interleave.h"
#include "internal.h"
#include "lines.h"

namespace ss {
namespace {

constexpr int kOsWPB = 4;  // wavefronts per block
constexpr int kOsThreads = kWave * kOsWPB;

struct OsState {
  double pnorm2;
  double last_res;
  int32_t k;     // passes applied to the image
  int32_t stop;  // 1: the image is final
};

struct OsDesc {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const void* val;
  const int64_t* col_ptr;
  const int32_t* row_idx;
  const void* val_t;
  const int64_t* col_ptr_os;   // subset-major CSC: subset s, column j at s*n + j
  const int32_t* row_idx_os;
  const void* val_t_os;
  const float* inv_col_sub;
  const float* p;
  const float* inv_row;
  float* f;
  float* z;
  double* res_hist;
  double* partials;
  OsState* st;
  int64_t m, n;
  int32_t S, R;
  int64_t blk0[3];    // first block of this system in the subset-row, all-row and column grids
  int32_t nblk[3];
};

enum { kSubRows = 0, kAllRows = 1, kCols = 2 };

struct OsParams {
  float lambda;
  int32_t max_iter;
  double tol;
  int32_t nonneg;
  int32_t res_every;  // the pass-start residual is taken when k % res_every == 0, and at k = max_iter
};

// Whether the residual of the image after k passes is evaluated.
__device__ inline bool residual_pass(const OsParams* prm, int k) {
  return k % prm->res_every == 0 || k >= prm->max_iter;
}

constexpr int kOsChunk = 16;
struct OsChunk {
  OsDesc d[kOsChunk];
  OsParams prm;
  int32_t count;
  int32_t first;
  int32_t zero_start;
};

// The system and block-local index of grid block b (uniform per block),
// from a block -> system table filled at set-up: the blocks of these
// kernels carry little work, so one lookup load beats a binary search.
template <int G>
__device__ inline int os_block(const OsDesc* t, const int32_t* b2s, int nsys, uint32_t ntiles, int xcd,
                               int64_t* local) {
  const uint32_t b = __builtin_amdgcn_readfirstlane(xcd ? xcd_remap(blockIdx.x, ntiles) : blockIdx.x);
  const int s = nsys == 1 ? 0 : __builtin_amdgcn_readfirstlane(gl(b2s)[b]);
  *local = static_cast<int64_t>(b) - t[s].blk0[G];
  return s;
}

__global__ void k_os_blk2sys(const OsDesc* t, int32_t* b0, int32_t* b1, int32_t* b2) {
  const OsDesc& d = t[blockIdx.x];
  int32_t* out[3] = {b0, b1, b2};
  for (int k = 0; k < 3; ++k)
    for (int64_t i = threadIdx.x; i < d.nblk[k]; i += blockDim.x) out[k][d.blk0[k] + i] = blockIdx.x;
}

__global__ __launch_bounds__(kOsThreads) void k_os_setup(OsChunk ch, OsDesc* table, OsParams* prm) {
  const OsDesc& d = ch.d[blockIdx.x];
  if (ch.zero_start)
    for (int64_t i = threadIdx.x; i < 2 * d.n; i += kOsThreads) d.f[i] = 0.0f;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < 2 * d.m; i += kOsThreads) {
    const double v = d.p[i];
    s += v * v;
  }
  __shared__ double red[kOsWPB];
  s = block_sum<kOsWPB>(s, red);
  if (threadIdx.x == 0) {
    table[ch.first + blockIdx.x] = d;
    d.st->pnorm2 = s;
    d.st->last_res = 0.0;
    d.st->k = 0;
    d.st->stop = 0;
    if (ch.first == 0 && blockIdx.x == 0) *prm = ch.prm;
  }
}

// Forward projection of rows [r0, r0 + rows) in tiles of RPW*kOsWPB rows.
// RES: FP64 partial of |p - A f|^2 per block into `partials`; otherwise
// z = W^-1 (p - A f).  Stream forms (SF): 0 entry-wise, 1 aligned chunks,
// 2 interleaved (the rows read from the workspace copy in the interleaved
// order; the sums run in the entry-wise order, so the results are the same
// bit for bit).
template <int WT, int RPW, int U, int SF, bool RES>
__global__ __launch_bounds__(kOsThreads) void k_os_fp(const OsParams* __restrict__ prm,
                                                      const OsDesc* __restrict__ table,
                                                      const int32_t* __restrict__ b2s, int nsys, uint32_t ntiles,
                                                      int xcd, int sub) {
  constexpr int L = kWave / RPW;
  __shared__ double red[kOsWPB];
  if (blockIdx.x >= ntiles) return;
  int64_t local;
  const int si = os_block<RES ? kAllRows : kSubRows>(table, b2s, nsys, ntiles, xcd, &local);
  const OsDesc& S = table[si];
  if (*gl(&S.st->stop)) return;
  if (RES && !residual_pass(prm, *gl(&S.st->k))) return;
  const int64_t r0 = RES ? 0 : static_cast<int64_t>(sub) * S.R;
  const int64_t r1 = RES ? S.m : r0 + S.R;
  const int glane = lane_id() % L;
  const int64_t row = r0 + local * (RPW * kOsWPB) + wave_id() * RPW + lane_id() / L;
  const bool in = row < r1;
  const int64_t li = in ? row : r1 - 1;
  const Vec<2> pv = load_vec<2>(S.p, li);
  const float w = gl(S.inv_row)[li];
  const int64_t lo = gl(S.row_ptr)[li];
  const int64_t hi = in ? gl(S.row_ptr)[li + 1] : lo;
  float acc[2] = {0.0f, 0.0f};
  if constexpr (SF == 2) line_dot_i<2, WT, L, U / SS_CHUNK>(S.col_idx, S.val, S.f, lo, hi, glane, acc);
  else line_dot<2, WT, L, U, SF == 1>(S.col_idx, S.val, S.f, lo, hi, glane, acc);
  acc[0] = group_sum<L>(acc[0]);
  acc[1] = group_sum<L>(acc[1]);
  const bool owner = glane == 0 && in;
  const float ra = pv.v[0] - acc[0], rb = pv.v[1] - acc[1];
  if constexpr (RES) {
    const double d = owner ? static_cast<double>(ra) * ra + static_cast<double>(rb) * rb : 0.0;
    const double tot = block_sum<kOsWPB>(d, red);
    if (threadIdx.x == 0) glw(S.partials)[local] = tot;
  } else {
    if (owner) store_vec<2>(S.z, row, Vec<2>{{ra * w, rb * w}});
  }
}

// One block per system: rel_res of the current image from the partials in
// index order, the history entry, the stop decision and the pass counter.
__global__ __launch_bounds__(kOsThreads) void k_os_fin(const OsDesc* __restrict__ table, const OsParams* prm) {
  const OsDesc& S = table[blockIdx.x];
  if (*gl(&S.st->stop)) return;
  if (!residual_pass(prm, *gl(&S.st->k))) {  // a pass without the residual
    __syncthreads();
    if (threadIdx.x == 0) S.st->k += 1;
    return;
  }
  __shared__ double red[kOsWPB];
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < S.nblk[kAllRows]; t += kOsThreads) acc += gl(S.partials)[t];
  const double rsum = block_sum<kOsWPB>(acc, red);
  if (threadIdx.x == 0) {
    OsState* st = S.st;
    const double pn = st->pnorm2;
    const double rel = pn > 0.0 ? sqrt(rsum / pn) : sqrt(rsum);
    const int k = st->k;
    if (S.res_hist) glw(S.res_hist)[k] = rel;
    st->last_res = rel;
    if (rel <= prm->tol || k >= prm->max_iter) st->stop = 1;
    else st->k = k + 1;
  }
}

// Back projection of subset `sub` and the in-place update, column by column.
template <int WT, int CPW, int U, bool CH>
__global__ __launch_bounds__(kOsThreads) void k_os_bp(const OsParams* __restrict__ prm,
                                                      const OsDesc* __restrict__ table,
                                                      const int32_t* __restrict__ b2s, int nsys, uint32_t ntiles,
                                                      int xcd, int sub) {
  constexpr int L = kWave / CPW;
  if (blockIdx.x >= ntiles) return;
  int64_t local;
  const int si = os_block<kCols>(table, b2s, nsys, ntiles, xcd, &local);
  const OsDesc& S = table[si];
  if (*gl(&S.st->stop)) return;
  const int glane = lane_id() % L;
  const int64_t col = local * (CPW * kOsWPB) + wave_id() * CPW + lane_id() / L;
  const bool in = col < S.n;
  const int64_t ci = in ? col : S.n - 1;
  const int64_t* cp = S.col_ptr_os + static_cast<int64_t>(sub) * S.n + ci;
  const int64_t lo = gl(cp)[0];
  const int64_t hi = in ? gl(cp)[1] : lo;
  Vec<2> fv = load_vec<2>(S.f, ci);
  const float tl = prm->lambda * gl(S.inv_col_sub)[static_cast<int64_t>(sub) * S.n + ci];
  float acc[2] = {0.0f, 0.0f};
  line_dot<2, WT, L, U, CH>(S.row_idx_os, S.val_t_os, S.z, lo, hi, glane, acc);
  acc[0] = group_sum<L>(acc[0]);
  acc[1] = group_sum<L>(acc[1]);
  if (glane == 0 && in) {
    fv.v[0] = fmaf(tl, acc[0], fv.v[0]);
    fv.v[1] = fmaf(tl, acc[1], fv.v[1]);
    if (prm->nonneg) fv = project_nonneg<2>(fv);
    store_vec<2>(S.f, col, fv);
  }
}

// Subset ranges of each column and the FP32 reciprocals of the FP64 subset
// column sums of A(2) (the second value of each FP32 pair): one thread per
// column walks its ascending rows.
__global__ void k_subsets_build(ss_system sys, int32_t S, int32_t R, int32_t* col_sub, float* inv_col_sub) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= sys.n) return;
  const float* v = static_cast<const float*>(sys.val_t);
  const int64_t base = sys.col_ptr[j], end = sys.col_ptr[j + 1];
  int64_t e = base;
  for (int s = 0; s < S; ++s) {
    col_sub[static_cast<int64_t>(s) * sys.n + j] = static_cast<int32_t>(e - base);
    const int64_t lim = static_cast<int64_t>(s + 1) * R;
    double sum = 0.0;
    for (; e < end && sys.row_idx[e] < lim; ++e) sum += static_cast<double>(v[2 * e + 1]);
    inv_col_sub[static_cast<int64_t>(s) * sys.n + j] = sum != 0.0 ? static_cast<float>(1.0 / sum) : 0.0f;
  }
  col_sub[static_cast<int64_t>(S) * sys.n + j] = static_cast<int32_t>(e - base);
}

// Copies each column's subset ranges into the subset-major CSC.
__global__ void k_subsets_scatter(ss_system sys, int32_t S, const int32_t* col_sub, const int64_t* col_ptr_os,
                                  int32_t* row_idx_os, float* val_t_os) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= sys.n) return;
  const int64_t base = sys.col_ptr[j];
  const float* v = static_cast<const float*>(sys.val_t);
  for (int s = 0; s < S; ++s) {
    const int64_t a = base + col_sub[static_cast<int64_t>(s) * sys.n + j];
    const int64_t b = base + col_sub[static_cast<int64_t>(s + 1) * sys.n + j];
    int64_t o = col_ptr_os[static_cast<int64_t>(s) * sys.n + j];
    for (int64_t e = a; e < b; ++e, ++o) {
      row_idx_os[o] = sys.row_idx[e];
      val_t_os[2 * o] = v[2 * e];
      val_t_os[2 * o + 1] = v[2 * e + 1];
    }
  }
}

// ------------------------------------------------------------------ host
struct OsCfg {
  int rpw, cpw, xcd, u, ch;
};

struct OsLayout {
  size_t params, table, states, b2s[3], total;
  std::vector<size_t> z_off, part_off;
  std::vector<size_t> fi_idx, fi_val;  // interleaved copies of the rows (chunked bit 2)
};

inline size_t al256(size_t v) { return (v + 255) & ~size_t{255}; }

OsLayout os_layout(const ss_system* sys, int nsys, int chunked) {
  OsLayout L;
  size_t o = 0;
  L.params = o;
  o += al256(sizeof(OsParams));
  L.table = o;
  o += al256(sizeof(OsDesc) * nsys);
  L.states = o;
  o += al256(sizeof(OsState) * nsys);
  // block -> system tables, sized for the smallest tiles (one line per wave)
  int64_t nb[3] = {0, 0, 0};
  for (int s = 0; s < nsys; ++s) {
    nb[0] += (sys[s].m + kOsWPB - 1) / kOsWPB;  // a subset has at most m rows
    nb[1] += (sys[s].m + kOsWPB - 1) / kOsWPB;
    nb[2] += (sys[s].n + kOsWPB - 1) / kOsWPB;
  }
  for (int k = 0; k < 3; ++k) {
    L.b2s[k] = o;
    o += al256(sizeof(int32_t) * static_cast<size_t>(nb[k]));
  }
  for (int s = 0; s < nsys; ++s) {
    L.z_off.push_back(o);
    o += al256(sizeof(float) * 2 * static_cast<size_t>(sys[s].m));
  }
  for (int s = 0; s < nsys; ++s) {
    L.part_off.push_back(o);
    o += al256(sizeof(double) * static_cast<size_t>((sys[s].m + kOsWPB - 1) / kOsWPB));  // 1 row per wave
  }
  if (chunked & 4) {
    for (int s = 0; s < nsys; ++s) {
      const size_t cap = static_cast<size_t>(sys[s].nnz) + SS_CHUNK;
      L.fi_idx.push_back(o);
      o += al256(sizeof(int32_t) * cap);
      L.fi_val.push_back(o);
      o += al256(2 * sizeof(float) * cap);
    }
  }
  L.total = o;
  return L;
}

ss_status os_validate(const ss_system* sys, const ss_subsets* sub, int nsys, const ss_sart_opts* o, const char* fn) {
  if (!sys || !sub || nsys <= 0 || !o) return fail(SS_E_ARG, "%s: NULL systems, subsets or options", fn);
  for (int s = 0; s < nsys; ++s) {
    const ss_system& Y = sys[s];
    if (Y.nvals != 2 || Y.wdtype != SS_F32)
      return fail(SS_E_ARG, "%s: system %d: ordered subsets need a folded FP32 pair", fn, s);
    if (ss_status e = check_ascending(&Y, fn)) return e;
    if (Y.m <= 0 || Y.n <= 0 || Y.nnz < 0 || Y.m > INT32_MAX || Y.n > INT32_MAX)
      return fail(SS_E_ARG, "%s: system %d has a bad size", fn, s);
    if (!Y.row_ptr || !Y.col_ptr || !Y.p || !Y.inv_row ||
        (Y.nnz > 0 && (!Y.col_idx || !Y.val || !Y.row_idx || !Y.val_t)))
      return fail(SS_E_ARG, "%s: system %d has a NULL array", fn, s);
    auto aligned = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    if (Y.nnz > 0 && !(aligned(Y.col_idx) && aligned(Y.val) && aligned(Y.row_idx) && aligned(Y.val_t)))
      return fail(SS_E_ARG, "%s: system %d: index and value arrays must be 16-byte aligned", fn, s);
    const ss_subsets& B = sub[s];
    if (B.S <= 0 || B.S > Y.m || Y.m % B.S != 0 || !B.col_sub || !B.inv_col_sub || !B.col_ptr_os ||
        (Y.nnz > 0 && (!B.row_idx_os || !B.val_t_os)))
      return fail(SS_E_ARG, "%s: system %d: S must divide m and the subset arrays be set", fn, s);
    if (Y.nnz > 0 && !(aligned(B.row_idx_os) && aligned(B.val_t_os)))
      return fail(SS_E_ARG, "%s: system %d: subset CSC arrays must be 16-byte aligned", fn, s);
  }
  if (!(o->lambda > 0.0f && o->lambda < 2.0f)) return fail(SS_E_ARG, "%s: lambda must be in (0, 2)", fn);
  if (o->max_iter < 0 || o->max_iter > (1 << 30)) return fail(SS_E_ARG, "%s: bad max_iter", fn);
  if (o->tol > 0.0 && o->check_every <= 0) return fail(SS_E_ARG, "%s: check_every must be > 0", fn);
  auto ok_pw = [](int v, int maxv) { return v == 0 || (v > 0 && v <= maxv && (v & (v - 1)) == 0); };
  if (!ok_pw(o->rows_per_wave, 8) || !ok_pw(o->cols_per_wave, 64))
    return fail(SS_E_ARG, "%s: rows_per_wave must be 0,1,2,4,8 and cols_per_wave 0,1,..,64", fn);
  if (o->unroll != 0 && o->unroll != 4 && o->unroll != 8) return fail(SS_E_ARG, "%s: unroll must be 0, 4 or 8", fn);
  if (o->chunked < 0 || o->chunked > 7) return fail(SS_E_ARG, "%s: chunked must be 0..7", fn);
  if (o->nonneg != 0 && o->nonneg != 1) return fail(SS_E_ARG, "%s: nonneg must be 0 or 1", fn);
  if (o->staged != 0) return fail(SS_E_ARG, "%s: the staged forms are for ss_sart_* only (staged must be 0)", fn);
  if (o->residual_every < 0) return fail(SS_E_ARG, "%s: residual_every must be >= 0", fn);
  return SS_OK;
}

// Lanes per line from the mean line length: the smallest power of two of
// lines per wavefront whose lanes still cover ~48 entries.
int os_per_wave(double mean_len, int maxv) {
  int v = 1;
  while (v < maxv && mean_len * v < 48.0) v <<= 1;
  return v;
}

// Defaults from the statistics of the systems: a subset back projection sees
// only 1/S of each column, so it packs more columns into a wavefront than
// the full back projection does.
OsCfg os_cfg(const ss_system* sys, int nsys, int S, const ss_sart_opts* o) {
  double nnz = 0, m = 0, n = 0;
  for (int s = 0; s < nsys; ++s) {
    nnz += static_cast<double>(sys[s].nnz);
    m += static_cast<double>(sys[s].m);
    n += static_cast<double>(sys[s].n);
  }
  OsCfg c;
  c.rpw = o->rows_per_wave ? o->rows_per_wave : os_per_wave(nnz / m, 8);
  // a subset holds ~1/S of each column: few entries, so few lanes per column
  // (measured on the 256-slice batch, S = 12, ~3 entries: one lane per
  // column, 5.2 ms per pass, against 8.1 ms with four)
  const double sub_len = nnz / (n * S);
  int lanes = 1;
  while (lanes < kWave && lanes * 4 < sub_len) lanes <<= 1;
  c.cpw = o->cols_per_wave ? o->cols_per_wave : kWave / lanes;
  c.xcd = o->xcd_remap ? 1 : 0;
  c.u = o->unroll ? o->unroll : 4;
  c.ch = o->chunked;
  return c;
}

struct OsGrid {
  uint32_t nb[3] = {0, 0, 0};
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <int WT, int U, int SF, bool RES>
void os_fp_rpw(int rpw, const OsParams* prm, const OsDesc* t, const int32_t* b2s, int nsys, uint32_t nb, int xcd,
               int sub, hipStream_t st) {
  const dim3 g(nb), b(kOsThreads);
  switch (rpw) {
    case 1: k_os_fp<WT, 1, U, SF, RES><<<g, b, 0, st>>>(prm, t, b2s, nsys, nb, xcd, sub); break;
    case 2: k_os_fp<WT, 2, U, SF, RES><<<g, b, 0, st>>>(prm, t, b2s, nsys, nb, xcd, sub); break;
    case 4: k_os_fp<WT, 4, U, SF, RES><<<g, b, 0, st>>>(prm, t, b2s, nsys, nb, xcd, sub); break;
    default: k_os_fp<WT, 8, U, SF, RES><<<g, b, 0, st>>>(prm, t, b2s, nsys, nb, xcd, sub); break;
  }
}

// The forward launch in the stream form of the chunked bits: bit 2
// interleaved, else bit 0 chunked, else entry-wise.
template <int U, bool RES>
void os_fp(const OsCfg& c, const OsParams* prm, const OsDesc* t, const int32_t* b2s, int nsys, uint32_t nb, int sub,
           hipStream_t st) {
  if (c.ch & 4) os_fp_rpw<SS_F32, U, 2, RES>(c.rpw, prm, t, b2s, nsys, nb, c.xcd, sub, st);
  else if (c.ch & 1) os_fp_rpw<SS_F32, U, 1, RES>(c.rpw, prm, t, b2s, nsys, nb, c.xcd, sub, st);
  else os_fp_rpw<SS_F32, U, 0, RES>(c.rpw, prm, t, b2s, nsys, nb, c.xcd, sub, st);
}

template <int WT, int U, bool CH>
void os_bp_cpw(int cpw, const OsParams* prm, const OsDesc* t, const int32_t* b2s, int nsys, uint32_t nb, int xcd,
               int sub, hipStream_t st) {
  const dim3 g(nb), b(kOsThreads);
  switch (cpw) {
    case 1: k_os_bp<WT, 1, U, CH><<<g, b, 0, st>>>(prm, t, b2s, nsys, nb, xcd, sub); break;
    case 2: k_os_bp<WT, 2, U, CH><<<g, b, 0, st>>>(prm, t, b2s, nsys, nb, xcd, sub); break;
    case 4: k_os_bp<WT, 4, U, CH><<<g, b, 0, st>>>(prm, t, b2s, nsys, nb, xcd, sub); break;
    case 8: k_os_bp<WT, 8, U, CH><<<g, b, 0, st>>>(prm, t, b2s, nsys, nb, xcd, sub); break;
    case 16: k_os_bp<WT, 16, U, CH><<<g, b, 0, st>>>(prm, t, b2s, nsys, nb, xcd, sub); break;
    case 32: k_os_bp<WT, 32, U, CH><<<g, b, 0, st>>>(prm, t, b2s, nsys, nb, xcd, sub); break;
    default: k_os_bp<WT, 64, U, CH><<<g, b, 0, st>>>(prm, t, b2s, nsys, nb, xcd, sub); break;
  }
}

// One pass group: residual, finalisation, then the S subset updates.
template <int U>
void os_pass(const OsCfg& c, const OsParams* prm, const OsDesc* t, const int32_t* const* b2s, int nsys, int S,
             const OsGrid& g, hipStream_t st) {
  const bool bch = c.ch & 2;
  os_fp<U, true>(c, prm, t, b2s[kAllRows], nsys, g.nb[kAllRows], 0, st);
  k_os_fin<<<nsys, kOsThreads, 0, st>>>(t, prm);
  for (int s = 0; s < S; ++s) {
    os_fp<U, false>(c, prm, t, b2s[kSubRows], nsys, g.nb[kSubRows], s, st);
    if (bch) os_bp_cpw<SS_F32, U, true>(c.cpw, prm, t, b2s[kCols], nsys, g.nb[kCols], c.xcd, s, st);
    else os_bp_cpw<SS_F32, U, false>(c.cpw, prm, t, b2s[kCols], nsys, g.nb[kCols], c.xcd, s, st);
  }
}

void os_passes(const OsCfg& c, const char* ws, const OsLayout& L, int nsys, int S, const OsGrid& g, int count,
               hipStream_t st) {
  const OsParams* prm = reinterpret_cast<const OsParams*>(ws + L.params);
  const OsDesc* t = reinterpret_cast<const OsDesc*>(ws + L.table);
  const int32_t* b2s[3] = {reinterpret_cast<const int32_t*>(ws + L.b2s[0]),
                           reinterpret_cast<const int32_t*>(ws + L.b2s[1]),
                           reinterpret_cast<const int32_t*>(ws + L.b2s[2])};
  for (int i = 0; i < count; ++i) {
    if (c.u == 8) os_pass<8>(c, prm, t, b2s, nsys, S, g, st);
    else os_pass<4>(c, prm, t, b2s, nsys, S, g, st);
  }
}

struct OsKey {
  int device;
  const void* ws;
  int nsys, S;
  uint32_t nb0, nb1, nb2;
  int rpw, cpw, xcd, u, ch, count;
  bool operator<(const OsKey& o) const {
    return std::tie(device, ws, nsys, S, nb0, nb1, nb2, rpw, cpw, xcd, u, ch, count) <
           std::tie(o.device, o.ws, o.nsys, o.S, o.nb0, o.nb1, o.nb2, o.rpw, o.cpw, o.xcd, o.u, o.ch, o.count);
  }
};

GraphCache<OsKey>& os_graphs() {
  static auto* g = new GraphCache<OsKey>(16);  // lives until process exit
  return *g;
}

}  // namespace
}  // namespace ss

using namespace ss;

extern "C" ss_status ss_subsets_build(const ss_system* sys, ss_subsets* sub, void* stream) {
  clear_error();
  if (!sys || !sub) return fail(SS_E_ARG, "ss_subsets_build: NULL argument");
  if (sys->nvals != 2 || sys->wdtype != SS_F32)
    return fail(SS_E_ARG, "ss_subsets_build: ordered subsets need a folded FP32 pair");
  if (ss_status e = check_ascending(sys, "ss_subsets_build")) return e;
  if (sys->m <= 0 || sys->n <= 0 || !sys->col_ptr || (sys->nnz > 0 && (!sys->row_idx || !sys->val_t)))
    return fail(SS_E_ARG, "ss_subsets_build: bad system");
  if (sub->S <= 0 || sub->S > sys->m || sys->m % sub->S != 0)
    return fail(SS_E_ARG, "ss_subsets_build: S = %d must divide m = %lld", sub->S, (long long)sys->m);
  if (!sub->col_sub || !sub->inv_col_sub || !sub->col_ptr_os || (sys->nnz > 0 && (!sub->row_idx_os || !sub->val_t_os)))
    return fail(SS_E_ARG, "ss_subsets_build: NULL subset arrays");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int S = sub->S;
  const unsigned nb = static_cast<unsigned>(cdiv(sys->n, 256));
  k_subsets_build<<<nb, 256, 0, st>>>(*sys, S, static_cast<int32_t>(sys->m / S), sub->col_sub, sub->inv_col_sub);
  SS_HIP_TRY(hipGetLastError());
  // offsets of the subset-major CSC: an exclusive scan, subset by subset,
  // of the per-column counts (on the host: set-up work, done once)
  const size_t cells = static_cast<size_t>(S + 1) * static_cast<size_t>(sys->n);
  std::vector<int32_t> cs(cells);
  SS_HIP_TRY(hipMemcpyAsync(cs.data(), sub->col_sub, sizeof(int32_t) * cells, hipMemcpyDeviceToHost, st));
  SS_HIP_TRY(hipStreamSynchronize(st));
  std::vector<int64_t> cp(static_cast<size_t>(S) * sys->n + 1);
  int64_t acc = 0;
  for (int s = 0; s < S; ++s)
    for (int64_t j = 0; j < sys->n; ++j) {
      cp[static_cast<size_t>(s) * sys->n + j] = acc;
      acc += cs[static_cast<size_t>(s + 1) * sys->n + j] - cs[static_cast<size_t>(s) * sys->n + j];
    }
  cp.back() = acc;
  if (acc != sys->nnz) return fail(SS_E_SHAPE, "ss_subsets_build: subset counts do not add up to nnz");
  SS_HIP_TRY(hipMemcpy(sub->col_ptr_os, cp.data(), sizeof(int64_t) * cp.size(), hipMemcpyHostToDevice));
  if (sys->nnz > 0) {
    k_subsets_scatter<<<nb, 256, 0, st>>>(*sys, S, sub->col_sub, sub->col_ptr_os, sub->row_idx_os,
                                          static_cast<float*>(sub->val_t_os));
    SS_HIP_TRY(hipGetLastError());
  }
  return SS_OK;
}

extern "C" ss_status ss_ossart_workspace_bytes(const ss_system* sys, const ss_subsets* sub, int32_t nsys,
                                               const ss_sart_opts* opts, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(SS_E_ARG, "ss_ossart_workspace_bytes: NULL bytes");
  if (ss_status s = os_validate(sys, sub, nsys, opts, "ss_ossart_workspace_bytes")) return s;
  *bytes = os_layout(sys, nsys, opts->chunked).total;
  return SS_OK;
}

extern "C" ss_status ss_ossart_solve(const ss_system* sys, const ss_subsets* sub, int32_t nsys, float* const* f,
                                     double* const* res_hist, const ss_sart_opts* opts, int32_t* passes,
                                     void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (ss_status s = os_validate(sys, sub, nsys, opts, "ss_ossart_solve")) return s;
  if (!f || !workspace) return fail(SS_E_ARG, "ss_ossart_solve: NULL images or workspace");
  const int S = sub[0].S;
  for (int s = 0; s < nsys; ++s) {
    if (!f[s] || (res_hist && !res_hist[s])) return fail(SS_E_ARG, "ss_ossart_solve: NULL image %d", s);
    if (sub[s].S != S) return fail(SS_E_ARG, "ss_ossart_solve: all systems must have the same S");
  }
  const OsLayout L = os_layout(sys, nsys, opts->chunked);
  if (workspace_bytes < L.total)
    return fail(SS_E_WORKSPACE, "ss_ossart_solve: workspace needs %zu bytes", L.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const OsCfg c = os_cfg(sys, nsys, S, opts);
  // descriptors, grids and states
  OsGrid g;
  std::vector<OsDesc> ds(nsys);
  const int64_t rows_blk = static_cast<int64_t>(c.rpw) * kOsWPB, cols_blk = static_cast<int64_t>(c.cpw) * kOsWPB;
  int64_t acc[3] = {0, 0, 0};
  for (int s = 0; s < nsys; ++s) {
    const ss_system& Y = sys[s];
    OsDesc& d = ds[s];
    d = OsDesc{};
    d.row_ptr = Y.row_ptr;
    d.col_idx = Y.col_idx;
    d.val = Y.val;
    if ((c.ch & 4) && Y.nnz > 0) {  // the rows in the interleaved order of the forward kernels' lanes
      d.col_idx = reinterpret_cast<int32_t*>(ws + L.fi_idx[s]);
      d.val = ws + L.fi_val[s];
      if (ss_status e = interleave_lines(Y.row_ptr, Y.m, Y.col_idx, Y.val, const_cast<int32_t*>(d.col_idx),
                                         const_cast<void*>(d.val), 2 * sizeof(float), kWave / c.rpw, st))
        return e;
    }
    d.col_ptr = Y.col_ptr;
    d.row_idx = Y.row_idx;
    d.val_t = Y.val_t;
    d.col_ptr_os = sub[s].col_ptr_os;
    d.row_idx_os = sub[s].row_idx_os;
    d.val_t_os = sub[s].val_t_os;
    d.inv_col_sub = sub[s].inv_col_sub;
    d.p = Y.p;
    d.inv_row = Y.inv_row;
    d.f = f[s];
    d.z = reinterpret_cast<float*>(ws + L.z_off[s]);
    d.res_hist = res_hist ? res_hist[s] : nullptr;
    d.partials = reinterpret_cast<double*>(ws + L.part_off[s]);
    d.st = reinterpret_cast<OsState*>(ws + L.states) + s;
    d.m = Y.m;
    d.n = Y.n;
    d.S = S;
    d.R = static_cast<int32_t>(Y.m / S);
    const int64_t nb[3] = {cdiv(d.R, rows_blk), cdiv(Y.m, rows_blk), cdiv(Y.n, cols_blk)};
    for (int k = 0; k < 3; ++k) {
      d.blk0[k] = acc[k];
      d.nblk[k] = static_cast<int32_t>(nb[k]);
      acc[k] += nb[k];
    }
  }
  for (int k = 0; k < 3; ++k) {
    if (acc[k] > static_cast<int64_t>(UINT32_MAX)) return fail(SS_E_ARG, "ss_ossart_solve: grid too large");
    g.nb[k] = static_cast<uint32_t>(acc[k]);
  }
  for (int s0 = 0; s0 < nsys; s0 += kOsChunk) {
    OsChunk ch{};
    ch.first = s0;
    ch.count = std::min(kOsChunk, nsys - s0);
    ch.zero_start = opts->zero_start;
    ch.prm = OsParams{opts->lambda, opts->max_iter, opts->tol, opts->nonneg,
                      opts->residual_every > 0 ? opts->residual_every : 1};
    for (int i = 0; i < ch.count; ++i) ch.d[i] = ds[s0 + i];
    k_os_setup<<<ch.count, kOsThreads, 0, st>>>(ch, reinterpret_cast<OsDesc*>(ws + L.table),
                                                  reinterpret_cast<OsParams*>(ws + L.params));
  }
  if (nsys > 1)
    k_os_blk2sys<<<nsys, 256, 0, st>>>(reinterpret_cast<const OsDesc*>(ws + L.table),
                                       reinterpret_cast<int32_t*>(ws + L.b2s[0]),
                                       reinterpret_cast<int32_t*>(ws + L.b2s[1]),
                                       reinterpret_cast<int32_t*>(ws + L.b2s[2]));
  SS_HIP_TRY(hipGetLastError());
  // max_iter passes and the residual of the final image: max_iter + 1 groups
  const int64_t total = static_cast<int64_t>(opts->max_iter) + 1;
  const int chunk = opts->tol > 0.0 ? static_cast<int>(std::min<int64_t>(opts->check_every, total))
                                    : static_cast<int>(std::min<int64_t>(total, 32));
  GraphEntry* graph = nullptr;
  if (opts->use_graph) {
    int dev = 0;
    SS_HIP_TRY(hipGetDevice(&dev));
    const OsKey key{dev, workspace, nsys, S, g.nb[0], g.nb[1], g.nb[2], c.rpw, c.cpw, c.xcd, c.u, c.ch, chunk};
    auto capture = [&](hipStream_t cs) { os_passes(c, ws, L, nsys, S, g, chunk, cs); };
    if (ss_status s = os_graphs().acquire(key, dev, capture, &graph)) return s;
  }
  std::vector<OsState> hs(nsys);
  auto read_states = [&]() -> ss_status {
    SS_HIP_TRY(hipMemcpyAsync(hs.data(), ws + L.states, sizeof(OsState) * nsys, hipMemcpyDeviceToHost, st));
    SS_HIP_TRY(hipStreamSynchronize(st));
    return SS_OK;
  };
  ss_status loop = SS_OK;
  for (int64_t done = 0; done < total && loop == SS_OK; done += chunk) {
    if (graph) {
      const hipError_t e = hipGraphLaunch(graph->exec, st);
      if (e != hipSuccess) loop = fail(SS_E_HIP, "hipGraphLaunch failed: %s", hipGetErrorString(e));
    } else {
      os_passes(c, ws, L, nsys, S, g, static_cast<int>(std::min<int64_t>(chunk, total - done)), st);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) loop = fail(SS_E_HIP, "ordered-subset launch failed: %s", hipGetErrorString(e));
    }
    if (loop == SS_OK && opts->tol > 0.0 && done + chunk < total) {
      loop = read_states();
      bool all = true;
      for (const auto& x : hs) all = all && x.stop;
      if (loop == SS_OK && all) break;
    }
  }
  if (graph) os_graphs().release(graph, st);
  if (loop != SS_OK) return loop;
  if (!passes && opts->tol <= 0.0) return SS_OK;
  if (ss_status s = read_states()) return s;
  ss_status result = SS_OK;
  for (int s = 0; s < nsys; ++s) {
    if (passes) passes[s] = hs[s].k;
    if (opts->tol > 0.0 && !(hs[s].last_res <= opts->tol)) result = SS_NOT_CONVERGED;
  }
  return result;
}
