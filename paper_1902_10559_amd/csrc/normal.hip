// The direct path (Theorem 2): the normal equations A(k)^T A(k) f(k) =
// A(k)^T p(k) of each half of the folded pair, solved by a Cholesky
// factorisation in FP64, and the halves recombined by eq. (5); for a single
// system (nvals = 1) the same solve on A itself.  The split turns one
// N x N factorisation into two of N/2 x N/2: 1/4 of the flops (the paper's
// 2^(alpha+beta) argument after Theorem 1, alpha + beta = 3 here), while
// forming B from the sparse rows costs about the same either way.
//
// Both halves go through the same launches (blockIdx.z selects the half).
// Steps per half: B = A^T A, lower triangle, and c = A^T p from the sparse
// rows (row-wise sums over the rays through each voxel, in shared memory);
// right-looking blocked Cholesky of B in place (64 x 64 diagonal blocks
// factored in registers, their inverses formed on the FP64 matrix cores,
// panel solves, trailing updates by an FP64 matrix-core GEMM,
// v_mfma_f64_16x16x4f64), the forward substitution riding on the
// factorisation's diagonal blocks and panel solves; back substitution, block
// by block.
// The whole solve is replayed from a captured graph.

#include <algorithm>
#include <cmath>
#include <mutex>
#include <tuple>
#include <vector>

#include "device.h"
#include "graph_cache.h"
#include "internal.h"

namespace ss {
namespace {

constexpr int kNb = 64;      // Cholesky block and GEMM tile
constexpr int kPanel = 256;  // columns per trailing update
constexpr int kTrail = 128;      // tile of the trailing update
constexpr int kTrailWaves = 8;   // wavefronts per trailing-update block
constexpr int64_t kNearSmall = 4096;  // rows below which trailing updates take 64 x 64 tiles

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Row j of B(h) = A(h)^T A(h) on and below the diagonal, and c[j] =
// (A(h)^T p(h))[j].  One block per row: B[j, c] is the sum over the rays i
// that cross voxel j (column j of the CSC, ascending i) of a_ij a_ic, from
// ray i's CSR row.  The columns 0..j are accumulated in shared memory,
// kFormCols at a time; within one ray a column occurs once, and a barrier
// separates rays, so every sum runs in ascending ray order (the result is
// the same from run to run).  The rays' row ranges and a_ij are staged in
// shared memory kFormRays at a time, and each thread's first entries of the
// next rays are in flight while the current ray is added.  Products of FP32
// values are exact in FP64.  The system's descriptor is read from device
// memory (a replayed solve reads the system of the current call).
constexpr int kFormCols = 4096;  // columns per pass: 39 KB of shared memory, four blocks per CU
constexpr int kFormRays = 256;
constexpr int kFormAhead = 4;  // rays whose entries are loaded ahead
constexpr int kFormThreads = 256;

__global__ __launch_bounds__(kFormThreads) void k_form_b(const ss_system* sysp, double* B, int64_t bs, double* c,
                                                         int64_t vs) {
  const ss_system sys = *sysp;
  __shared__ double acc[kFormCols];
  __shared__ int64_t rs[kFormRays];
  __shared__ int32_t rl[kFormRays];
  __shared__ double ra[kFormRays], rp[kFormRays];
  const int tid = threadIdx.x;
  const int64_t j = blockIdx.x;
  const int h = blockIdx.z;  // the half: A(1) or A(2)
  B += h * bs;
  c += h * vs;
  const int64_t n = sys.n;
  const int nv = sys.nvals;
  const float* vt = static_cast<const float*>(sys.val_t);
  const float* v = static_cast<const float*>(sys.val);
  const int64_t e0 = sys.col_ptr[j], e1 = sys.col_ptr[j + 1];
  double cj = 0.0;  // the first wavefront
  for (int64_t c0 = 0; c0 <= j; c0 += kFormCols) {
    const int w = static_cast<int>(std::min<int64_t>(kFormCols, j + 1 - c0));
    for (int t = tid; t < w; t += kFormThreads) acc[t] = 0.0;
    for (int64_t eb = e0; eb < e1; eb += kFormRays) {
      const int nr = static_cast<int>(std::min<int64_t>(kFormRays, e1 - eb));
      __syncthreads();
      for (int t = tid; t < nr; t += kFormThreads) {
        const int64_t i = sys.row_idx[eb + t];
        const int64_t b0 = sys.row_ptr[i];
        rs[t] = b0;
        rl[t] = static_cast<int32_t>(sys.row_ptr[i + 1] - b0);
        ra[t] = static_cast<double>(vt[nv * (eb + t) + h]);
        rp[t] = static_cast<double>(sys.p[nv * i + h]);
      }
      __syncthreads();
      // c[j]: the first wavefront sums the batch's a_ij p_i, lane l taking
      // rays l, l + 64, ... in order, then a butterfly across the lanes (a
      // fixed order; partners add the same two values, so every lane holds
      // the same sum) -- not one thread's serial loop, which the other
      // wavefronts would wait for at the first barrier
      if (c0 == 0 && tid < kWave) {
        double s = 0.0;
        for (int t = tid; t < nr; t += kWave) s += ra[t] * rp[t];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
        cj += s;
      }
      // Entry tid of ray r is loaded kFormAhead rays ahead, into a ring of
      // registers, raw (a position past the ray's end reads its first
      // entry, which every ray through voxel j has; the value is dropped at
      // use): the loads of the next rays are in flight while the current
      // one is added, and nothing waits on them before their turn.
      int32_t cq[kFormAhead];
      float vq[kFormAhead];
      auto fetch = [&](int r, int d) {
        const int rr = r < nr ? r : nr - 1;
        const int64_t e = rs[rr] + (tid < rl[rr] ? tid : 0);
        cq[d] = sys.col_idx[e];
        vq[d] = v[nv * e + h];
      };
      // issued in slot order, as in the loop (the loads complete in order,
      // and the loop waits for slot d with the later slots still in flight)
#pragma unroll
      for (int d = 0; d < kFormAhead; ++d) {
        fetch(d, d);
        __builtin_amdgcn_sched_barrier(0);
      }
      for (int r0 = 0; r0 < nr; r0 += kFormAhead) {
#pragma unroll
        for (int d = 0; d < kFormAhead; ++d) {
          // a group runs whole (a ray past the batch adds nothing), so that
          // no exit in the middle makes the ring's registers be copied
          const int r = r0 + d < nr ? r0 + d : nr - 1;
          const double a = ra[r];
          const int64_t b0 = rs[r];
          const int len = r0 + d < nr ? rl[r] : 0;
          const int64_t cur_col = cq[d];
          if (tid < len && cur_col >= c0 && cur_col < c0 + w) acc[cur_col - c0] += a * static_cast<double>(vq[d]);
          // refilled once read, so the slot keeps its registers
          fetch(r0 + d + kFormAhead, d);
          for (int k = tid + kFormThreads; k < len; k += kFormThreads) {
            const int64_t cc = sys.col_idx[b0 + k];
            if (cc >= c0 && cc < c0 + w) acc[cc - c0] += a * static_cast<double>(v[nv * (b0 + k) + h]);
          }
          __syncthreads();
        }
      }
    }
    for (int t = tid; t < w; t += kFormThreads) B[j * n + c0 + t] = acc[t];
  }
  if (tid == 0) c[j] = cj;
}

// C[i, j] = beta * C[i, j] + alpha * sum_k X[i, k] Y[j, k] over an nr x nc
// region of C, one TM x TM tile per block of NW wavefronts (2 x NW/2, each
// TM/2 x 2TM/NW as matrix-core tiles of 16 x 16); blockIdx.x is the tile
// row, blockIdx.y the tile column.  With `lower`, tiles above the diagonal of the
// region are skipped and elements above it are left alone.  X (nr rows), Y
// (nc rows) and C are row-major with leading dimensions ldx, ldy, ldc; K
// terms.  C may be X itself when nc <= TM (one tile column): a block reads
// all of its X rows before it writes them.  K is staged through shared
// memory kKc columns at a time, k-major, in two buffers: the next chunk's
// global loads are in flight while the current one is multiplied.
// Operand layouts of v_mfma_f64_16x16x4f64 for lane l (g = l / 16):
//   A[m][k]: m = l % 16, k = g;  B[k][n]: n = l % 16, k = g;
//   D[m][n]: m = g + 4 r (r = 0..3, the accumulator's element), n = l % 16
// (rows interleaved by 4, unlike the 4 consecutive rows of the FP32 forms).
constexpr int kKc = 16;
template <int TM, int NW, bool HI = false>
__global__ __launch_bounds__(NW * 64) void k_gemm_nt(const double* X, int64_t ldx, const double* Y, int64_t ldy,
                                                 double* C, int64_t ldc, int64_t nr, int64_t nc, int64_t K,
                                                 double alpha, double beta, int lower, int64_t xs_, int64_t ys_,
                                                 int64_t cs_) {
  // HI: a launch on the factorisation's chain, whose waves share compute
  // units with the concurrent far update's: they win instruction issue
  if constexpr (HI) __builtin_amdgcn_s_setprio(3);
  constexpr int NT = NW * 64;                 // threads
  constexpr int WM = TM / 2, WN = 2 * TM / NW;  // this wave's sub-tile
  constexpr int MR = WM / 16, MC = WN / 16;   // 16 x 16 tiles per wave
  constexpr int PER = TM * kKc / NT / 2;      // double pairs staged per thread per operand
  constexpr int LDS_LD = TM + 1;
  static_assert(PER >= 1 && MR >= 1 && MC >= 1, "tile shape");
  const int64_t ti = blockIdx.x, tj = blockIdx.y;
  if (lower && tj > ti) return;
  X += blockIdx.z * xs_;  // the half
  Y += blockIdx.z * ys_;
  C += blockIdx.z * cs_;
  const int64_t r0 = ti * TM, c0 = tj * TM;
  __shared__ double xs[2][kKc][LDS_LD];
  __shared__ double ys[2][kKc][LDS_LD];
  const int lane = lane_id(), w = wave_id();
  const int wr = (w / (NW / 2)) * WM, wc = (w % (NW / 2)) * WN;
  const int g = lane / 16, l16 = lane % 16;
  f64x4 acc[MR][MC];
#pragma unroll
  for (int a = 0; a < MR; ++a)
#pragma unroll
    for (int q = 0; q < MC; ++q) acc[a][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  // staging: pair p of thread tid is row (tid + NT p) / (kKc/2), columns 2 ((tid + NT p) % (kKc/2)) + {0, 1}
  double2 xr[PER], yr[PER];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + NT * p;
      const int rr = e / (kKc / 2), kk = 2 * (e % (kKc / 2));
      const int64_t k = k0 + kk;
      const int64_t xi = r0 + rr, yi = c0 + rr;
      // two 8-byte loads: a row start need not be 16-byte aligned
      double2 vx = {0.0, 0.0}, vy = {0.0, 0.0};
      if (xi < nr) {
        if (k < K) vx.x = X[xi * ldx + k];
        if (k + 1 < K) vx.y = X[xi * ldx + k + 1];
      }
      if (yi < nc) {
        if (k < K) vy.x = Y[yi * ldy + k];
        if (k + 1 < K) vy.y = Y[yi * ldy + k + 1];
      }
      xr[p] = vx;
      yr[p] = vy;
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + NT * p;
      const int rr = e / (kKc / 2), kk = 2 * (e % (kKc / 2));
      xs[b][kk][rr] = xr[p].x;
      xs[b][kk + 1][rr] = xr[p].y;
      ys[b][kk][rr] = yr[p].x;
      ys[b][kk + 1][rr] = yr[p].y;
    }
  };
  // on the chain (HI) with the 64 x 64 tiles, C's values are loaded first,
  // so that the epilogue does not wait for them after the products (with
  // the 128 x 128 tiles the registers this holds cost more than it gains)
  constexpr bool kPre = HI && TM == 64;
  double cold[MR][MC][4];
  if constexpr (kPre) {
    if (beta != 0.0) {
#pragma unroll
      for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int q = 0; q < MC; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i = r0 + wr + 16 * a + g + 4 * r;
            const int64_t j = c0 + wc + 16 * q + l16;
            cold[a][q][r] = (i < nr && j < nc && (!lower || j <= i)) ? C[i * ldc + j] : 0.0;
          }
    }
  }
  const int64_t nch = (K + kKc - 1) / kKc;
  load(0);
  store(0);
  __syncthreads();
  for (int64_t ch = 0; ch < nch; ++ch) {
    const int b = static_cast<int>(ch & 1);
    if (ch + 1 < nch) load((ch + 1) * kKc);
#pragma unroll
    for (int kk = 0; kk < kKc; kk += 4) {
      double av[MR], bv[MC];
#pragma unroll
      for (int a = 0; a < MR; ++a) av[a] = xs[b][kk + g][wr + 16 * a + l16];
#pragma unroll
      for (int q = 0; q < MC; ++q) bv[q] = ys[b][kk + g][wc + 16 * q + l16];
#pragma unroll
      for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int q = 0; q < MC; ++q) acc[a][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[q], acc[a][q], 0, 0, 0);
    }
    if (ch + 1 < nch) store(b ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < MR; ++a)
#pragma unroll
    for (int q = 0; q < MC; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = r0 + wr + 16 * a + g + 4 * r;
        const int64_t j = c0 + wc + 16 * q + l16;
        if (i < nr && j < nc && (!lower || j <= i)) {
          double* cp = C + i * ldc + j;
          double cv0 = 0.0;
          if (beta != 0.0) {
            if constexpr (kPre) cv0 = cold[a][q][r];
            else cv0 = *cp;
          }
          *cp = (beta == 0.0 ? 0.0 : beta * cv0) + alpha * acc[a][q][r];
        }
      }
}

// The chain's small products (K <= 64: the panel solve, times L_kk^{-T}, and
// the in-panel update): C = beta C + alpha X Y^T on 64 x 64 tiles by four
// wavefronts (a 32 x 32 quarter each, 2 x 2 matrix-core tiles), with all K
// columns of the tile's X and Y rows loaded at once and staged k-major in
// shared memory behind one barrier -- one memory latency per launch where
// k_gemm_nt's chunks of kKc take K / kKc of them in sequence.  Same
// arguments and conventions as k_gemm_nt (C may be X itself: every X load
// precedes the barrier, every C store follows it).
template <bool HI>
__global__ __launch_bounds__(256) void k_gemm_nt_k64(const double* X, int64_t ldx, const double* Y, int64_t ldy,
                                                    double* C, int64_t ldc, int64_t nr, int64_t nc, int64_t K,
                                                    double alpha, double beta, int lower, int64_t xs_, int64_t ys_,
                                                    int64_t cs_, const double* yv, double* cv, int64_t vs_) {
  if constexpr (HI) __builtin_amdgcn_s_setprio(3);
  constexpr int TM = kNb, NT = 256, PER = TM * TM / NT, LD = TM + 1;
  const int64_t ti = blockIdx.x, tj = blockIdx.y;
  if (lower && tj > ti) return;
  X += blockIdx.z * xs_;  // the half
  Y += blockIdx.z * ys_;
  C += blockIdx.z * cs_;
  const int64_t r0 = ti * TM, c0 = tj * TM;
  __shared__ double xs[TM * LD], ys[TM * LD];  // [k][row]
  __shared__ double ysub[TM], red[2][TM];
  double cval = 0.0;
  if (cv) {  // the forward substitution's update rides on the panel solve
    yv += blockIdx.z * vs_;
    cv += blockIdx.z * vs_;
    if (threadIdx.x < TM) ysub[threadIdx.x] = yv[threadIdx.x];
    if (threadIdx.x < TM && r0 + threadIdx.x < nr) cval = cv[r0 + threadIdx.x];  // read early, written last
  }
  const int lane = lane_id(), w = wave_id(), g = lane / 16, l16 = lane % 16;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  // element e = tid + NT p: row e / TM, column k = e % TM (a row's K
  // columns are read by consecutive threads)
  double vx[PER], vy[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + NT * p, rr = e / TM, k = e % TM;
    const int64_t xi = r0 + rr, yi = c0 + rr;
    vx[p] = (xi < nr && k < K) ? X[xi * ldx + k] : 0.0;
    vy[p] = (yi < nc && k < K) ? Y[yi * ldy + k] : 0.0;
  }
  // C's values too, where they are read (beta != 0): their loads are in
  // flight with the operands' instead of after the products
  double cold[2][2][4];
  if (beta != 0.0) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = r0 + wr + 16 * a + g + 4 * r;
          const int64_t j = c0 + wc + 16 * q + l16;
          cold[a][q][r] = (i < nr && j < nc && (!lower || j <= i)) ? C[i * ldc + j] : 0.0;
        }
  }
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + NT * p, rr = e / TM, k = e % TM;
    xs[k * LD + rr] = vx[p];
    ys[k * LD + rr] = vy[p];
  }
  __syncthreads();
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[a][q] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < TM; kk += 4) {
    double av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = xs[(kk + g) * LD + wr + 16 * a + l16];
#pragma unroll
    for (int q = 0; q < 2; ++q) bv[q] = ys[(kk + g) * LD + wc + 16 * q + l16];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[a][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[q], acc[a][q], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = r0 + wr + 16 * a + g + 4 * r;
        const int64_t j = c0 + wc + 16 * q + l16;
        if (i < nr && j < nc && (!lower || j <= i))
          C[i * ldc + j] = (beta == 0.0 ? 0.0 : beta * cold[a][q][r]) + alpha * acc[a][q][r];
      }
  // with cv (the panel solve, C = X Y^T = the new rows of L's column block
  // k): c[i] -= sum_j L[i][j] y_k[j] for the tile's rows, a lane's 2 x 16
  // columns, then the 16 lanes of a row, then the two column halves
  if (cv) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = acc[a][0][r] * ysub[wc + l16] + acc[a][1][r] * ysub[wc + 16 + l16];
        v += __shfl_xor(v, 1, kWave);
        v += __shfl_xor(v, 2, kWave);
        v += __shfl_xor(v, 4, kWave);
        v += __shfl_xor(v, 8, kWave);
        if (l16 == 0) red[w & 1][wr + 16 * a + g + 4 * r] = v;
      }
    __syncthreads();
    if (threadIdx.x < TM && r0 + threadIdx.x < nr) cv[r0 + threadIdx.x] = cval - (red[0][threadIdx.x] + red[1][threadIdx.x]);
  }
}

// Cholesky of the diagonal block B[k0.., k0..] (size nb <= 64), padded to
// 64 with the identity, and the inverse of its factor, by kDiagWaves
// wavefronts.  The factorisation: thread (t, q) (q = wavefront) holds
// columns kSeg q .. kSeg q + kSeg - 1 of row t of the block in registers.
// Step j, one barrier: the owners of column j put its entries below the
// diagonal in shared memory (zeros on and above it) and the pivot d in a
// slot of its own; then every thread forms sc = B[t][j] / d (a reciprocal
// estimate refined by one Newton step), which is zero for t <= j, and
// subtracts sc B[c][j] from each of its entries -- no masks on this chain
// of 64 dependent steps -- and the owners turn column j into L's
// (B[t][j] / sqrt(d), from the reciprocal-square-root estimate and one
// Newton step).  The inverse X = L^{-1} then comes from L in shared memory,
// not from updates inside the chain (which doubled each step's work): the
// four 16 x 16 diagonal blocks by forward substitution, one wavefront each
// (lane = column, 1 / L_ii from the chain's 1/sqrt(d)), then two levels of
// inv([A 0; C D]) = [X_A 0; -X_D C X_A  X_D] on the FP64 matrix cores
// (16 x 16 blocks, then 32 x 32).  L goes back to B (lower part, nb x nb),
// L^{-1} to Linv (64 x 64 row-major, zero above the diagonal).  A
// non-positive pivot sets *flag and is replaced by 1 so that the rest stays
// finite.
constexpr int kDiagWaves = 8;
constexpr int kSeg = kNb / kDiagWaves;
constexpr int kDiagLd = kNb + 1;  // padded rows of L and X in shared memory
constexpr int kDiagTd = 33;       // padded rows of the 32 x 32 product
__global__ __launch_bounds__(64 * kDiagWaves) void k_potrf_diag(double* B, int64_t ld, int64_t k0, int nb,
                                                               double* Linv, int32_t* flag, int64_t bs,
                                                               int64_t ls, const double* c, double* y, int64_t vs) {
  __builtin_amdgcn_s_setprio(3);  // on the chain: wins issue over the far update's waves
  __shared__ double colj[2][kNb], dj[2], ipj[kNb], cv[kNb];
  __shared__ double Ls[kNb * kDiagLd], Xs[kNb * kDiagLd], Ts[32 * kDiagTd];
  const int t = lane_id(), q = wave_id();
  B += blockIdx.z * bs;  // the half
  Linv += blockIdx.z * ls;
  c += blockIdx.z * vs;
  y += blockIdx.z * vs;
  // c_k, final here: every earlier block's panel solve has updated it
  if (threadIdx.x < kNb) cv[threadIdx.x] = threadIdx.x < static_cast<unsigned>(nb) ? c[k0 + threadIdx.x] : 0.0;
  double row[kSeg];
#pragma unroll
  for (int cc = 0; cc < kSeg; ++cc) {
    const int c = kSeg * q + cc;
    row[cc] = (t < nb && c <= t) ? B[(k0 + t) * ld + k0 + c] : (c == t ? 1.0 : 0.0);
  }
  bool bad = false;
  for (int s = 0; s < kNb / kSeg; ++s) {
#pragma unroll
    for (int jj = 0; jj < kSeg; ++jj) {
      const int j = kSeg * s + jj, b = jj & 1;
      if (q == s) {
        colj[b][t] = (t > j) ? row[jj] : 0.0;
        if (t == j) dj[b] = row[jj];
      }
      __syncthreads();
      double d = dj[b];
      if (!(d > 0.0)) {
        bad = true;
        d = 1.0;
      }
      double rd = __builtin_amdgcn_rcp(d);
      rd = __builtin_fma(__builtin_fma(-d, rd, 1.0), rd, rd);
      const double ct = colj[b][t];
      const double sc = ct * rd;  // zero for t <= j
      double ip = __builtin_amdgcn_rsq(d);
      ip = ip * (1.5 - 0.5 * d * ip * ip);
      if (q == s) {
        row[jj] = (t > j) ? ct * ip : (t == j ? d * ip : 0.0);
        if (t == j) ipj[j] = ip;
      }
#pragma unroll
      for (int cc = 0; cc < kSeg; ++cc) row[cc] -= sc * colj[b][kSeg * q + cc];
    }
  }
  if (bad && t == 0 && q == 0) *flag = 1;
  // entries above the diagonal took updates along the way: only c <= t is L
#pragma unroll
  for (int cc = 0; cc < kSeg; ++cc) {
    const int c = kSeg * q + cc;
    if (t < nb && c <= t) B[(k0 + t) * ld + k0 + c] = row[cc];
    Ls[t * kDiagLd + c] = (c <= t) ? row[cc] : 0.0;
  }
  __syncthreads();
  const int l16 = t & 15, g = t >> 4;
  if (q < 4) {  // diagonal block q: lane l16 solves for column l16
    const int o = 16 * q;
    double x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      double a = (r == l16) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < r; ++k) a -= Ls[(o + r) * kDiagLd + o + k] * x[k];
      x[r] = a * ipj[o + r];
    }
    if (t < 16)
#pragma unroll
      for (int r = 0; r < 16; ++r) Xs[(o + r) * kDiagLd + o + l16] = x[r];
  }
  __syncthreads();
  // 16 x 16 blocks (I, J) = (2q+1, 2q): X_IJ = -X_II (L_IJ X_JJ); the first
  // product's accumulator element r holds rows 4r + g, which is the second
  // product's k-chunk r as its B operand
  if (q < 2) {
    const int I = 2 * q + 1, J = 2 * q;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ls[(16 * I + l16) * kDiagLd + 16 * J + 4 * kc + g],
                                                 Xs[(16 * J + 4 * kc + g) * kDiagLd + 16 * J + l16], acc, 0, 0, 0);
    f64x4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 4; ++r)
      x = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[(16 * I + l16) * kDiagLd + 16 * I + 4 * r + g], acc[r], x, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) Xs[(16 * I + 4 * r + g) * kDiagLd + 16 * J + l16] = -x[r];
  }
  __syncthreads();
  // 32 x 32 level: T = C X_A (C = L[32:64, 0:32]), tile (I2, J2) per wavefront
  const int I2 = 2 + (q >> 1), J2 = q & 1;
  if (q < 4) {
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int K = J2; K < 2; ++K)
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ls[(16 * I2 + l16) * kDiagLd + 16 * K + 4 * kc + g],
                                                   Xs[(16 * K + 4 * kc + g) * kDiagLd + 16 * J2 + l16], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) Ts[(16 * (I2 - 2) + 4 * r + g) * kDiagTd + 16 * J2 + l16] = acc[r];
  }
  __syncthreads();
  // X[I2][J2] = -sum over K = 2 .. I2 of X_D[I2][K] T[K][J2]
  if (q < 4) {
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int K = 2; K <= I2; ++K)
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[(16 * I2 + l16) * kDiagLd + 16 * K + 4 * kc + g],
                                                   Ts[(16 * (K - 2) + 4 * kc + g) * kDiagTd + 16 * J2 + l16], acc,
                                                   0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) Xs[(16 * I2 + 4 * r + g) * kDiagLd + 16 * J2 + l16] = -acc[r];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kNb * kNb; e += 64 * kDiagWaves) {
    const int i = e / kNb, cc = e % kNb;
    Linv[e] = (cc <= i) ? Xs[i * kDiagLd + cc] : 0.0;
  }
  // the forward substitution's block: y_k = L_kk^{-1} c_k, thread (row,
  // part) summing 8 columns, the 8 parts added across adjacent lanes in a
  // fixed order
  {
    const int r = threadIdx.x / 8, part = threadIdx.x % 8;
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int cc = 8 * part + u;  // Xs above the diagonal blocks was never written
      if (cc <= r) a += Xs[r * kDiagLd + cc] * cv[cc];
    }
    a += __shfl_xor(a, 1, kWave);
    a += __shfl_xor(a, 2, kWave);
    a += __shfl_xor(a, 4, kWave);
    if (part == 0 && r < nb) y[k0 + r] = a;
  }
}

// Back substitution's first block: x_k = L_kk^{-T} y_k for the last block
// (the four wavefronts' partial sums added in wavefront order).  The forward
// substitution L y = c has no kernels of its own: each diagonal block's
// kernel forms y_k = L_kk^{-1} c_k, and each panel solve subtracts
// L[rows below, k] y_k from c.
__global__ __launch_bounds__(256) void k_diag_bwd(const double* Linv, const double* y, double* x, int64_t k0, int nb,
                                                  int64_t ls, int64_t vs) {
  __shared__ double part[4][kNb];
  Linv += blockIdx.z * ls;  // the half
  y += blockIdx.z * vs;
  x += blockIdx.z * vs;
  const int t = lane_id(), w = wave_id();
  double a = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int q = 16 * w + u;
    a += Linv[q * kNb + t] * (q < nb ? y[k0 + q] : 0.0);
  }
  part[w][t] = a;
  __syncthreads();
  if (threadIdx.x < kNb && t < nb) x[k0 + t] = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
}

// Back substitution, block k of L^T x = y (from the last block; k >= 1):
// with x_k already formed, y[i] -= sum_t L[k0+t, i] x_k[t] for this block's
// 64 rows i < k0 (wavefront w takes t = 16w .. 16w+15, lanes run along i;
// the four partial sums added in wavefront order).  The last block's rows
// are block k-1's: it then forms x_{k-1} = L^{-T}_{k-1,k-1} y_{k-1}.
__global__ __launch_bounds__(256) void k_bwd_step(const double* L, int64_t ld, int64_t n, int64_t k0, int nb,
                                                  const double* Linv_prev, double* y, double* x, int64_t bs,
                                                  int64_t ls, int64_t vs) {
  __shared__ double xk[kNb], yn[kNb];
  __shared__ double part[4][kNb];
  const int tid = threadIdx.x;
  L += blockIdx.z * bs;  // the half
  Linv_prev += blockIdx.z * ls;
  y += blockIdx.z * vs;
  x += blockIdx.z * vs;
  if (tid < kNb) xk[tid] = tid < nb ? x[k0 + tid] : 0.0;
  const int w = wave_id();
  // the last block's inverse entries, loaded before they are needed (they
  // do not depend on this step's results)
  const bool last = blockIdx.x + 1 == gridDim.x;
  double lv[16];
  if (last) {
#pragma unroll
    for (int u = 0; u < 16; ++u) lv[u] = Linv_prev[(16 * w + u) * kNb + lane_id()];
  }
  // this block's L entries and y values too: in flight with x_k's loads,
  // before the barrier
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNb + lane_id();  // < k0: the grid covers k0 rows
  const double yold = tid < kNb ? y[i] : 0.0;
  double lk[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int64_t row = std::min<int64_t>(k0 + 16 * w + u, n - 1);  // past n: x_k is 0 there
    lk[u] = L[row * ld + i];
  }
  __syncthreads();
  double a = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) a += lk[u] * xk[16 * w + u];
  part[w][lane_id()] = a;
  __syncthreads();
  double ynew = 0.0;
  if (tid < kNb) {
    ynew = yold - (((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid]);
    y[i] = ynew;
  }
  if (!last) return;
  if (tid < kNb) yn[tid] = ynew;
  __syncthreads();
  const int t = lane_id();
  double b = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) b += lv[u] * yn[16 * w + u];
  part[w][t] = b;
  __syncthreads();
  if (tid < kNb) x[k0 - kNb + t] = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
}

// f[j] = (f2 + f1) / 2, f[N-1-j] = (f2 - f1) / 2 (eq. (5)), or a copy for
// a single system.
// Clears the factorisation's failure flag (a kernel, not a memset, so
// that the solve's graph holds kernels only).
__global__ void k_clear_flag(int32_t* flag) {
  if (threadIdx.x == 0) *flag = 0;
}

__global__ void k_recombine_f64(const double* h1, const double* h2, int64_t n, int nv, double* f) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (nv == 1) {
    f[j] = h1[j];
  } else {
    f[j] = 0.5 * (h2[j] + h1[j]);
    f[2 * n - 1 - j] = 0.5 * (h2[j] - h1[j]);
  }
}

// Per half h (blockIdx.z of every launch): B at b + h*bs, c, y, x at
// c/y/x + h*vs, the inverted diagonal blocks at linv + h*ls (in doubles).
struct NormalLayout {
  size_t b, c, y, x, linv, flag, sysc, total;
  int64_t bs, vs, ls;
};

inline size_t al(size_t v) { return (v + 255) & ~size_t{255}; }

NormalLayout normal_layout(const ss_system* sys) {
  const size_t n = static_cast<size_t>(sys->n), nv = static_cast<size_t>(sys->nvals);
  const size_t nt = (n + kNb - 1) / kNb;
  NormalLayout L;
  L.bs = static_cast<int64_t>(al(sizeof(double) * n * n) / sizeof(double));
  L.vs = static_cast<int64_t>(al(sizeof(double) * n) / sizeof(double));
  L.ls = static_cast<int64_t>(nt * kNb * kNb);
  size_t o = 0;
  L.b = o;
  o += sizeof(double) * static_cast<size_t>(L.bs) * nv;
  L.c = o;
  o += sizeof(double) * static_cast<size_t>(L.vs) * nv;
  L.y = o;
  o += sizeof(double) * static_cast<size_t>(L.vs) * nv;
  L.x = o;
  o += sizeof(double) * static_cast<size_t>(L.vs) * 2;  // two halves even for nvals = 1 (the second unused)
  L.linv = o;
  o += al(sizeof(double) * static_cast<size_t>(L.ls) * nv);
  L.flag = o;
  o += 256;
  L.sysc = o;  // a copy of the system's descriptor, read by the formation
  o += al(sizeof(ss_system));
  L.total = o;
  return L;
}

ss_status check_normal(const ss_system* sys, const char* fn) {
  if (!sys) return fail(SS_E_ARG, "%s: NULL system", fn);
  if (sys->wdtype != SS_F32 || (sys->nvals != 1 && sys->nvals != 2))
    return fail(SS_E_ARG, "%s: an FP32 system with nvals 1 or 2 is required", fn);
  if (ss_status e = check_ascending(sys, fn)) return e;
  if (sys->m <= 0 || sys->n <= 0 || sys->nnz < 0 || !sys->col_ptr || !sys->p ||
      (sys->nnz > 0 && (!sys->row_idx || !sys->val_t)))
    return fail(SS_E_ARG, "%s: bad system", fn);
  if (sys->n > (int64_t{1} << 17) || sys->m > (int64_t{1} << 30))
    return fail(SS_E_ARG, "%s: system too large for the dense path", fn);
  return SS_OK;
}

inline unsigned blocks(int64_t count, int per) { return static_cast<unsigned>((count + per - 1) / per); }

// The factorisation's second stream and its events, one set per device,
// created on first use and kept for the process.  A call holds its
// device's lock from start to end, so calls that overlap on one device run
// one after the other.
struct Lookahead {
  hipStream_t side = nullptr;
  std::vector<hipEvent_t> ev;
  std::mutex mu;
};
constexpr int kMaxDevices = 64;
Lookahead g_lookahead[kMaxDevices];

ss_status lookahead_resources(Lookahead& la, size_t events) {
  if (!la.side) SS_HIP_TRY(hipStreamCreateWithFlags(&la.side, hipStreamNonBlocking));
  while (la.ev.size() < events) {
    hipEvent_t e;
    SS_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    la.ev.push_back(e);
  }
  return SS_OK;
}

// Graphs of whole solves, one per device, workspace, image and shape.
struct NormalKey {
  int device;
  const void* ws;
  const double* f;
  int64_t n;
  int nvals;
  bool operator<(const NormalKey& o) const {
    return std::tie(device, ws, f, n, nvals) < std::tie(o.device, o.ws, o.f, o.n, o.nvals);
  }
};

GraphCache<NormalKey>& normal_graphs() {
  static auto* c = new GraphCache<NormalKey>(16);  // lives until process exit
  return *c;
}

}  // namespace
}  // namespace ss

using namespace ss;

extern "C" ss_status ss_normal_workspace_bytes(const ss_system* sys, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(SS_E_ARG, "ss_normal_workspace_bytes: NULL bytes");
  if (ss_status s = check_normal(sys, "ss_normal_workspace_bytes")) return s;
  *bytes = normal_layout(sys).total;
  return SS_OK;
}

extern "C" ss_status ss_normal_solve(const ss_system* sys, double* f, void* workspace, size_t workspace_bytes,
                                     void* stream) {
  clear_error();
  if (ss_status s = check_normal(sys, "ss_normal_solve")) return s;
  if (!f || !workspace) return fail(SS_E_ARG, "ss_normal_solve: NULL image or workspace");
  const NormalLayout L = normal_layout(sys);
  if (workspace_bytes < L.total) return fail(SS_E_WORKSPACE, "ss_normal_solve: workspace needs %zu bytes", L.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  double* B = reinterpret_cast<double*>(ws + L.b);
  int32_t* flag = reinterpret_cast<int32_t*>(ws + L.flag);
  const int64_t n = sys->n;
  const int64_t nt = (n + kNb - 1) / kNb;
  const unsigned nv = static_cast<unsigned>(sys->nvals);
  double* c = reinterpret_cast<double*>(ws + L.c);
  double* y = reinterpret_cast<double*>(ws + L.y);
  double* x = reinterpret_cast<double*>(ws + L.x);
  double* Linv = reinterpret_cast<double*>(ws + L.linv);
  const int64_t bs = L.bs, vs = L.vs, ls = L.ls;
  auto tiles = [](int64_t v, int t) { return static_cast<unsigned>((v + t - 1) / t); };
  int dev = 0;
  SS_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SS_E_ARG, "ss_normal_solve: device %d out of range", dev);
  Lookahead& la = g_lookahead[dev];
  std::lock_guard<std::mutex> lock(la.mu);
  const int64_t npanel = (n + kPanel - 1) / kPanel;
  if (ss_status s = lookahead_resources(la, static_cast<size_t>(2 * npanel + 1))) return s;
  hipEvent_t* evF = la.ev.data();              // panel p factored
  hipEvent_t* evU = la.ev.data() + npanel;     // panel p's far trailing update done
  hipEvent_t evFork = la.ev[static_cast<size_t>(2 * npanel)];
  hipStream_t sb = la.side;

  // The whole solve (some 3 n/64 + 2 n/256 dependent launches on two
  // streams) is captured once per shape and workspace and replayed as a
  // graph: the chain's launches then follow each other without the host's
  // per-launch gaps.  The system's arrays are read through a descriptor
  // copied into the workspace before every replay, so a cached graph holds
  // no pointer of the caller's system.
  const ss_system* sysd = reinterpret_cast<const ss_system*>(ws + L.sysc);
  const int nvals = sys->nvals;
  auto enqueue = [&](hipStream_t st) -> ss_status {
    k_clear_flag<<<1, 64, 0, st>>>(flag);
    // Both halves go through every launch together (blockIdx.z = half): they
    // are independent systems, so the latency-bound steps of the
    // factorisation are shared between them.
    k_form_b<<<dim3(static_cast<unsigned>(n), 1, nv), kFormThreads, 0, st>>>(sysd, B, bs, c, vs);
    SS_HIP_TRY(hipEventRecord(evFork, st));
    SS_HIP_TRY(hipStreamWaitEvent(sb, evFork, 0));
    // Blocked right-looking Cholesky, lower, in place, with a look-ahead of
    // one panel.  Panel p (kPanel columns) is factored on the caller's stream
    // 64 columns at a time (diagonal block, panel solve as a product with
    // L_kk^{-T}, update of the panel's remaining columns).  Its trailing update
    // is cut in two: the next panel's columns (near), on the caller's stream,
    // and everything to their right (far), on the second stream, where it
    // runs while the next panel is factored.  Ordering: panel p waits for the
    // far update of panel p-2 (the last one that touches its columns and has
    // not been waited for); the near update of panel p waits for the far
    // update of panel p-1 (both write panel p+1's columns); the far update of
    // panel p waits for panel p's factor.
    for (int64_t p = 0; p < npanel; ++p) {
      const int64_t K0 = p * kPanel;
      const int64_t W = std::min<int64_t>(kPanel, n - K0);
      if (p >= 2) SS_HIP_TRY(hipStreamWaitEvent(st, evU[p - 2], 0));
      for (int64_t k0 = K0; k0 < K0 + W; k0 += kNb) {
        const int nb = static_cast<int>(std::min<int64_t>(kNb, K0 + W - k0));
        double* Lk = Linv + (k0 / kNb) * kNb * kNb;
        k_potrf_diag<<<dim3(1, 1, nv), 64 * kDiagWaves, 0, st>>>(B, n, k0, nb, Lk, flag, bs, ls, c, y, vs);
        const int64_t below = n - k0 - nb;
        if (below <= 0) continue;  // nb < 64 only for the last block
        double* P = B + (k0 + nb) * n + k0;
        k_gemm_nt_k64<true><<<dim3(tiles(below, kNb), 1, nv), 256, 0, st>>>(P, n, Lk, kNb, P, n, below, nb, nb, 1.0, 0.0, 0,
                                                                        bs, ls, bs, y + k0, c + k0 + nb, vs);
        const int64_t pw = K0 + W - (k0 + nb);
        if (pw > 0)
          k_gemm_nt_k64<true><<<dim3(tiles(below, kNb), tiles(pw, kNb), nv), 256, 0, st>>>(
              P, n, P, n, P + nb, n, below, pw, nb, -1.0, 1.0, 1, bs, bs, bs, nullptr, nullptr, 0);
      }
      SS_HIP_TRY(hipEventRecord(evF[p], st));
      const int64_t rest = n - K0 - W;
      if (rest > 0) {
        double* Q = B + (K0 + W) * n + K0;
        const int64_t W1 = std::min<int64_t>(kPanel, rest);
        if (p >= 1) SS_HIP_TRY(hipStreamWaitEvent(st, evU[p - 1], 0));
        // the near update is on the chain: where it is short, smaller tiles
        // (four times the blocks) finish it sooner
        if (rest <= kNearSmall)
          k_gemm_nt<kNb, 4, true><<<dim3(tiles(rest, kNb), tiles(W1, kNb), nv), 256, 0, st>>>(Q, n, Q, n, Q + W, n, rest, W1, W,
                                                                                     -1.0, 1.0, 1, bs, bs, bs);
        else
          k_gemm_nt<kTrail, kTrailWaves, true><<<dim3(tiles(rest, kTrail), tiles(W1, kTrail), nv), 64 * kTrailWaves, 0, st>>>(
              Q, n, Q, n, Q + W, n, rest, W1, W, -1.0, 1.0, 1, bs, bs, bs);
        const int64_t far = rest - W1;
        if (far > 0) {
          SS_HIP_TRY(hipStreamWaitEvent(sb, evF[p], 0));
          double* Qf = Q + W1 * n;
          if (far <= kNearSmall)  // a short far update fills the chip only with the smaller tiles
            k_gemm_nt<kNb, 4><<<dim3(tiles(far, kNb), tiles(far, kNb), nv), 256, 0, sb>>>(
                Qf, n, Qf, n, Qf + W + W1, n, far, far, W, -1.0, 1.0, 1, bs, bs, bs);
          else
            k_gemm_nt<kTrail, kTrailWaves><<<dim3(tiles(far, kTrail), tiles(far, kTrail), nv), 64 * kTrailWaves, 0,
                                              sb>>>(Qf, n, Qf, n, Qf + W + W1, n, far, far, W, -1.0, 1.0, 1, bs, bs, bs);
        }
      }
      SS_HIP_TRY(hipEventRecord(evU[p], sb));
    }
    SS_HIP_TRY(hipStreamWaitEvent(st, evU[npanel - 1], 0));
    // L y = c ran with the factorisation (each diagonal block forms its
    // y_k, each panel solve updates c below it); now L^T x = y, 64 rows a
    // step
    {
      const int64_t k0 = (nt - 1) * kNb;
      k_diag_bwd<<<dim3(1, 1, nv), 256, 0, st>>>(Linv + (nt - 1) * kNb * kNb, y, x, k0,
                                                 static_cast<int>(n - k0), ls, vs);
    }
    for (int64_t k = nt - 1; k >= 1; --k) {
      const int64_t k0 = k * kNb;
      const int nb = static_cast<int>(std::min<int64_t>(kNb, n - k0));
      k_bwd_step<<<dim3(static_cast<unsigned>(k0 / kNb), 1, nv), 256, 0, st>>>(B, n, n, k0, nb,
                                                                                Linv + (k - 1) * kNb * kNb, y, x, bs,
                                                                                ls, vs);
    }
    k_recombine_f64<<<blocks(n, 256), 256, 0, st>>>(x, x + vs, n, nvals, f);
    return hipGetLastError() == hipSuccess ? SS_OK : fail(SS_E_HIP, "ss_normal_solve: launch failed");
  };
  SS_HIP_TRY(hipMemcpyAsync(ws + L.sysc, sys, sizeof(ss_system), hipMemcpyHostToDevice, st));
  const NormalKey key{dev, ws, f, n, nvals};
  ss_status cap = SS_OK;
  GraphEntry* g = nullptr;
  auto capture = [&](hipStream_t cs) { cap = enqueue(cs); };
  if (ss_status s = normal_graphs().acquire(key, dev, capture, &g)) return s;
  if (cap != SS_OK) {
    normal_graphs().drop(key);
    return cap;
  }
  const hipError_t le = hipGraphLaunch(g->exec, st);
  normal_graphs().release(g, st);
  if (le != hipSuccess) return fail(SS_E_HIP, "ss_normal_solve: graph launch failed: %s", hipGetErrorString(le));
  SS_HIP_TRY(hipGetLastError());
  int32_t hflag = 0;
  SS_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof hflag, hipMemcpyDeviceToHost, st));
  SS_HIP_TRY(hipStreamSynchronize(st));
  if (hflag) return fail(SS_E_SHAPE, "ss_normal_solve: the normal matrix is not positive definite (A lacks full column rank)");
  return SS_OK;
}
