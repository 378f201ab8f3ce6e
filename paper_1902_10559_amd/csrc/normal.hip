// The direct path (Theorem 2): the normal equations A(k)^T A(k) f(k) =
// A(k)^T p(k) of each half of the folded pair, solved by a Cholesky
// factorisation in FP64, and the halves recombined by eq. (5); for a single
// system (nvals = 1) the same solve on A itself.  The split turns one
// N x N factorisation of an N x N matrix formed from M rays into two of
// (N/2)^2 from M/2 rays: 1/4 of the flops of forming B and 1/4 of the
// factorisation's (the paper's 2^(alpha+beta) argument after Theorem 1).
//
// Steps per half: A^T densified (n rows of m FP64, row j = column j of A,
// from the CSC); c = A^T p; B = A^T A, lower triangle, by an FP64 matrix-core
// GEMM (v_mfma_f64_16x16x4f64); right-looking blocked Cholesky of B in place
// (64 x 64 diagonal blocks factored in shared memory, panel solves, trailing
// updates by the same GEMM); forward and back substitution, block by block.

#include <algorithm>
#include <cmath>
#include <vector>

#include "device.h"
#include "internal.h"

namespace ss {
namespace {

constexpr int kNb = 64;  // Cholesky block and GEMM tile

typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ void k_zero_f64(double* p, int64_t count) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

// At[j * m + i] = A(h)[i, j]; c[j] = sum_i A(h)[i, j] p(h)[i].  One thread
// per column j of the half's CSC; value h of each entry's nv values.
__global__ void k_densify(ss_system sys, int h, double* At, double* c) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= sys.n) return;
  const float* v = static_cast<const float*>(sys.val_t);
  const int nv = sys.nvals;
  double acc = 0.0;
  for (int64_t e = sys.col_ptr[j]; e < sys.col_ptr[j + 1]; ++e) {
    const int64_t i = sys.row_idx[e];
    const double a = v[nv * e + h];
    At[j * sys.m + i] = a;
    acc += a * static_cast<double>(sys.p[nv * i + h]);
  }
  c[j] = acc;
}

// C[i, j] = beta * C[i, j] + alpha * sum_k X[i, k] Y[j, k] for the tiles of C
// on or below the diagonal (i-tile >= j-tile), 64 x 64 per block of 4
// wavefronts (2 x 2, 32 x 32 each as 2 x 2 matrix-core tiles).  X, Y, C
// row-major with leading dimensions ldx, ldy, ldc; n x n output, K terms.
// Operand layouts of v_mfma_f64_16x16x4f64 for lane l (g = l / 16):
//   A[m][k]: m = l % 16, k = g;  B[k][n]: n = l % 16, k = g;
//   D[m][n]: m = g + 4 r (r = 0..3, the accumulator's element), n = l % 16
// (rows interleaved by 4, unlike the 4 consecutive rows of the FP32 forms).
constexpr int kKc = 16;
__global__ __launch_bounds__(256) void k_gemm_nt_lower(const double* __restrict__ X, int64_t ldx,
                                                       const double* __restrict__ Y, int64_t ldy, double* C,
                                                       int64_t ldc, int64_t n, int64_t K, double alpha,
                                                       double beta) {
  // triangular block index -> (ti, tj), ti >= tj
  const int64_t b = blockIdx.x;
  int64_t ti = static_cast<int64_t>((std::sqrt(8.0 * static_cast<double>(b) + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
  while (ti * (ti + 1) / 2 > b) --ti;
  const int64_t tj = b - ti * (ti + 1) / 2;
  const int64_t r0 = ti * kNb, c0 = tj * kNb;
  __shared__ double xs[kNb][kKc + 1];
  __shared__ double ys[kNb][kKc + 1];
  const int lane = lane_id(), w = wave_id();
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;  // this wave's 32 x 32 quadrant
  const int g = lane / 16, l16 = lane % 16;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[a][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = 0; k0 < K; k0 += kKc) {
    // stage 64 x 16 of X (rows r0..) and of Y (rows c0..), zero outside
    for (int t = threadIdx.x; t < kNb * kKc; t += 256) {
      const int rr = t / kKc, kk = t % kKc;
      const int64_t k = k0 + kk;
      const int64_t xr = r0 + rr, yr = c0 + rr;
      xs[rr][kk] = (xr < n && k < K) ? X[xr * ldx + k] : 0.0;
      ys[rr][kk] = (yr < n && k < K) ? Y[yr * ldy + k] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKc; kk += 4) {
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double av = xs[wr + 16 * a + l16][kk + g];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const double bv = ys[wc + 16 * q + l16][kk + g];
          acc[a][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[a][q], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = r0 + wr + 16 * a + g + 4 * r;
        const int64_t j = c0 + wc + 16 * q + l16;
        if (i < n && j < n && j <= i) {
          double* cp = C + i * ldc + j;
          *cp = (beta == 0.0 ? 0.0 : beta * *cp) + alpha * acc[a][q][r];
        }
      }
}

// Cholesky of the diagonal block B[k0.., k0..] (size nb <= 64) in shared
// memory, lower factor written back; thread t owns row t.  A non-positive
// pivot sets *flag and is replaced by 1 so that the rest stays finite.
__global__ __launch_bounds__(64) void k_potrf_diag(double* B, int64_t ld, int64_t k0, int nb, int32_t* flag) {
  __shared__ double s[kNb][kNb + 1];
  const int t = threadIdx.x;
  if (t < nb)
    for (int c = 0; c <= t; ++c) s[t][c] = B[(k0 + t) * ld + k0 + c];
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (t == 0) {
      double d = s[j][j];
      if (!(d > 0.0)) {
        *flag = 1;
        d = 1.0;
      }
      s[j][j] = std::sqrt(d);
    }
    __syncthreads();
    if (t > j && t < nb) s[t][j] /= s[j][j];
    __syncthreads();
    if (t > j && t < nb)
      for (int c = j + 1; c <= t; ++c) s[t][c] -= s[t][j] * s[c][j];
    __syncthreads();
  }
  if (t < nb)
    for (int c = 0; c <= t; ++c) B[(k0 + t) * ld + k0 + c] = s[t][c];
}

// Panel below the diagonal block: rows k0+nb .. n-1 of columns k0 ..
// k0+nb-1 become X with X L^T = B (L the factored diagonal block, read from
// global memory: every thread reads the same entry).  One thread per row,
// its row kept in its own column of a shared array.
__global__ __launch_bounds__(64) void k_trsm_panel(double* B, int64_t ld, int64_t n, int64_t k0, int nb) {
  __shared__ double xt[kNb][kNb];
  const int t = threadIdx.x;
  const int64_t row = k0 + nb + static_cast<int64_t>(blockIdx.x) * kNb + t;
  if (row >= n) return;
  for (int c = 0; c < nb; ++c) xt[c][t] = B[row * ld + k0 + c];
  for (int c = 0; c < nb; ++c) {
    const double x = xt[c][t] / B[(k0 + c) * ld + k0 + c];
    xt[c][t] = x;
    for (int c2 = c + 1; c2 < nb; ++c2) xt[c2][t] -= x * B[(k0 + c2) * ld + k0 + c];
  }
  for (int c = 0; c < nb; ++c) B[row * ld + k0 + c] = xt[c][t];
}

// Forward substitution on block k: y[k0..k0+nb) = L_kk^{-1} c[k0..);
// then every later row: c[i] -= sum_t L[i, k0+t] y[k0+t].
__global__ __launch_bounds__(64) void k_trsv_fwd_diag(const double* L, int64_t ld, int64_t k0, int nb, double* c) {
  __shared__ double y[kNb];
  const int t = threadIdx.x;
  if (t < nb) y[t] = c[k0 + t];
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (t == 0) y[j] /= L[(k0 + j) * ld + k0 + j];
    __syncthreads();
    if (t > j && t < nb) y[t] -= L[(k0 + t) * ld + k0 + j] * y[j];
    __syncthreads();
  }
  if (t < nb) c[k0 + t] = y[t];
}

__global__ void k_trsv_fwd_update(const double* L, int64_t ld, int64_t n, int64_t k0, int nb, double* c) {
  const int64_t i = k0 + nb + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int t = 0; t < nb; ++t) acc += L[i * ld + k0 + t] * c[k0 + t];
  c[i] -= acc;
}

// Back substitution with L^T on block k (from the last): f[k0..) =
// L_kk^{-T} y[k0..); then every earlier row: y[i] -= sum_t L[k0+t, i] f[k0+t].
__global__ __launch_bounds__(64) void k_trsv_bwd_diag(const double* L, int64_t ld, int64_t k0, int nb, double* y) {
  __shared__ double f[kNb];
  const int t = threadIdx.x;
  if (t < nb) f[t] = y[k0 + t];
  __syncthreads();
  for (int j = nb - 1; j >= 0; --j) {
    if (t == 0) f[j] /= L[(k0 + j) * ld + k0 + j];
    __syncthreads();
    if (t < j) f[t] -= L[(k0 + j) * ld + k0 + t] * f[j];
    __syncthreads();
  }
  if (t < nb) y[k0 + t] = f[t];
}

__global__ void k_trsv_bwd_update(const double* L, int64_t ld, int64_t k0, int nb, double* y) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= k0) return;
  double acc = 0.0;
  for (int t = 0; t < nb; ++t) acc += L[(k0 + t) * ld + i] * y[k0 + t];
  y[i] -= acc;
}

// f[j] = (f2 + f1) / 2, f[N-1-j] = (f2 - f1) / 2 (eq. (5)), or a copy for
// a single system.
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

struct NormalLayout {
  size_t at, b, c[2], flag, total;
};

inline size_t al(size_t v) { return (v + 255) & ~size_t{255}; }

NormalLayout normal_layout(const ss_system* sys) {
  NormalLayout L;
  size_t o = 0;
  L.at = o;
  o += al(sizeof(double) * static_cast<size_t>(sys->n) * static_cast<size_t>(sys->m));
  L.b = o;
  o += al(sizeof(double) * static_cast<size_t>(sys->n) * static_cast<size_t>(sys->n));
  for (int h = 0; h < 2; ++h) {
    L.c[h] = o;
    o += al(sizeof(double) * static_cast<size_t>(sys->n));
  }
  L.flag = o;
  o += 256;
  L.total = o;
  return L;
}

ss_status check_normal(const ss_system* sys, const char* fn) {
  if (!sys) return fail(SS_E_ARG, "%s: NULL system", fn);
  if (sys->wdtype != SS_F32 || (sys->nvals != 1 && sys->nvals != 2))
    return fail(SS_E_ARG, "%s: an FP32 system with nvals 1 or 2 is required", fn);
  if (sys->m <= 0 || sys->n <= 0 || sys->nnz < 0 || !sys->col_ptr || !sys->p ||
      (sys->nnz > 0 && (!sys->row_idx || !sys->val_t)))
    return fail(SS_E_ARG, "%s: bad system", fn);
  if (sys->n > (int64_t{1} << 20) || sys->m > (int64_t{1} << 24))
    return fail(SS_E_ARG, "%s: system too large for the dense path", fn);
  return SS_OK;
}

inline unsigned blocks(int64_t count, int per) { return static_cast<unsigned>((count + per - 1) / per); }

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
  double* At = reinterpret_cast<double*>(ws + L.at);
  double* B = reinterpret_cast<double*>(ws + L.b);
  int32_t* flag = reinterpret_cast<int32_t*>(ws + L.flag);
  const int64_t n = sys->n, m = sys->m;
  const int64_t nt = (n + kNb - 1) / kNb;
  SS_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
  for (int h = 0; h < sys->nvals; ++h) {
    double* c = reinterpret_cast<double*>(ws + L.c[h]);
    k_zero_f64<<<4096, 256, 0, st>>>(At, n * m);
    k_densify<<<blocks(n, 256), 256, 0, st>>>(*sys, h, At, c);
    // B = At At^T (lower tiles)
    k_gemm_nt_lower<<<static_cast<unsigned>(nt * (nt + 1) / 2), 256, 0, st>>>(At, m, At, m, B, n, n, m, 1.0, 0.0);
    // blocked Cholesky, lower, in place
    for (int64_t k = 0; k < nt; ++k) {
      const int64_t k0 = k * kNb;
      const int nb = static_cast<int>(std::min<int64_t>(kNb, n - k0));
      k_potrf_diag<<<1, 64, 0, st>>>(B, n, k0, nb, flag);
      const int64_t rest = n - k0 - nb;
      if (rest > 0) {
        k_trsm_panel<<<blocks(rest, kNb), 64, 0, st>>>(B, n, n, k0, nb);
        const int64_t rt = (rest + kNb - 1) / kNb;
        // trailing B[k0+nb.., k0+nb..] -= P P^T with P the panel (K = nb)
        double* T = B + (k0 + nb) * n + (k0 + nb);
        const double* P = B + (k0 + nb) * n + k0;
        k_gemm_nt_lower<<<static_cast<unsigned>(rt * (rt + 1) / 2), 256, 0, st>>>(P, n, P, n, T, n, rest, nb, -1.0,
                                                                                 1.0);
      }
    }
    // L y = c, then L^T x = y (in place in c)
    for (int64_t k = 0; k < nt; ++k) {
      const int64_t k0 = k * kNb;
      const int nb = static_cast<int>(std::min<int64_t>(kNb, n - k0));
      k_trsv_fwd_diag<<<1, 64, 0, st>>>(B, n, k0, nb, c);
      if (n - k0 - nb > 0) k_trsv_fwd_update<<<blocks(n - k0 - nb, 256), 256, 0, st>>>(B, n, n, k0, nb, c);
    }
    for (int64_t k = nt - 1; k >= 0; --k) {
      const int64_t k0 = k * kNb;
      const int nb = static_cast<int>(std::min<int64_t>(kNb, n - k0));
      k_trsv_bwd_diag<<<1, 64, 0, st>>>(B, n, k0, nb, c);
      if (k0 > 0) k_trsv_bwd_update<<<blocks(k0, 256), 256, 0, st>>>(B, n, k0, nb, c);
    }
  }
  k_recombine_f64<<<blocks(n, 256), 256, 0, st>>>(reinterpret_cast<double*>(ws + L.c[0]),
                                                  reinterpret_cast<double*>(ws + L.c[1]), n, sys->nvals, f);
  SS_HIP_TRY(hipGetLastError());
  int32_t hflag = 0;
  SS_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof hflag, hipMemcpyDeviceToHost, st));
  SS_HIP_TRY(hipStreamSynchronize(st));
  if (hflag) return fail(SS_E_SHAPE, "ss_normal_solve: the normal matrix is not positive definite (A lacks full column rank)");
  return SS_OK;
}
