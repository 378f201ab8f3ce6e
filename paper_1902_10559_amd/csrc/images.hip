// Image-side operations: the recombination of Theorem 1 (eq. (5)), its
// inverse, and the forward projection q = A f of eq. (1).

#include <algorithm>

#include "device.h"
#include "internal.h"

namespace ss {
namespace {

// f[j] = (f2[j] + f1[j]) / 2, f[N-1-j] = (f2[j] - f1[j]) / 2.  Halving is
// exact, so each output is the correctly rounded FP32 sum or difference
// scaled by 0.5.
__global__ void k_recombine(const float2* __restrict__ f12, int64_t n, float* __restrict__ f) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const float2 h = f12[j];
  f[j] = (h.y + h.x) * 0.5f;
  f[2 * n - 1 - j] = (h.y - h.x) * 0.5f;
}

// Up to kRecombineChunk images per launch, their descriptors in the kernel
// arguments; image k owns blocks [blk0[k], blk0[k + 1]).
constexpr int kRecombineChunk = 32;
struct RecombineChunk {
  const float2* f12[kRecombineChunk];
  float* f[kRecombineChunk];
  int64_t n[kRecombineChunk];
  uint32_t blk0[kRecombineChunk + 1];
  int32_t count;
};

__global__ void k_recombine_chunk(RecombineChunk ch) {
  const uint32_t b = blockIdx.x;
  int k = 0;
  while (k + 1 < ch.count && ch.blk0[k + 1] <= b) ++k;  // uniform per block
  const int64_t j = static_cast<int64_t>(b - ch.blk0[k]) * blockDim.x + threadIdx.x;
  const int64_t n = ch.n[k];
  if (j >= n) return;
  const float2 h = ch.f12[k][j];
  ch.f[k][j] = (h.y + h.x) * 0.5f;
  ch.f[k][2 * n - 1 - j] = (h.y - h.x) * 0.5f;
}

// f1[j] = f[j] - f[N-1-j], f2[j] = f[j] + f[N-1-j].
__global__ void k_image_fold(const float* __restrict__ f, int64_t n, float2* __restrict__ f12) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const float a = f[j], b = f[2 * n - 1 - j];
  f12[j] = make_float2(a - b, a + b);
}

__global__ void k_fold_rhs(const float* __restrict__ p, int64_t m, float2* __restrict__ p12) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const float a = p[i], b = p[2 * m - 1 - i];
  p12[i] = make_float2(a - b, a + b);
}

constexpr int kProjWaves = 4;

// q[i] = sum_j A[i,j] f[j]; one wavefront per row, FP32 accumulation.
__global__ __launch_bounds__(kWave* kProjWaves) void k_project(ss_matrix_dev A, const float* __restrict__ f,
                                                               float* __restrict__ q) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kProjWaves + wave_id();
  if (i >= A.M) return;
  float acc = 0.0f;
  for (int64_t k = A.row_ptr[i] + lane_id(); k < A.row_ptr[i + 1]; k += kWave)
    acc = fmaf(A.val[k], f[A.col_idx[k]], acc);
  acc = group_sum<kWave>(acc);
  if (lane_id() == 0) q[i] = acc;
}

}  // namespace
}  // namespace ss

using namespace ss;

extern "C" ss_status ss_recombine(const float* f12, int64_t n, float* f, void* stream) {
  clear_error();
  if (!f12 || !f || n <= 0) return fail(SS_E_ARG, "ss_recombine: bad argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  k_recombine<<<static_cast<unsigned>((n + 255) / 256), 256, 0, st>>>(reinterpret_cast<const float2*>(f12), n, f);
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_recombine_batch(const float* const* f12, const int64_t* n, float* const* f, int32_t count,
                                       void* stream) {
  clear_error();
  if (!f12 || !n || !f || count < 0) return fail(SS_E_ARG, "ss_recombine_batch: bad argument");
  for (int32_t k = 0; k < count; ++k)
    if (!f12[k] || !f[k] || n[k] <= 0) return fail(SS_E_ARG, "ss_recombine_batch: bad image %d", k);
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int32_t k0 = 0; k0 < count; k0 += kRecombineChunk) {
    RecombineChunk ch{};
    ch.count = std::min(kRecombineChunk, count - k0);
    uint64_t blocks = 0;
    for (int i = 0; i < ch.count; ++i) {
      ch.f12[i] = reinterpret_cast<const float2*>(f12[k0 + i]);
      ch.f[i] = f[k0 + i];
      ch.n[i] = n[k0 + i];
      ch.blk0[i] = static_cast<uint32_t>(blocks);
      blocks += static_cast<uint64_t>((n[k0 + i] + 255) / 256);
      if (blocks > UINT32_MAX) return fail(SS_E_ARG, "ss_recombine_batch: images too large");
    }
    ch.blk0[ch.count] = static_cast<uint32_t>(blocks);
    k_recombine_chunk<<<static_cast<unsigned>(blocks), 256, 0, st>>>(ch);
  }
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_image_fold(const float* f, int64_t N, float* f12, void* stream) {
  clear_error();
  if (!f || !f12 || N <= 0) return fail(SS_E_ARG, "ss_image_fold: bad argument");
  if (N % 2) return fail(SS_E_ODD, "ss_image_fold: N must be even");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = N / 2;
  k_image_fold<<<static_cast<unsigned>((n + 255) / 256), 256, 0, st>>>(f, n, reinterpret_cast<float2*>(f12));
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_project(const ss_matrix_dev* A, const float* f, float* q, void* stream) {
  clear_error();
  if (!A || !A->row_ptr || !f || !q || A->M <= 0 || A->N <= 0 || A->nnz < 0 ||
      (A->nnz > 0 && (!A->col_idx || !A->val)))
    return fail(SS_E_ARG, "ss_project: bad argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  k_project<<<static_cast<unsigned>((A->M + kProjWaves - 1) / kProjWaves), kWave * kProjWaves, 0, st>>>(*A, f, q);
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_fold_rhs(const float* p, int64_t M, float* p12, void* stream) {
  clear_error();
  if (!p || !p12 || M <= 0) return fail(SS_E_ARG, "ss_fold_rhs: bad argument");
  if (M % 2) return fail(SS_E_ODD, "ss_fold_rhs: M must be even");
  const int64_t m = M / 2;
  k_fold_rhs<<<static_cast<unsigned>((m + 255) / 256), 256, 0, static_cast<hipStream_t>(stream)>>>(
      p, m, reinterpret_cast<float2*>(p12));
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}
