// Host-side assembly of a system matrix from per-ray segment lists, shared
// by the geometry builders: rays are traced twice (count, then fill) on a
// pool of host threads, and the CSC copy is a counting sort of the CSR
// entries by column, stable in rows.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <utility>
#include <vector>

#include "internal.h"

namespace ss {
namespace host {

using Segments = std::vector<std::pair<int32_t, double>>;

// body(i, scratch, segments) for i = 0 .. M-1 on nthreads threads, in chunks
// of 256 rays; each thread owns its scratch and segment vectors.
template <class F>
void parallel_rows(int64_t M, int nthreads, F&& body) {
  std::atomic<int64_t> next{0};
  const int64_t chunk = 256;
  auto worker = [&]() {
    std::vector<double> scratch;
    Segments seg;
    scratch.reserve(4096);
    seg.reserve(4096);
    for (;;) {
      const int64_t s = next.fetch_add(chunk);
      if (s >= M) break;
      const int64_t e = std::min(M, s + chunk);
      for (int64_t i = s; i < e; ++i) body(i, scratch, seg);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
}

template <class T>
T* alloc(int64_t count) {
  return static_cast<T*>(std::malloc(sizeof(T) * static_cast<size_t>(std::max<int64_t>(count, 1))));
}

inline int threads(int32_t requested) {
  const int nt = requested > 0 ? requested : static_cast<int>(std::thread::hardware_concurrency());
  return std::max(1, std::min(nt, 256));
}

// Fills *out (M x N) from trace(i, scratch, segments), which must leave in
// `segments` the (column, FP64 length) pairs of ray i with distinct columns
// in ascending order; values are rounded to FP32.
template <class Trace>
ss_status assemble(int64_t M, int64_t N, int nthreads, Trace&& trace, const char* fn, ss_matrix* out) {
  ss_matrix A{};
  A.M = M;
  A.N = N;
  A.row_ptr = alloc<int64_t>(M + 1);
  if (!A.row_ptr) return fail(SS_E_NOMEM, "%s: out of host memory", fn);
  A.row_ptr[0] = 0;
  parallel_rows(M, nthreads, [&](int64_t i, std::vector<double>& sc, Segments& seg) {
    trace(i, sc, seg);
    A.row_ptr[i + 1] = static_cast<int64_t>(seg.size());
  });
  for (int64_t i = 0; i < M; ++i) A.row_ptr[i + 1] += A.row_ptr[i];
  const int64_t nnz = A.row_ptr[M];
  A.nnz = nnz;
  A.col_idx = alloc<int32_t>(nnz);
  A.val = alloc<float>(nnz);
  A.col_ptr = alloc<int64_t>(N + 1);
  A.row_idx = alloc<int32_t>(nnz);
  A.val_t = alloc<float>(nnz);
  if (!A.col_idx || !A.val || !A.col_ptr || !A.row_idx || !A.val_t) {
    ss_matrix_free(&A);
    return fail(SS_E_NOMEM, "%s: out of host memory (nnz=%lld)", fn, static_cast<long long>(nnz));
  }
  parallel_rows(M, nthreads, [&](int64_t i, std::vector<double>& sc, Segments& seg) {
    trace(i, sc, seg);
    int64_t o = A.row_ptr[i];
    for (const auto& s : seg) {
      A.col_idx[o] = s.first;
      A.val[o] = static_cast<float>(s.second);
      ++o;
    }
  });
  std::memset(A.col_ptr, 0, sizeof(int64_t) * static_cast<size_t>(N + 1));
  for (int64_t e = 0; e < nnz; ++e) A.col_ptr[A.col_idx[e] + 1]++;
  for (int64_t j = 0; j < N; ++j) A.col_ptr[j + 1] += A.col_ptr[j];
  std::vector<int64_t> fill(A.col_ptr, A.col_ptr + N);
  for (int64_t i = 0; i < M; ++i) {
    for (int64_t e = A.row_ptr[i]; e < A.row_ptr[i + 1]; ++e) {
      const int64_t o = fill[A.col_idx[e]]++;
      A.row_idx[o] = static_cast<int32_t>(i);
      A.val_t[o] = A.val[e];
    }
  }
  *out = A;
  return SS_OK;
}

}  // namespace host
}  // namespace ss
