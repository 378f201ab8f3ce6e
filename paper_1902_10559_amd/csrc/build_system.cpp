// ss_build_system: the system matrix A of eq. (1) for a symmetric scan.
//
// Weights are intersection lengths of each ray with each voxel, found by
// Siddon's method: the parameters alpha at which the ray crosses the grid's
// x- and z-planes, sorted, cut the ray into segments that each lie inside
// one voxel; a segment's length is |D - S| * (alpha_{t+1} - alpha_t) and its
// voxel is the one containing its midpoint.  All of it runs in FP64 and is
// rounded to FP32 at the end.
//
// Eq. (2) comes out bitwise because the input coordinates are exact mirror
// pairs and every step is sign-symmetric: plane positions are
// (k - nx/2) * pitch (so X[nx-k] == -X[k]), a mirrored ray has the same
// sorted alpha list, and the voxel column of a midpoint is computed from |x|.
// This file is compiled without floating-point contraction so that the same
// expressions give the same bits on every ray.
//
// Rays are traced twice (count, then fill) on a pool of host threads
// (host_build.h), which also forms the CSC copy.

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "host_build.h"
#include "internal.h"

namespace {

constexpr double kMinSegment = 1e-9;  // mm; shorter segments are corner touches

struct Tracer {
  int nx, nz;
  double pitch;
  double x_lo, x_hi, z_top;  // grid box: x in [x_lo, x_hi], z in [0, z_top]

  explicit Tracer(const ss_grid& g)
      : nx(g.nx), nz(g.nz), pitch(g.pitch),
        x_lo(static_cast<double>(0 - g.nx / 2) * g.pitch),
        x_hi(static_cast<double>(g.nx - g.nx / 2) * g.pitch),
        z_top(static_cast<double>(g.nz) * g.pitch) {}

  double xplane(int k) const { return static_cast<double>(k - nx / 2) * pitch; }
  double zplane(int l) const { return static_cast<double>(l) * pitch; }

  int64_t snake(int64_t c, int64_t r) const {
    return c * nz + ((c & 1) == 0 ? r : nz - 1 - r);
  }

  // Appends (snake index, length) of every segment of the ray S -> E to
  // `out`, in order along the ray; `alphas` is scratch.
  void trace(double sx, double sz, double ex, double ez,
             std::vector<double>& alphas,
             std::vector<std::pair<int32_t, double>>& out) const {
    out.clear();
    alphas.clear();
    const double dx = ex - sx;
    const double dz = ez - sz;
    const double d = std::sqrt(dx * dx + dz * dz);
    double lo = 0.0, hi = 1.0;
    if (dx != 0.0) {
      const double a0 = (x_lo - sx) / dx, a1 = (x_hi - sx) / dx;
      lo = std::max(lo, std::min(a0, a1));
      hi = std::min(hi, std::max(a0, a1));
    } else if (!(x_lo < sx && sx < x_hi)) {
      return;
    }
    if (dz != 0.0) {
      const double a0 = (0.0 - sz) / dz, a1 = (z_top - sz) / dz;
      lo = std::max(lo, std::min(a0, a1));
      hi = std::min(hi, std::max(a0, a1));
    } else if (!(0.0 < sz && sz < z_top)) {
      return;
    }
    if (!(lo < hi)) return;
    alphas.push_back(lo);
    alphas.push_back(hi);
    if (dx != 0.0) {
      // candidate planes around the x-range of the chord; the exact test on
      // alpha below decides which are crossed
      const double xa = sx + lo * dx, xb = sx + hi * dx;
      int k0 = static_cast<int>(std::floor((std::min(xa, xb) - x_lo) / pitch)) - 1;
      int k1 = static_cast<int>(std::ceil((std::max(xa, xb) - x_lo) / pitch)) + 1;
      k0 = std::max(k0, 0);
      k1 = std::min(k1, nx);
      for (int k = k0; k <= k1; ++k) {
        const double a = (xplane(k) - sx) / dx;
        if (a > lo && a < hi) alphas.push_back(a);
      }
    }
    if (dz != 0.0) {
      const double za = sz + lo * dz, zb = sz + hi * dz;
      int l0 = static_cast<int>(std::floor(std::min(za, zb) / pitch)) - 1;
      int l1 = static_cast<int>(std::ceil(std::max(za, zb) / pitch)) + 1;
      l0 = std::max(l0, 0);
      l1 = std::min(l1, nz);
      for (int l = l0; l <= l1; ++l) {
        const double a = (zplane(l) - sz) / dz;
        if (a > lo && a < hi) alphas.push_back(a);
      }
    }
    std::sort(alphas.begin(), alphas.end());
    const int half = nx / 2;
    for (size_t t = 0; t + 1 < alphas.size(); ++t) {
      const double len = d * (alphas[t + 1] - alphas[t]);
      if (!(len > kMinSegment)) continue;
      const double mid = 0.5 * (alphas[t] + alphas[t + 1]);
      const double xm = sx + mid * dx;
      const double zm = sz + mid * dz;
      const int64_t c = xm >= 0.0
                            ? half + static_cast<int64_t>(std::floor(xm / pitch))
                            : half - 1 - static_cast<int64_t>(std::floor(-xm / pitch));
      const int64_t r = static_cast<int64_t>(std::floor((z_top - zm) / pitch));
      if (c < 0 || c >= nx || r < 0 || r >= nz) continue;  // unreachable for interior midpoints
      out.emplace_back(static_cast<int32_t>(snake(c, r)), len);
    }
    std::sort(out.begin(), out.end(),
              [](const std::pair<int32_t, double>& a,
                 const std::pair<int32_t, double>& b) { return a.first < b.first; });
  }
};

}  // namespace

extern "C" ss_status ss_snake_order(const ss_grid* grid, int64_t* snake) {
  ss::clear_error();
  if (!grid || !snake) return ss::fail(SS_E_ARG, "ss_snake_order: NULL argument");
  if (grid->nx <= 0 || grid->nz <= 0) return ss::fail(SS_E_ARG, "ss_snake_order: bad grid size");
  const int64_t nx = grid->nx, nz = grid->nz;
  for (int64_t r = 0; r < nz; ++r)
    for (int64_t c = 0; c < nx; ++c)
      snake[r * nx + c] = c * nz + ((c & 1) == 0 ? r : nz - 1 - r);
  return SS_OK;
}

extern "C" void ss_matrix_free(ss_matrix* A) {
  if (!A) return;
  std::free(A->row_ptr);
  std::free(A->col_idx);
  std::free(A->val);
  std::free(A->col_ptr);
  std::free(A->row_idx);
  std::free(A->val_t);
  std::memset(A, 0, sizeof *A);
}

extern "C" ss_status ss_build_system(const ss_grid* grid, const ss_geometry* geom,
                                     int32_t nthreads, ss_matrix* out) {
  ss::clear_error();
  if (!grid || !geom || !out || !geom->src_x || !geom->src_z || !geom->bin_x)
    return ss::fail(SS_E_ARG, "ss_build_system: NULL argument");
  if (grid->nx <= 0 || grid->nz <= 0 || !(grid->pitch > 0.0) || geom->K <= 0 || geom->B <= 0)
    return ss::fail(SS_E_ARG, "ss_build_system: sizes and pitch must be positive");
  if (grid->nx % 2 || geom->K % 2 || geom->B % 2)
    return ss::fail(SS_E_ODD, "ss_build_system: nx=%d, K=%d and B=%d must be even",
                    grid->nx, geom->K, geom->B);
  const int K = geom->K, B = geom->B;
  for (int k = 0; k < K; ++k) {
    if (geom->src_x[K - 1 - k] != -geom->src_x[k] || geom->src_z[K - 1 - k] != geom->src_z[k])
      return ss::fail(SS_E_ASYM, "ss_build_system: source %d is not the mirror of source %d", K - 1 - k, k);
    if (k + 1 < K && !(geom->src_x[k] <= geom->src_x[k + 1]))
      return ss::fail(SS_E_ARG, "ss_build_system: src_x must ascend");
  }
  for (int b = 0; b < B; ++b) {
    if (geom->bin_x[B - 1 - b] != -geom->bin_x[b])
      return ss::fail(SS_E_ASYM, "ss_build_system: bin %d is not the mirror of bin %d", B - 1 - b, b);
    if (b + 1 < B && !(geom->bin_x[b] < geom->bin_x[b + 1]))
      return ss::fail(SS_E_ARG, "ss_build_system: bin_x must ascend strictly");
  }
  const int64_t M = static_cast<int64_t>(K) * B;
  const int64_t N = static_cast<int64_t>(grid->nx) * grid->nz;
  if (N > INT32_MAX || M > INT32_MAX)
    return ss::fail(SS_E_ARG, "ss_build_system: M and N must fit in int32");
  const int nt = ss::host::threads(nthreads);
  const Tracer tr(*grid);
  auto ray = [&](int64_t i, std::vector<double>& al, ss::host::Segments& seg) {
    const int64_t k = i / B, b = i % B;
    tr.trace(geom->src_x[k], geom->src_z[k], geom->bin_x[b], geom->det_z, al, seg);
  };
  return ss::host::assemble(M, N, nt, ray, "ss_build_system", out);
}
