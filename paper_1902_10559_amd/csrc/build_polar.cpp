// ss_build_polar_system: the system matrix A of eq. (1) for a polar voxel
// grid scanned by parallel beams, the second symmetric geometry of the
// paper's closing example (tomographic gamma scanning of a cylindrical
// container, Fig. 4, renumbered so that the system splits in two).
//
// A ray is the line {t n + u d}, n = (cos phi, sin phi), d = (sin phi,
// -cos phi).  Its crossings with the ring circles (roots of a quadratic in
// u) and with the lines through the centre that carry the sector boundaries,
// clipped to the disk and sorted, cut the chord into segments that each lie
// in one voxel: the voxel of the segment's midpoint, from its radius and
// from atan2(|x|, z).  A line can cross one annular sector twice (the inner
// circle is concave), and then the voxel gets the sum of the two pieces.
// All of it in FP64, rounded to FP32 at the end.
//
// Eq. (2) comes out bitwise: a mirrored ray (phi -> -phi, t -> -t) has its
// point and direction negated exactly in x, so its quadratic has the same
// coefficients; the boundary line of a mirrored sector has the exactly
// negated x direction, so the crossing parameter is the same; and the
// voxel of a midpoint is found through |x|.  This file is compiled without
// floating-point contraction so that the same expressions give the same
// bits on every ray.

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "host_build.h"
#include "internal.h"

namespace {

constexpr double kMinSegment = 1e-9;  // mm
constexpr double kPi = 3.14159265358979323846;

struct PolarTracer {
  int rings, sectors;
  double radius, width;                       // width: sector angle 2 pi / S
  std::vector<std::pair<double, double>> e;   // boundary-line directions, S/2 of them

  explicit PolarTracer(const ss_polar_grid& g)
      : rings(g.rings), sectors(g.sectors), radius(g.radius), width(2.0 * kPi / g.sectors) {
    const int s2 = sectors / 2;
    e.assign(static_cast<size_t>(s2), {0.0, 0.0});
    std::vector<bool> set(static_cast<size_t>(s2), false);
    for (int s = 0; s < s2; ++s) {
      if (s == 0) {
        e[0] = {0.0, 1.0};
      } else if (2 * s == s2) {
        e[s] = {1.0, 0.0};
      } else if (2 * s < s2) {
        const double a = 2.0 * kPi * s / sectors;
        e[s] = {std::sin(a), std::cos(a)};
      } else {
        continue;
      }
      set[s] = true;
    }
    // the line s2 - s is the mirror of line s: exact x-negation
    for (int s = 0; s < s2; ++s)
      if (!set[s]) e[s] = {-e[s2 - s].first, e[s2 - s].second};
  }

  int64_t index(int64_t r, int64_t h, bool left) const {
    const int64_t half = r * (sectors / 2) + h;
    return left ? half : static_cast<int64_t>(rings) * sectors - 1 - half;
  }

  void trace(double phi, double t, std::vector<double>& cuts, ss::host::Segments& out) const {
    out.clear();
    cuts.clear();
    const double c = std::cos(std::fabs(phi));
    const double sn = std::copysign(std::sin(std::fabs(phi)), phi);
    const double px = t * c, pz = t * sn, dx = sn, dz = -c;
    const double a = dx * dx + dz * dz;
    const double b = 2.0 * (px * dx + pz * dz);
    const double pp = px * px + pz * pz;
    const double disc = b * b - 4.0 * a * (pp - radius * radius);
    if (!(disc > 0.0)) return;
    const double q = std::sqrt(disc);
    const double u0 = (-b - q) / (2.0 * a), u1 = (-b + q) / (2.0 * a);
    cuts.push_back(u0);
    cuts.push_back(u1);
    for (int r = 1; r < rings; ++r) {
      const double rho = r * radius / rings;
      const double dr = b * b - 4.0 * a * (pp - rho * rho);
      if (dr > 0.0) {
        const double qr = std::sqrt(dr);
        cuts.push_back((-b - qr) / (2.0 * a));
        cuts.push_back((-b + qr) / (2.0 * a));
      }
    }
    for (const auto& ev : e) {
      const double den = dx * ev.second - dz * ev.first;
      if (den != 0.0) cuts.push_back(-(px * ev.second - pz * ev.first) / den);
    }
    std::sort(cuts.begin(), cuts.end());
    const double dlen = std::sqrt(a);
    const int s2 = sectors / 2;
    // segments between consecutive cuts inside [u0, u1], in order along the ray
    double prev = u0;
    for (double v : cuts) {
      if (v < u0 || v > u1 || v <= prev) continue;
      const double len = (v - prev) * dlen;
      const double mid = 0.5 * (prev + v);
      prev = v;
      if (!(len > kMinSegment)) continue;
      const double mx = px + mid * dx, mz = pz + mid * dz;
      const double rho = std::sqrt(mx * mx + mz * mz);
      const int64_t ring = static_cast<int64_t>(std::floor(rho * rings / radius));
      if (ring >= rings || mx == 0.0) continue;
      const int64_t h = std::min<int64_t>(static_cast<int64_t>(std::floor(std::atan2(std::fabs(mx), mz) / width)),
                                          s2 - 1);
      out.emplace_back(static_cast<int32_t>(index(ring, h, mx < 0.0)), len);
    }
    // a line meets an annular sector in at most two pieces (the sector is
    // an annulus, met at most twice, cut by a convex wedge); their sum does
    // not depend on the order
    std::stable_sort(out.begin(), out.end(),
                     [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                       return x.first < y.first;
                     });
    size_t w = 0;
    for (size_t r = 0; r < out.size(); ++r) {
      if (w > 0 && out[w - 1].first == out[r].first)
        out[w - 1].second += out[r].second;
      else
        out[w++] = out[r];
    }
    out.resize(w);
  }
};

}  // namespace

extern "C" ss_status ss_build_polar_system(const ss_polar_grid* grid, const ss_parallel_scan* scan,
                                           int32_t nthreads, ss_matrix* out) {
  ss::clear_error();
  if (!grid || !scan || !out || !scan->phi || !scan->offset)
    return ss::fail(SS_E_ARG, "ss_build_polar_system: NULL argument");
  if (grid->rings <= 0 || grid->sectors <= 0 || !(grid->radius > 0.0) || scan->K <= 0 || scan->B <= 0)
    return ss::fail(SS_E_ARG, "ss_build_polar_system: sizes and radius must be positive");
  if (grid->sectors % 2 || scan->K % 2 || scan->B % 2)
    return ss::fail(SS_E_ODD, "ss_build_polar_system: sectors=%d, K=%d and B=%d must be even", grid->sectors,
                    scan->K, scan->B);
  const int K = scan->K, B = scan->B;
  for (int k = 0; k < K; ++k) {
    if (scan->phi[K - 1 - k] != -scan->phi[k])
      return ss::fail(SS_E_ASYM, "ss_build_polar_system: view %d is not the mirror of view %d", K - 1 - k, k);
    if (!(std::fabs(scan->phi[k]) < 0.5 * kPi) || (k + 1 < K && !(scan->phi[k] < scan->phi[k + 1])))
      return ss::fail(SS_E_ARG, "ss_build_polar_system: phi must ascend strictly inside (-pi/2, pi/2)");
  }
  for (int b = 0; b < B; ++b) {
    if (scan->offset[B - 1 - b] != -scan->offset[b])
      return ss::fail(SS_E_ASYM, "ss_build_polar_system: offset %d is not the mirror of offset %d", B - 1 - b, b);
    if (b + 1 < B && !(scan->offset[b] < scan->offset[b + 1]))
      return ss::fail(SS_E_ARG, "ss_build_polar_system: offsets must ascend strictly");
  }
  const int64_t M = static_cast<int64_t>(K) * B;
  const int64_t N = static_cast<int64_t>(grid->rings) * grid->sectors;
  if (N > INT32_MAX || M > INT32_MAX) return ss::fail(SS_E_ARG, "ss_build_polar_system: M and N must fit in int32");
  const PolarTracer tr(*grid);
  auto ray = [&](int64_t i, std::vector<double>& cuts, ss::host::Segments& seg) {
    tr.trace(scan->phi[i / B], scan->offset[i % B], cuts, seg);
  };
  return ss::host::assemble(M, N, ss::host::threads(nthreads), ray, "ss_build_polar_system", out);
}
