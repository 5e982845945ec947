// safety.cpp -- host construction of the safety grid: per cell of a uniform
// grid over the mesh, a lower bound of the distance from any point of the cell
// to the nearest triangle.
//
// A photon whose free path to its next bulk interaction is shorter than the
// bound of its cell cannot hit a triangle before that interaction, so its
// closest-hit search can be skipped with exactly the search's answer ("no
// hit").  Most steps in a large liquid-xenon volume are Rayleigh scatters far
// from any surface.
//
// Construction: every cell overlapped by a triangle's bounding box is marked
// occupied (conservative); an exact Euclidean distance transform (the lower
// envelope of parabolas, Felzenszwalb and Huttenlocher, "Distance transforms
// of sampled functions", 2012) gives, for every cell centre, the distance D to
// the nearest occupied cell centre.  For a point p in cell A and the nearest
// triangle point q in occupied cell B, |p - q| >= |c_A - c_B| - 2h with h the
// cell's half diagonal, so the stored bound is max(0, D - 2h) minus a margin for
// FP32 positions.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "xp_internal.h"

namespace xp {
namespace {

// 1-D squared distance transform of f (length n) into d, in place semantics:
// d[q] = min_p ((q - p)^2 + f[p]).
void dt1d(const std::vector<double>& f, std::vector<double>& d, int n, std::vector<int>& v,
          std::vector<double>& z) {
  const double inf = std::numeric_limits<double>::infinity();
  int k = 0;
  v[0] = 0;
  z[0] = -inf;
  z[1] = inf;
  int first = -1;
  for (int q = 0; q < n; ++q)
    if (std::isfinite(f[q])) {
      first = q;
      break;
    }
  if (first < 0) {
    for (int q = 0; q < n; ++q) d[q] = inf;
    return;
  }
  v[0] = first;
  for (int q = first + 1; q < n; ++q) {
    if (!std::isfinite(f[q])) continue;
    double s = ((f[q] + double(q) * q) - (f[v[k]] + double(v[k]) * v[k])) / (2.0 * q - 2.0 * v[k]);
    while (s <= z[k]) {
      --k;
      s = ((f[q] + double(q) * q) - (f[v[k]] + double(v[k]) * v[k])) / (2.0 * q - 2.0 * v[k]);
    }
    ++k;
    v[k] = q;
    z[k] = s;
    z[k + 1] = inf;
  }
  k = 0;
  for (int q = 0; q < n; ++q) {
    while (z[k + 1] < q) ++k;
    const double dq = double(q) - v[k];
    d[q] = dq * dq + f[v[k]];
  }
}

}  // namespace

bool build_safety_grid(const float* vtx, const int32_t* tri, int64_t nt, int cells_longest,
                       SafetyGrid& out, std::string& err) {
  out = SafetyGrid();
  if (cells_longest <= 0) return true;  // no grid
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t t = 0; t < nt; ++t)
    for (int j = 0; j < 3; ++j) {
      const float* p = vtx + 3 * int64_t(tri[3 * t + j]);
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], double(p[k]));
        hi[k] = std::max(hi[k], double(p[k]));
      }
    }
  double ext = 0.0;
  for (int k = 0; k < 3; ++k) ext = std::max(ext, hi[k] - lo[k]);
  if (!(ext > 0.0)) {
    err = "degenerate mesh extent";
    return false;
  }
  const double cell = ext / cells_longest;
  int n[3];
  for (int k = 0; k < 3; ++k) {
    lo[k] -= cell;  // one cell of border on each side
    n[k] = int(std::ceil((hi[k] + cell - lo[k]) / cell));
    n[k] = std::max(n[k], 1);
  }
  const int64_t total = int64_t(n[0]) * n[1] * n[2];
  if (total > (int64_t(1) << 27)) {
    err = "safety grid too large";
    return false;
  }
  const double inf = std::numeric_limits<double>::infinity();
  std::vector<double> g(total, inf);
  auto idx = [&](int64_t x, int64_t y, int64_t z) { return (z * n[1] + y) * n[0] + x; };
  // conservative occupancy: every cell overlapped by a triangle's bounding box
  for (int64_t t = 0; t < nt; ++t) {
    double a[3] = {1e300, 1e300, 1e300}, b[3] = {-1e300, -1e300, -1e300};
    for (int j = 0; j < 3; ++j) {
      const float* p = vtx + 3 * int64_t(tri[3 * t + j]);
      for (int k = 0; k < 3; ++k) {
        a[k] = std::min(a[k], double(p[k]));
        b[k] = std::max(b[k], double(p[k]));
      }
    }
    int c0[3], c1[3];
    for (int k = 0; k < 3; ++k) {
      c0[k] = std::max(0, int(std::floor((a[k] - lo[k]) / cell)));
      c1[k] = std::min(n[k] - 1, int(std::floor((b[k] - lo[k]) / cell)));
    }
    for (int z = c0[2]; z <= c1[2]; ++z)
      for (int y = c0[1]; y <= c1[1]; ++y)
        for (int x = c0[0]; x <= c1[0]; ++x) g[idx(x, y, z)] = 0.0;
  }
  // exact squared Euclidean distance transform, one axis at a time
  const int nmax = std::max(n[0], std::max(n[1], n[2]));
  std::vector<double> f(nmax), d(nmax), zz(nmax + 1);
  std::vector<int> v(nmax);
  for (int z = 0; z < n[2]; ++z)
    for (int y = 0; y < n[1]; ++y) {
      for (int x = 0; x < n[0]; ++x) f[x] = g[idx(x, y, z)];
      dt1d(f, d, n[0], v, zz);
      for (int x = 0; x < n[0]; ++x) g[idx(x, y, z)] = d[x];
    }
  for (int z = 0; z < n[2]; ++z)
    for (int x = 0; x < n[0]; ++x) {
      for (int y = 0; y < n[1]; ++y) f[y] = g[idx(x, y, z)];
      dt1d(f, d, n[1], v, zz);
      for (int y = 0; y < n[1]; ++y) g[idx(x, y, z)] = d[y];
    }
  for (int y = 0; y < n[1]; ++y)
    for (int x = 0; x < n[0]; ++x) {
      for (int z = 0; z < n[2]; ++z) f[z] = g[idx(x, y, z)];
      dt1d(f, d, n[2], v, zz);
      for (int z = 0; z < n[2]; ++z) g[idx(x, y, z)] = d[z];
    }
  const double two_h = std::sqrt(3.0) * cell;
  // margin for FP32 photon positions (ulp 2.4e-7 m at 2.7 m) and cell lookup
  const double margin = 1e-6 + 1e-6 * ext;
  out.values.resize(total);
  for (int64_t i = 0; i < total; ++i) {
    const double dd = std::isfinite(g[i]) ? std::sqrt(g[i]) * cell : inf;
    const double s = dd - two_h - margin;
    out.values[i] = s > 0.0 ? float(s) * (1.0f - 1e-6f) : 0.0f;
  }
  for (int k = 0; k < 3; ++k) {
    out.n[k] = n[k];
    out.lo[k] = float(lo[k]);
  }
  out.inv_cell = float(1.0 / cell);
  return true;
}

}  // namespace xp
