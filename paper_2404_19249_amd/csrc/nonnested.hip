// Interpolation between nonnested meshes (Sec. 3.2, Algorithm 1): the value
// at a fine node of a function that is P1 on an unrelated coarse tetrahedral
// mesh.  For every point: a spatial search structure over the coarse
// vertices gives a nearby vertex, an element having that vertex starts a
// walk that moves, while some barycentric coordinate of the point is
// negative, to the neighbour across the face opposite that coordinate; the
// containing element's barycentric coordinates are the interpolation
// weights.  Per-mesh setup on the host (like the rest of the setup).
//
// Differences from the paper's FreeFEM form: the quadtree of vertices is a
// uniform grid of vertex buckets (the point's bucket, else the nearest
// non-empty shell); when several coordinates are negative the walk crosses
// the face of the most negative one (the paper picks one at random; the
// containing element, hence the interpolated value, does not depend on the
// path).  A point outside the coarse mesh (the walk reaches a boundary face)
// is projected onto the last element: negative coordinates are set to zero
// and the rest rescaled to sum 1.
#include "kernels.h"
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <unordered_map>
#include <vector>

namespace ks {

namespace {

struct FaceKey {
  int32_t a, b, c;
  bool operator==(const FaceKey &o) const { return a == o.a && b == o.b && c == o.c; }
};
struct FaceHash {
  size_t operator()(const FaceKey &k) const {
    uint64_t h = (uint64_t)(uint32_t)k.a * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)(uint32_t)k.b + 0x7F4A7C159E3779B9ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)(uint32_t)k.c + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

// barycentric coordinates of x in tetrahedron t (vertices v0..v3)
void barycentric(const double *cv, const int32_t *t, const double *x, double lam[4]) {
  const double *p0 = cv + 3 * (int64_t)t[0];
  double J[3][3], r[3];
  for (int d = 0; d < 3; ++d) {
    for (int j = 0; j < 3; ++j) J[d][j] = cv[3 * (int64_t)t[j + 1] + d] - p0[d];
    r[d] = x[d] - p0[d];
  }
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  // Cramer's rule for J l = r, l = (lambda_1, lambda_2, lambda_3)
  double l[3];
  for (int j = 0; j < 3; ++j) {
    double M[3][3];
    for (int d = 0; d < 3; ++d)
      for (int i = 0; i < 3; ++i) M[d][i] = (i == j) ? r[d] : J[d][i];
    l[j] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
            M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) /
           det;
  }
  lam[1] = l[0];
  lam[2] = l[1];
  lam[3] = l[2];
  lam[0] = 1.0 - l[0] - l[1] - l[2];
}

}  // namespace

int nonnested_weights(int ncv, const double *cv, int nct, const int32_t *ctet, int npts, const double *pts,
                      int32_t *vid, double *w) {
  if (ncv < 4 || nct < 1) return -1;
  // face adjacency: nbr[4 t + f] = element across the face opposite vertex f
  std::vector<int32_t> nbr((size_t)4 * nct, -1);
  {
    std::unordered_map<FaceKey, int64_t, FaceHash> open;
    open.reserve((size_t)2 * nct + 16);
    for (int t = 0; t < nct; ++t)
      for (int f = 0; f < 4; ++f) {
        int32_t v[3], n = 0;
        for (int j = 0; j < 4; ++j)
          if (j != f) v[n++] = ctet[4 * (int64_t)t + j];
        std::sort(v, v + 3);
        const FaceKey key{v[0], v[1], v[2]};
        auto it = open.find(key);
        if (it == open.end()) {
          open.emplace(key, 4 * (int64_t)t + f);
        } else {
          const int64_t o = it->second;
          nbr[4 * (size_t)t + f] = (int32_t)(o / 4);
          nbr[(size_t)o] = t;
          open.erase(it);
        }
      }
  }
  // one element per vertex
  std::vector<int32_t> vtet(ncv, -1);
  for (int t = 0; t < nct; ++t)
    for (int j = 0; j < 4; ++j) {
      const int32_t v = ctet[4 * (int64_t)t + j];
      if (v < 0 || v >= ncv) return -1;
      if (vtet[v] < 0) vtet[v] = t;
    }
  // uniform bucket grid over the vertices' bounding box, about one vertex per bucket
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int v = 0; v < ncv; ++v)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], cv[3 * (int64_t)v + d]);
      hi[d] = std::max(hi[d], cv[3 * (int64_t)v + d]);
    }
  const int G = std::max(1, (int)std::cbrt((double)ncv));
  double inv[3];
  for (int d = 0; d < 3; ++d) inv[d] = hi[d] > lo[d] ? G / (hi[d] - lo[d]) : 0.0;
  auto cell = [&](const double *x, int c[3]) {
    for (int d = 0; d < 3; ++d) c[d] = std::max(0, std::min(G - 1, (int)std::floor((x[d] - lo[d]) * inv[d])));
  };
  std::vector<int32_t> bstart((size_t)G * G * G + 1, 0), bverts(ncv);
  {
    std::vector<int32_t> bid(ncv);
    for (int v = 0; v < ncv; ++v) {
      int c[3];
      cell(cv + 3 * (int64_t)v, c);
      bid[v] = c[0] + G * (c[1] + G * c[2]);
      bstart[bid[v] + 1]++;
    }
    for (size_t b = 0; b + 1 < bstart.size(); ++b) bstart[b + 1] += bstart[b];
    std::vector<int32_t> pos(bstart.begin(), bstart.end() - 1);
    for (int v = 0; v < ncv; ++v) bverts[pos[bid[v]]++] = v;
  }
  const int max_steps = 64 + 64 * (int)std::cbrt((double)nct);
  int failures = 0;
  for (int p = 0; p < npts; ++p) {
    const double *x = pts + 3 * (int64_t)p;
    // nearest vertex among the buckets of the first non-empty shell around x
    int c[3];
    cell(x, c);
    int best = -1;
    double bd = 1e300;
    for (int r = 0; r <= G && best < 0; ++r)
      for (int k = c[2] - r; k <= c[2] + r; ++k)
        for (int j = c[1] - r; j <= c[1] + r; ++j)
          for (int i = c[0] - r; i <= c[0] + r; ++i) {
            if (i < 0 || j < 0 || k < 0 || i >= G || j >= G || k >= G) continue;
            if (std::max(std::abs(i - c[0]), std::max(std::abs(j - c[1]), std::abs(k - c[2]))) != r) continue;
            const int b = i + G * (j + G * k);
            for (int q = bstart[b]; q < bstart[b + 1]; ++q) {
              const int v = bverts[q];
              double dd = 0.0;
              for (int d = 0; d < 3; ++d) {
                const double e = cv[3 * (int64_t)v + d] - x[d];
                dd += e * e;
              }
              if (dd < bd) {
                bd = dd;
                best = v;
              }
            }
          }
    int t = vtet[best] >= 0 ? vtet[best] : 0;  // a vertex in no element: start anywhere
    double lam[4];
    barycentric(cv, ctet + 4 * (int64_t)t, x, lam);
    for (int step = 0; step < max_steps; ++step) {
      int f = 0;
      for (int j = 1; j < 4; ++j)
        if (lam[j] < lam[f]) f = j;
      if (lam[f] >= -1e-12) break;  // inside (up to rounding)
      const int tn = nbr[4 * (size_t)t + f];
      if (tn < 0) break;            // outside the coarse mesh: project below
      t = tn;
      barycentric(cv, ctet + 4 * (int64_t)t, x, lam);
    }
    double s = 0.0;
    for (int j = 0; j < 4; ++j) {
      if (lam[j] < 0.0) lam[j] = 0.0;
      s += lam[j];
    }
    if (!(s > 0.0)) {
      ++failures;
      s = 1.0;
    }
    for (int j = 0; j < 4; ++j) {
      vid[4 * (int64_t)p + j] = ctet[4 * (int64_t)t + j];
      w[4 * (int64_t)p + j] = lam[j] / s;
    }
  }
  return failures ? -2 : 0;
}

}  // namespace ks
