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

// search structures of a source mesh: face neighbours, one element per
// vertex, and a uniform bucket grid of the vertices (about one per bucket)
struct LocateIndex {
  std::vector<int32_t> nbr, vtet, bstart, bverts;
  double lo[3], inv[3];
  int G = 1, max_steps = 64;
};

static int build_locate_index(int ncv, const double *cv, int nct, const int32_t *ctet, LocateIndex &ix) {
  if (ncv < 4 || nct < 1) return -1;
  // face adjacency: nbr[4 t + f] = element across the face opposite vertex f
  std::vector<int32_t> &nbr = ix.nbr;
  nbr.assign((size_t)4 * nct, -1);
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
  std::vector<int32_t> &vtet = ix.vtet;
  vtet.assign(ncv, -1);
  for (int t = 0; t < nct; ++t)
    for (int j = 0; j < 4; ++j) {
      const int32_t v = ctet[4 * (int64_t)t + j];
      if (v < 0 || v >= ncv) return -1;
      if (vtet[v] < 0) vtet[v] = t;
    }
  // uniform bucket grid over the vertices' bounding box, about one vertex per bucket
  double hi[3] = {-1e300, -1e300, -1e300};
  for (int d = 0; d < 3; ++d) ix.lo[d] = 1e300;
  for (int v = 0; v < ncv; ++v)
    for (int d = 0; d < 3; ++d) {
      ix.lo[d] = std::min(ix.lo[d], cv[3 * (int64_t)v + d]);
      hi[d] = std::max(hi[d], cv[3 * (int64_t)v + d]);
    }
  const int G = std::max(1, (int)std::cbrt((double)ncv));
  ix.G = G;
  for (int d = 0; d < 3; ++d) ix.inv[d] = hi[d] > ix.lo[d] ? G / (hi[d] - ix.lo[d]) : 0.0;
  ix.bstart.assign((size_t)G * G * G + 1, 0);
  ix.bverts.resize(ncv);
  {
    std::vector<int32_t> bid(ncv);
    for (int v = 0; v < ncv; ++v) {
      int c[3];
      for (int d = 0; d < 3; ++d)
        c[d] = std::max(0, std::min(G - 1, (int)std::floor((cv[3 * (int64_t)v + d] - ix.lo[d]) * ix.inv[d])));
      bid[v] = c[0] + G * (c[1] + G * c[2]);
      ix.bstart[bid[v] + 1]++;
    }
    for (size_t b = 0; b + 1 < ix.bstart.size(); ++b) ix.bstart[b + 1] += ix.bstart[b];
    std::vector<int32_t> pos(ix.bstart.begin(), ix.bstart.end() - 1);
    for (int v = 0; v < ncv; ++v) ix.bverts[pos[bid[v]]++] = v;
  }
  ix.max_steps = 64 + 64 * (int)std::cbrt((double)nct);
  return 0;
}

int nonnested_weights(int ncv, const double *cv, int nct, const int32_t *ctet, int npts, const double *pts,
                      int32_t *vid, double *w) {
  LocateIndex ix;
  if (build_locate_index(ncv, cv, nct, ctet, ix) < 0) return -1;
  const std::vector<int32_t> &nbr = ix.nbr, &vtet = ix.vtet, &bstart = ix.bstart, &bverts = ix.bverts;
  const int G = ix.G;
  const double *lo = ix.lo, *inv = ix.inv;
  auto cell = [&](const double *x, int c[3]) {
    for (int d = 0; d < 3; ++d) c[d] = std::max(0, std::min(G - 1, (int)std::floor((x[d] - lo[d]) * inv[d])));
  };
  const int max_steps = ix.max_steps;
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

// The same search on the GPU, one thread per point: nearest vertex in the
// first non-empty shell of buckets, then the walk across the face opposite
// the most negative barycentric coordinate, projection onto the last
// element outside the mesh.  The index is built on the host.
__device__ void d_barycentric(const double *__restrict__ cv, const int32_t *__restrict__ t, const double *x,
                              double lam[4]) {
  const double *p0 = cv + 3 * (int64_t)t[0];
  double J[3][3], r[3];
  for (int d = 0; d < 3; ++d) {
    for (int j = 0; j < 3; ++j) J[d][j] = cv[3 * (int64_t)t[j + 1] + d] - p0[d];
    r[d] = x[d] - p0[d];
  }
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  double l[3];
  for (int j = 0; j < 3; ++j) {
    double M[3][3];
    for (int d = 0; d < 3; ++d)
      for (int q = 0; q < 3; ++q) M[d][q] = (q == j) ? r[d] : J[d][q];
    l[j] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
            M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) /
           det;
  }
  lam[1] = l[0];
  lam[2] = l[1];
  lam[3] = l[2];
  lam[0] = 1.0 - l[0] - l[1] - l[2];
}

struct LocateDev {
  const double *cv;
  const int32_t *tet, *nbr, *vtet, *bstart, *bverts;
  double lo[3], inv[3];
  int G, max_steps;
};

__global__ void k_locate(LocateDev ix, int npts, const double *__restrict__ pts, int32_t *__restrict__ vid,
                         double *__restrict__ w, int *__restrict__ failures) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const int G = ix.G;
  double x[3];
  int c[3];
  for (int d = 0; d < 3; ++d) {
    x[d] = pts[3 * (int64_t)p + d];
    c[d] = max(0, min(G - 1, (int)floor((x[d] - ix.lo[d]) * ix.inv[d])));
  }
  int best = -1;
  double bd = 1e300;
  for (int r = 0; r <= G && best < 0; ++r)
    for (int k = c[2] - r; k <= c[2] + r; ++k)
      for (int j = c[1] - r; j <= c[1] + r; ++j)
        for (int i = c[0] - r; i <= c[0] + r; ++i) {
          if (i < 0 || j < 0 || k < 0 || i >= G || j >= G || k >= G) continue;
          if (max(abs(i - c[0]), max(abs(j - c[1]), abs(k - c[2]))) != r) continue;
          const int b = i + G * (j + G * k);
          for (int q = ix.bstart[b]; q < ix.bstart[b + 1]; ++q) {
            const int v = ix.bverts[q];
            double dd = 0.0;
            for (int d = 0; d < 3; ++d) {
              const double e = ix.cv[3 * (int64_t)v + d] - x[d];
              dd += e * e;
            }
            if (dd < bd) {
              bd = dd;
              best = v;
            }
          }
        }
  int t = (best >= 0 && ix.vtet[best] >= 0) ? ix.vtet[best] : 0;
  double lam[4];
  d_barycentric(ix.cv, ix.tet + 4 * (int64_t)t, x, lam);
  for (int step = 0; step < ix.max_steps; ++step) {
    int f = 0;
    for (int j = 1; j < 4; ++j)
      if (lam[j] < lam[f]) f = j;
    if (lam[f] >= -1e-12) break;
    const int tn = ix.nbr[4 * (int64_t)t + f];
    if (tn < 0) break;
    t = tn;
    d_barycentric(ix.cv, ix.tet + 4 * (int64_t)t, x, lam);
  }
  double s = 0.0;
  for (int j = 0; j < 4; ++j) {
    if (lam[j] < 0.0) lam[j] = 0.0;
    s += lam[j];
  }
  if (!(s > 0.0)) {
    atomicAdd(failures, 1);
    s = 1.0;
  }
  for (int j = 0; j < 4; ++j) {
    vid[4 * (int64_t)p + j] = ix.tet[4 * (int64_t)t + j];
    w[4 * (int64_t)p + j] = lam[j] / s;
  }
}

int nonnested_weights_device(int ncv, const double *cv, int nct, const int32_t *ctet, int npts, const double *pts_dev,
                             int32_t *vid_dev, double *w_dev, hipStream_t s) {
  LocateIndex ix;
  if (build_locate_index(ncv, cv, nct, ctet, ix) < 0) return -1;
  if (npts <= 0) return 0;
  std::vector<void *> bufs;
  auto up = [&](const void *src, size_t bytes) -> void * {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 4)) != hipSuccess) return nullptr;
    bufs.push_back(p);
    if (hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return nullptr;
    return p;
  };
  const int zero = 0;
  LocateDev d{};
  d.cv = static_cast<const double *>(up(cv, sizeof(double) * 3 * (size_t)ncv));
  d.tet = static_cast<const int32_t *>(up(ctet, sizeof(int32_t) * 4 * (size_t)nct));
  d.nbr = static_cast<const int32_t *>(up(ix.nbr.data(), sizeof(int32_t) * ix.nbr.size()));
  d.vtet = static_cast<const int32_t *>(up(ix.vtet.data(), sizeof(int32_t) * ix.vtet.size()));
  d.bstart = static_cast<const int32_t *>(up(ix.bstart.data(), sizeof(int32_t) * ix.bstart.size()));
  d.bverts = static_cast<const int32_t *>(up(ix.bverts.data(), sizeof(int32_t) * ix.bverts.size()));
  int *fail = static_cast<int *>(up(&zero, sizeof(int)));
  int rc = 0, hfail = 0;
  if (!d.cv || !d.tet || !d.nbr || !d.vtet || !d.bstart || !d.bverts || !fail) {
    rc = -3;
  } else {
    for (int k = 0; k < 3; ++k) {
      d.lo[k] = ix.lo[k];
      d.inv[k] = ix.inv[k];
    }
    d.G = ix.G;
    d.max_steps = ix.max_steps;
    hipLaunchKernelGGL(k_locate, dim3((npts + 255) / 256), dim3(256), 0, s, d, npts, pts_dev, vid_dev, w_dev, fail);
    if (hipMemcpyAsync(&hfail, fail, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = -4;
    else if (hfail)
      rc = -2;
  }
  for (void *p : bufs) (void)hipFree(p);
  return rc;
}

// pts[node2int[v]] = coords[v] for the interior nodes v
__global__ void k_interior_coords(int nn, const int32_t *__restrict__ node2int, const double *__restrict__ coords,
                                  double *__restrict__ pts) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  const int r = node2int[v];
  if (r >= 0)
    for (int d = 0; d < 3; ++d) pts[3 * (int64_t)r + d] = coords[3 * (int64_t)v + d];
}
void launch_interior_coords(int nn, const int32_t *node2int, const double *coords, double *pts, hipStream_t s) {
  if (nn > 0) hipLaunchKernelGGL(k_interior_coords, dim3((nn + 255) / 256), dim3(256), 0, s, nn, node2int, coords, pts);
}
// ELL form over a source mesh's unknowns: idx = sint[vid] (-1 and weight 0
// for source nodes without an unknown)
__global__ void k_ell_from_vertices(int64_t n4, const int32_t *__restrict__ vid, const double *__restrict__ w,
                                    const int32_t *__restrict__ sint, int32_t *__restrict__ idx,
                                    double *__restrict__ wo) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n4) return;
  const int u = sint[vid[i]];
  const bool keep = u >= 0 && w[i] != 0.0;
  idx[i] = keep ? u : -1;
  wo[i] = keep ? w[i] : 0.0;
}
void launch_ell_from_vertices(int npts, const int32_t *vid, const double *w, const int32_t *sint, int32_t *idx,
                              double *wo, hipStream_t s) {
  const int64_t n4 = (int64_t)npts * 4;
  if (n4 > 0)
    hipLaunchKernelGGL(k_ell_from_vertices, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, n4, vid, w, sint,
                       idx, wo);
}

}  // namespace ks
