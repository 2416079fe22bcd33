// Multigrid-preconditioned CG for the Hartree Poisson problem K_II v = f.
//
// The paper solves its Poisson and boundary value problems with
// algebraic-multigrid-preconditioned Krylov methods (PETSc GAMG).  Here the
// coarse spaces are the P1 spaces of uniform Kuhn (Freudenthal) meshes of the
// same box, each with half the cells per side of the level above; the
// interpolation of a level's nodes into the next coarser mesh is closed-form
// point location (the coarse tetrahedron containing a point follows from the
// ordering of its cell-local coordinates), which is exact for nested uniform
// levels and a smooth (non-nested) transfer from the moved fine mesh.  Coarse
// operators are Galerkin products A_l = P_l^T A_{l-1} P_l, formed once per
// mesh on the host; the coarsest (at most 512 unknowns) is inverted densely.
//
// Preconditioner: one symmetric V-cycle with Chebyshev smoothing (degree 2,
// Jacobi-scaled, interval [lambda_max / 8, 1.1 lambda_max] of D^-1 A from a
// power iteration), the same polynomial before and after the coarse
// correction, so the preconditioner is symmetric positive definite.
#include "common.h"
#include "kernels.h"
#include <algorithm>
#include <cstring>
#include <climits>
#include <cmath>
#include <thread>
#include <vector>

namespace ks {

namespace {

template <typename F>
void par_for(int64_t n, F f) {
  const int nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 4096 || nt == 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([=]() {
      for (int64_t i = a; i < b; ++i) f(i);
    });
  }
  for (auto &x : th) x.join();
}

struct HostCSR {
  int n = 0, m = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> v;
};

// y = A x
void host_spmv(const HostCSR &A, const std::vector<double> &x, std::vector<double> &y) {
  y.assign(A.n, 0.0);
  par_for(A.n, [&](int64_t i) {
    double s = 0.0;
    for (int j = A.rp[i]; j < A.rp[i + 1]; ++j) s += A.v[j] * x[A.ci[j]];
    y[i] = s;
  });
}

// C = P^T A P with P given as ELL-4 (idx -1 = unused), A square n x n, P n x nc
HostCSR galerkin(const HostCSR &A, const std::vector<int32_t> &Pi, const std::vector<double> &Pw, int nc) {
  const int n = A.n;
  // AP row by row (sparse, coarse columns)
  std::vector<std::vector<std::pair<int32_t, double>>> AP(n);
  par_for(n, [&](int64_t i) {
    std::vector<std::pair<int32_t, double>> &row = AP[i];
    for (int j = A.rp[i]; j < A.rp[i + 1]; ++j) {
      const int c = A.ci[j];
      for (int t = 0; t < 4; ++t)
        if (Pi[4 * (size_t)c + t] >= 0) row.push_back({Pi[4 * (size_t)c + t], A.v[j] * Pw[4 * (size_t)c + t]});
    }
    std::sort(row.begin(), row.end(), [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
      return a.first < b.first;
    });
    size_t o = 0;
    for (size_t t = 0; t < row.size(); ++t) {
      if (o > 0 && row[o - 1].first == row[t].first) row[o - 1].second += row[t].second;
      else row[o++] = row[t];
    }
    row.resize(o);
  });
  // transpose of P: coarse row -> (fine row, weight)
  std::vector<int32_t> tp(nc + 1, 0);
  for (int i = 0; i < n; ++i)
    for (int t = 0; t < 4; ++t)
      if (Pi[4 * (size_t)i + t] >= 0) tp[Pi[4 * (size_t)i + t] + 1]++;
  for (int a = 0; a < nc; ++a) tp[a + 1] += tp[a];
  std::vector<int32_t> tf(tp[nc]);
  std::vector<double> tw(tp[nc]);
  {
    std::vector<int32_t> pos(tp.begin(), tp.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int t = 0; t < 4; ++t) {
        const int a = Pi[4 * (size_t)i + t];
        if (a >= 0) {
          tf[pos[a]] = i;
          tw[pos[a]++] = Pw[4 * (size_t)i + t];
        }
      }
  }
  // C rows: sum over fine rows i of P_ia * AP_i
  std::vector<std::vector<std::pair<int32_t, double>>> C(nc);
  par_for(nc, [&](int64_t a) {
    std::vector<std::pair<int32_t, double>> acc;
    for (int t = tp[a]; t < tp[a + 1]; ++t) {
      const double w = tw[t];
      for (const auto &e : AP[tf[t]]) acc.push_back({e.first, w * e.second});
    }
    std::sort(acc.begin(), acc.end(), [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
      return x.first < y.first;
    });
    size_t o = 0;
    for (size_t u = 0; u < acc.size(); ++u) {
      if (o > 0 && acc[o - 1].first == acc[u].first) acc[o - 1].second += acc[u].second;
      else acc[o++] = acc[u];
    }
    acc.resize(o);
    C[a].swap(acc);
  });
  HostCSR out;
  out.n = out.m = nc;
  out.rp.assign(nc + 1, 0);
  for (int a = 0; a < nc; ++a) out.rp[a + 1] = out.rp[a] + (int32_t)C[a].size();
  out.ci.resize(out.rp[nc]);
  out.v.resize(out.rp[nc]);
  par_for(nc, [&](int64_t a) {
    int o = out.rp[a];
    for (const auto &e : C[a]) {
      out.ci[o] = e.first;
      out.v[o++] = e.second;
    }
  });
  return out;
}

// largest eigenvalue of D^-1 A (power iteration from a fixed start)
double lambda_max_jacobi(const HostCSR &A) {
  std::vector<double> d(A.n, 1.0), x(A.n), y;
  for (int i = 0; i < A.n; ++i) {
    for (int j = A.rp[i]; j < A.rp[i + 1]; ++j)
      if (A.ci[j] == i) d[i] = A.v[j];
    x[i] = 1.0 + 0.37 * std::sin(0.91 * i);  // deterministic, not an eigenvector
  }
  double lam = 1.0;
  for (int it = 0; it < 20; ++it) {
    host_spmv(A, x, y);
    double nx = 0.0, ny = 0.0, xy = 0.0;
    for (int i = 0; i < A.n; ++i) {
      y[i] /= d[i];
      nx += x[i] * x[i];
      xy += x[i] * y[i];
      ny += y[i] * y[i];
    }
    lam = xy / nx;
    const double s = 1.0 / std::sqrt(ny);
    for (int i = 0; i < A.n; ++i) x[i] = y[i] * s;
  }
  return lam;
}

}  // namespace

// point location in the uniform Kuhn mesh of [-L, L]^3 with nH cells per
// side: the (up to 4) interior vertices of the tetrahedron containing x and
// their barycentric weights; vertex id = (i-1) + ni ((j-1) + ni (k-1)),
// ni = nH - 1; boundary vertices are dropped (zero Dirichlet values).
void kuhn_interp(const double *x, double L, int nH, int32_t *idx, double *w) {
  const int ni = nH - 1;
  const double h = 2.0 * L / nH;
  int cell[3];
  double xi[3];
  for (int d = 0; d < 3; ++d) {
    const double t = (x[d] + L) / h;
    int ci = (int)std::floor(t);
    ci = std::max(0, std::min(nH - 1, ci));
    cell[d] = ci;
    xi[d] = std::min(1.0, std::max(0.0, t - ci));
  }
  int ord[3] = {0, 1, 2};
  std::sort(ord, ord + 3, [&](int a, int b) { return xi[a] > xi[b] || (xi[a] == xi[b] && a < b); });
  const double lam[4] = {1.0 - xi[ord[0]], xi[ord[0]] - xi[ord[1]], xi[ord[1]] - xi[ord[2]], xi[ord[2]]};
  int v[3] = {cell[0], cell[1], cell[2]};
  int cnt = 0;
  for (int t = 0; t < 4; ++t) idx[t] = -1, w[t] = 0.0;
  for (int j = 0; j < 4; ++j) {
    if (j > 0) v[ord[j - 1]] += 1;
    bool inner = true;
    for (int d = 0; d < 3; ++d)
      if (v[d] <= 0 || v[d] >= nH) inner = false;
    if (!inner || lam[j] == 0.0) continue;
    idx[cnt] = (v[0] - 1) + ni * ((v[1] - 1) + ni * (v[2] - 1));
    w[cnt] = lam[j];
    ++cnt;
  }
}

// ------------------------------------------------------------ device
__global__ void k_cheb(int n, const double *__restrict__ r, const double *__restrict__ dinv, double c1,
                       double c2, double *__restrict__ d, double *__restrict__ x, int first) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double di = (first ? 0.0 : c1 * d[i]) + c2 * dinv[i] * r[i];
    d[i] = di;
    x[i] = (first == 2 ? 0.0 : x[i]) + di;
  }
}
static void launch_cheb(int n, const double *r, const double *dinv, double c1, double c2, double *d,
                        double *x, int first, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_cheb, dim3(std::min(4096, (n + 255) / 256)), dim3(256), 0, s, n, r, dinv, c1, c2, d,
                       x, first);
}
// the Chebyshev update in FP32
__global__ void k_cheb32(int n, const float *__restrict__ r, const float *__restrict__ dinv, float c1, float c2,
                         float *__restrict__ d, float *__restrict__ x, int first) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float di = (first ? 0.0f : c1 * d[i]) + c2 * dinv[i] * r[i];
    d[i] = di;
    x[i] = (first == 2 ? 0.0f : x[i]) + di;
  }
}
static void launch_cheb32(int n, const float *r, const float *dinv, double c1, double c2, float *d, float *x,
                          int first, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_cheb32, dim3(std::min(4096, (n + 255) / 256)), dim3(256), 0, s, n, r, dinv, (float)c1,
                       (float)c2, d, x, first);
}
__global__ void k_f2d(int n, const float *__restrict__ a, double *__restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = (double)a[i];
}
// x32 += P xc (P: ELL-4 interpolation from the next coarser level)
__global__ void k_prolong_add32(int n, const int32_t *__restrict__ Pidx, const double *__restrict__ Pw,
                                const double *__restrict__ xc, float *__restrict__ x) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int c = 0; c < 4; ++c) {
      const int id = Pidx[4 * (int64_t)i + c];
      if (id >= 0) v += Pw[4 * (int64_t)i + c] * xc[id];
    }
    x[i] += (float)v;
  }
}
__global__ void k_invert(int n, const double *__restrict__ a, double *__restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = 1.0 / a[i];
}

// x = G b for the dense n x n matrix G (row-major): one wavefront per row,
// lanes striding the row (coalesced), butterfly sum across the wavefront
__global__ void __launch_bounds__(256) k_dense_matvec(int n, const double *__restrict__ G,
                                                     const double *__restrict__ b, double *__restrict__ x) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;
  const double *g = G + (int64_t)row * n;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += g[j] * b[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) x[row] = s;
}

// y = A x (b null) or y = b - A x for a matrix in column-major ELL form
// ([w][n]: entry j of row i at j n + i, in the row's CSR order, padding with
// value 0): one row per lane, so that the index, value and (on a lattice)
// vector loads of a wavefront are coalesced; fixed summation order
__global__ void __launch_bounds__(256) k_ell_spmv(int n, int w, const int32_t *__restrict__ col,
                                                 const double *__restrict__ val, const double *__restrict__ x,
                                                 const double *__restrict__ b, double *__restrict__ y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double acc = 0.0;
#pragma unroll 4
    for (int j = 0; j < w; ++j) acc += val[(int64_t)j * n + i] * x[col[(int64_t)j * n + i]];
    y[i] = b ? b[i] - acc : acc;
  }
}
static void launch_ell_spmv(int n, int w, const int32_t *col, const double *val, const double *x, const double *b,
                            double *y, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_ell_spmv, dim3(std::min(4096, (n + 255) / 256)), dim3(256), 0, s, n, w, col, val, x, b, y);
}
// column-major ELL copy of a host CSR matrix with n rows (padding: column 0,
// value 0); false when a row is longer than max_w
static bool to_ell(int n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                   const std::vector<double> &v, int max_w, int &w, std::vector<int32_t> &ec,
                   std::vector<double> &ev) {
  w = 0;
  for (int i = 0; i < n; ++i) w = std::max(w, rp[i + 1] - rp[i]);
  if (w > max_w || w == 0) return false;
  ec.assign((size_t)w * n, 0);
  ev.assign((size_t)w * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = rp[i]; j < rp[i + 1]; ++j) {
      ec[(size_t)(j - rp[i]) * n + i] = ci[j];
      ev[(size_t)(j - rp[i]) * n + i] = v[j];
    }
  return true;
}
constexpr int ELL_MAX_W = 64;

struct MGLevel {
  int n = 0;
  const int32_t *rp = nullptr, *ci = nullptr;  // operator (level 0: the context's CSR)
  const double *val = nullptr;
  // the operator in ELL form on the coarse levels (aw = 0: not built), and
  // the restriction to the next level in ELL form (rw = 0: CSR only)
  int aw = 0, rw = 0;
  int32_t *acol = nullptr, *rcol = nullptr;
  double *aval = nullptr, *rval = nullptr;
  double *dinv = nullptr;
  double lmax = 2.0;
  // transfer to the next coarser level: restriction R = P^T (CSR, rows =
  // coarse nodes) and prolongation P (ELL-4, rows = this level's nodes)
  int32_t *Rrp = nullptr, *Rci = nullptr, *Pidx = nullptr;
  double *Rv = nullptr, *Pw = nullptr;
  double *b = nullptr, *x = nullptr, *r = nullptr, *d = nullptr;
};

struct Multigrid {
  std::vector<MGLevel> lv;
  const Tiling *til0 = nullptr;  // halo tiles of the level-0 operator (nullptr: row kernel)
  int tb0 = 256;
  double *coarse_inv = nullptr;  // dense inverse of the coarsest operator
  double *pr = nullptr, *pz = nullptr, *pp = nullptr, *pq = nullptr;  // PCG vectors (level 0)
  // FP32 smoothing on level 0 (the V-cycle is a preconditioner; the outer
  // CG stays FP64): operator values, 1/diag and the level's vectors in FP32
  bool f32 = false;
  float *val32 = nullptr, *dinv32 = nullptr, *x32 = nullptr, *r32 = nullptr, *d32 = nullptr, *b32 = nullptr;
  std::vector<void *> mem;
  ~Multigrid() {
    for (void *p : mem) (void)hipFree(p);
  }
  template <typename T>
  bool alloc(T **p, size_t n) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n * sizeof(T), 256)) != hipSuccess) return false;
    mem.push_back(q);
    *p = reinterpret_cast<T *>(q);
    return true;
  }
};

void mg_destroy(Multigrid *mg) { delete mg; }
void mg_set_tiling(Multigrid *mg, const Tiling *til0, int tb0) {
  if (mg) {
    mg->til0 = til0;
    mg->tb0 = tb0;
    // the FP32 level 0 needs halo tiles that serve one FP32 column
    if (mg->val32) mg->f32 = til0 && tiled_fits_f32(mg->lv[0].n, 1, *til0, tb0);
  }
}
int mg_levels(const Multigrid *mg) { return mg ? (int)mg->lv.size() : 0; }

// Build the hierarchy.  Level 0 is the given operator (device CSR plus its
// host copy for the Galerkin products); coords: the level-0 unknowns'
// coordinates [n][3]; L: half side of the box; n1: cells per side of the
// first uniform coarse level (after `first`, when given).  Returns nullptr
// when no coarse level fits.
Multigrid *mg_build(int n0, const int32_t *rp_d, const int32_t *ci_d, const double *val_d, const Tiling *til0,
                    int tb0,
                    const std::vector<int32_t> &rp_h, const std::vector<int32_t> &ci_h,
                    const std::vector<double> &val_h, const std::vector<double> &coords, double L, int n1,
                    hipStream_t s, const MGFirst *first) {
  if (n1 < 2) return nullptr;
  Multigrid *mg = new Multigrid();
  mg->til0 = til0;
  mg->tb0 = tb0;
  auto bail = [&]() {
    delete mg;
    return (Multigrid *)nullptr;
  };
  HostCSR A;
  A.n = A.m = n0;
  A.rp = rp_h;
  A.ci = ci_h;
  A.v = val_h;
  std::vector<double> X = coords;  // this level's node coordinates
  int n_cells = n1;
  {
    MGLevel l0;
    l0.n = n0;
    l0.rp = rp_d;
    l0.ci = ci_d;
    l0.val = val_d;
    mg->lv.push_back(l0);
  }
  std::vector<HostCSR> ops;
  ops.push_back(A);
  bool use_first = first && first->nc > 0 && first->Pi.size() == (size_t)n0 * 4 &&
                   first->Pw.size() == (size_t)n0 * 4 && first->X.size() == (size_t)first->nc * 3;
  while (true) {
    MGLevel &f = mg->lv.back();
    const HostCSR &Af = ops.back();
    f.lmax = lambda_max_jacobi(Af);
    const bool from_first = use_first;
    const int ni = n_cells - 1;
    const int nc = from_first ? first->nc : ni * ni * ni;
    if (nc < 1) break;
    // interpolation of this level's nodes from the coarse mesh
    std::vector<int32_t> Pi((size_t)f.n * 4);
    std::vector<double> Pw((size_t)f.n * 4);
    if (from_first) {
      Pi = first->Pi;
      Pw = first->Pw;
    } else {
      par_for(f.n, [&](int64_t i) { kuhn_interp(&X[3 * i], L, n_cells, &Pi[4 * i], &Pw[4 * i]); });
    }
    HostCSR Ac = galerkin(Af, Pi, Pw, nc);
    // a coarse node no fine node interpolates from leaves a zero row: the
    // hierarchy is then unusable (the caller keeps the Jacobi-PCG solver)
    for (int a = 0; a < nc; ++a) {
      bool has = false;
      for (int j = Ac.rp[a]; j < Ac.rp[a + 1]; ++j) has = has || (Ac.ci[j] == a && Ac.v[j] > 0.0);
      if (!has) return bail();
    }
    // restriction CSR = P^T
    std::vector<int32_t> Rrp(nc + 1, 0), Rci;
    std::vector<double> Rv;
    for (int i = 0; i < f.n; ++i)
      for (int t = 0; t < 4; ++t)
        if (Pi[4 * (size_t)i + t] >= 0) Rrp[Pi[4 * (size_t)i + t] + 1]++;
    for (int a = 0; a < nc; ++a) Rrp[a + 1] += Rrp[a];
    Rci.resize(Rrp[nc]);
    Rv.resize(Rrp[nc]);
    {
      std::vector<int32_t> pos(Rrp.begin(), Rrp.end() - 1);
      for (int i = 0; i < f.n; ++i)
        for (int t = 0; t < 4; ++t) {
          const int a = Pi[4 * (size_t)i + t];
          if (a >= 0) {
            Rci[pos[a]] = i;
            Rv[pos[a]++] = Pw[4 * (size_t)i + t];
          }
        }
    }
    if (!mg->alloc(&f.Rrp, nc + 1) || !mg->alloc(&f.Rci, Rci.size()) || !mg->alloc(&f.Rv, Rv.size()) ||
        !mg->alloc(&f.Pidx, Pi.size()) || !mg->alloc(&f.Pw, Pw.size()))
      return bail();
    if (hipMemcpyAsync(f.Rrp, Rrp.data(), sizeof(int32_t) * (nc + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(f.Rci, Rci.data(), sizeof(int32_t) * Rci.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(f.Rv, Rv.data(), sizeof(double) * Rv.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(f.Pidx, Pi.data(), sizeof(int32_t) * Pi.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(f.Pw, Pw.data(), sizeof(double) * Pw.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return bail();
    {
      std::vector<int32_t> ec;
      std::vector<double> ev;
      int w = 0;
      if (to_ell(nc, Rrp, Rci, Rv, ELL_MAX_W, w, ec, ev)) {
        if (!mg->alloc(&f.rcol, ec.size()) || !mg->alloc(&f.rval, ev.size())) return bail();
        if (hipMemcpyAsync(f.rcol, ec.data(), sizeof(int32_t) * ec.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(f.rval, ev.data(), sizeof(double) * ev.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return bail();
        f.rw = w;
      }
    }
    // the coarse level
    MGLevel cl;
    cl.n = nc;
    int32_t *crp, *cci;
    double *cv;
    if (!mg->alloc(&crp, nc + 1) || !mg->alloc(&cci, Ac.ci.size()) || !mg->alloc(&cv, Ac.v.size())) return bail();
    if (hipMemcpyAsync(crp, Ac.rp.data(), sizeof(int32_t) * (nc + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(cci, Ac.ci.data(), sizeof(int32_t) * Ac.ci.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(cv, Ac.v.data(), sizeof(double) * Ac.v.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return bail();
    cl.rp = crp;
    cl.ci = cci;
    cl.val = cv;
    {
      std::vector<int32_t> ec;
      std::vector<double> ev;
      int w = 0;
      if (to_ell(nc, Ac.rp, Ac.ci, Ac.v, ELL_MAX_W, w, ec, ev)) {
        if (!mg->alloc(&cl.acol, ec.size()) || !mg->alloc(&cl.aval, ev.size())) return bail();
        if (hipMemcpyAsync(cl.acol, ec.data(), sizeof(int32_t) * ec.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(cl.aval, ev.data(), sizeof(double) * ev.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return bail();
        cl.aw = w;
      }
    }
    // node coordinates of the coarse level (the given level's, else the
    // interior lattice vertices)
    std::vector<double> Xc((size_t)nc * 3);
    if (from_first) {
      Xc = first->X;
    } else {
      const double h = 2.0 * L / n_cells;
      for (int kz = 0; kz < ni; ++kz)
        for (int jy = 0; jy < ni; ++jy)
          for (int ix = 0; ix < ni; ++ix) {
            const size_t a = ix + (size_t)ni * (jy + (size_t)ni * kz);
            Xc[3 * a] = -L + h * (ix + 1);
            Xc[3 * a + 1] = -L + h * (jy + 1);
            Xc[3 * a + 2] = -L + h * (kz + 1);
          }
    }
    mg->lv.push_back(cl);
    ops.push_back(std::move(Ac));
    X.swap(Xc);
    if (from_first) {
      use_first = false;
      if (nc <= 512 || n_cells < 2) break;
      continue;  // the uniform levels start at n_cells
    }
    if (nc <= 512 || n_cells < 4) break;  // coarsest: dense
    n_cells /= 2;
  }
  if (mg->lv.size() < 2) return bail();
  // dense inverse of the coarsest operator
  {
    const HostCSR &Ac = ops.back();
    const int n = Ac.n;
    std::vector<double> G((size_t)n * n, 0.0), I((size_t)n * n, 0.0);
    for (int a = 0; a < n; ++a)
      for (int j = Ac.rp[a]; j < Ac.rp[a + 1]; ++j) G[(size_t)a * n + Ac.ci[j]] = Ac.v[j];
    for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
    for (int p = 0; p < n; ++p) {
      int piv = p;
      for (int r = p + 1; r < n; ++r)
        if (std::fabs(G[(size_t)r * n + p]) > std::fabs(G[(size_t)piv * n + p])) piv = r;
      if (!(std::fabs(G[(size_t)piv * n + p]) > 0.0)) return bail();
      if (piv != p)
        for (int j = 0; j < n; ++j) {
          std::swap(G[(size_t)p * n + j], G[(size_t)piv * n + j]);
          std::swap(I[(size_t)p * n + j], I[(size_t)piv * n + j]);
        }
      const double dd = 1.0 / G[(size_t)p * n + p];
      for (int j = 0; j < n; ++j) {
        G[(size_t)p * n + j] *= dd;
        I[(size_t)p * n + j] *= dd;
      }
      for (int r = 0; r < n; ++r) {
        if (r == p) continue;
        const double fct = G[(size_t)r * n + p];
        if (fct == 0.0) continue;
        for (int j = 0; j < n; ++j) {
          G[(size_t)r * n + j] -= fct * G[(size_t)p * n + j];
          I[(size_t)r * n + j] -= fct * I[(size_t)p * n + j];
        }
      }
    }
    if (!mg->alloc(&mg->coarse_inv, (size_t)n * n)) return bail();
    if (hipMemcpyAsync(mg->coarse_inv, I.data(), sizeof(double) * n * n, hipMemcpyHostToDevice, s) != hipSuccess)
      return bail();
  }
  // work vectors and inverse diagonals
  if (!mg->alloc(&mg->pr, n0) || !mg->alloc(&mg->pz, n0) || !mg->alloc(&mg->pp, n0) || !mg->alloc(&mg->pq, n0))
    return bail();
  for (size_t l = 0; l < mg->lv.size(); ++l) {
    MGLevel &v = mg->lv[l];
    if (!mg->alloc(&v.b, v.n) || !mg->alloc(&v.x, v.n) || !mg->alloc(&v.r, v.n) || !mg->alloc(&v.d, v.n) ||
        !mg->alloc(&v.dinv, v.n))
      return bail();
    std::vector<double> dh(v.n, 1.0);
    const HostCSR &Al = ops[l];
    for (int i = 0; i < Al.n; ++i)
      for (int j = Al.rp[i]; j < Al.rp[i + 1]; ++j)
        if (Al.ci[j] == i) dh[i] = 1.0 / Al.v[j];
    if (hipMemcpyAsync(v.dinv, dh.data(), sizeof(double) * v.n, hipMemcpyHostToDevice, s) != hipSuccess)
      return bail();
  }
  {
    // FP32 level 0 (smoothing and residuals of the finest level)
    const int64_t nnz0 = rp_h[n0];
    if (nnz0 > 0 && nnz0 < INT32_MAX) {
      MGLevel &v0 = mg->lv[0];
      if (mg->alloc(&mg->val32, (size_t)nnz0 + 8) && mg->alloc(&mg->dinv32, n0) && mg->alloc(&mg->x32, n0) &&
          mg->alloc(&mg->r32, n0) && mg->alloc(&mg->d32, n0) && mg->alloc(&mg->b32, n0)) {
        launch_to_float(nnz0, val_d, mg->val32, s);
        launch_to_float(n0, v0.dinv, mg->dinv32, s);
        mg->f32 = til0 && tiled_fits_f32(n0, 1, *til0, tb0);
      }
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess) return bail();
  return mg;
}

// y = A x (b null) or y = b - A x on one level (halo tiles on level 0)
static void lv_spmv(const Multigrid *mg, const MGLevel &v, const double *x, double *y, const double *b,
                    hipStream_t s) {
  if (v.aw > 0) {
    launch_ell_spmv(v.n, v.aw, v.acol, v.aval, x, b, y, s);
    return;
  }
  if (&v == &mg->lv[0] && mg->til0 &&
      launch_spmm_tiled(v.n, 1, *mg->til0, mg->tb0, v.rp, v.val, x, y, b, s) == 0)
    return;
  launch_spmm(v.n, v.rp, v.ci, v.val, x, 1, y, 1, 1, b, 1, b ? 1 : 0, nullptr, s);
}

// Chebyshev smoothing of degree MG_CHEB_DEG on the Jacobi-scaled operator,
// targeting [lmax / 8, 1.1 lmax]: d_1 = D^-1 r_0 / theta, then
// d_j = rho_j rho_{j-1} d_{j-1} + (2 rho_j / delta) D^-1 r_{j-1} with
// rho_1 = 1 / sigma, rho_j = 1 / (2 sigma - rho_{j-1}); x += d_j each step
constexpr int MG_CHEB_DEG = 2;
struct ChebCoef {
  double theta, delta, sigma;
};
static ChebCoef cheb_coef(double lmax) {
  const double lo = lmax / 8.0, hi = 1.1 * lmax;
  ChebCoef c;
  c.theta = 0.5 * (hi + lo);
  c.delta = 0.5 * (hi - lo);
  c.sigma = c.theta / c.delta;
  return c;
}
// smoothing of A x = b on level l; zero_init: x = 0 in
static void mg_smooth(const Multigrid *mg, MGLevel &v, const double *b, bool zero_init, hipStream_t s) {
  const ChebCoef cc = cheb_coef(v.lmax);
  if (zero_init) {
    launch_cheb(v.n, b, v.dinv, 0.0, 1.0 / cc.theta, v.d, v.x, 2, s);
  } else {
    lv_spmv(mg, v, v.x, v.r, b, s);
    launch_cheb(v.n, v.r, v.dinv, 0.0, 1.0 / cc.theta, v.d, v.x, 1, s);
  }
  double rho_prev = 1.0 / cc.sigma;
  for (int j = 1; j < MG_CHEB_DEG; ++j) {
    const double rho = 1.0 / (2.0 * cc.sigma - rho_prev);
    lv_spmv(mg, v, v.x, v.r, b, s);  // r = b - A x
    launch_cheb(v.n, v.r, v.dinv, rho * rho_prev, 2.0 * rho / cc.delta, v.d, v.x, 0, s);
    rho_prev = rho;
  }
}

static void vcycle(Multigrid *mg, int l, const double *b, double *x, hipStream_t s);

// b_c = R r = P^T r from level v to the next coarser level c
static void restrict_to(const MGLevel &v, MGLevel &c, hipStream_t s) {
  if (v.rw > 0) launch_ell_spmv(c.n, v.rw, v.rcol, v.rval, v.r, nullptr, c.b, s);
  else launch_spmm(c.n, v.Rrp, v.Rci, v.Rv, v.r, 1, c.b, 1, 1, nullptr, 0, 0, nullptr, s);
}

// r32 = b32 - A x32 on level 0 (FP32 halo tiles); false if they cannot serve
static bool spmv0_f32(const Multigrid *mg, hipStream_t s) {
  const MGLevel &v = mg->lv[0];
  return mg->til0 &&
         launch_spmm_tiled_f32(v.n, 1, *mg->til0, mg->tb0, v.rp, mg->val32, mg->x32, mg->r32, mg->b32, s) == 0;
}

// The V-cycle with level 0 smoothed in FP32: the same Chebyshev steps as
// mg_smooth, the residual restricted and the correction prolonged through
// FP64 coarse levels
static void vcycle0_f32(Multigrid *mg, const double *b, double *x, hipStream_t s) {
  MGLevel &v = mg->lv[0];
  const int n = v.n;
  const ChebCoef cc = cheb_coef(v.lmax);
  const int g = std::min(4096, (n + 255) / 256);
  auto cheb_rest = [&]() {  // steps 2 .. MG_CHEB_DEG after the first
    double rho_prev = 1.0 / cc.sigma;
    for (int j = 1; j < MG_CHEB_DEG; ++j) {
      const double rho = 1.0 / (2.0 * cc.sigma - rho_prev);
      spmv0_f32(mg, s);
      launch_cheb32(n, mg->r32, mg->dinv32, rho * rho_prev, 2.0 * rho / cc.delta, mg->d32, mg->x32, 0, s);
      rho_prev = rho;
    }
  };
  launch_to_float(n, b, mg->b32, s);
  // pre-smoothing from zero
  launch_cheb32(n, mg->b32, mg->dinv32, 0.0, 1.0 / cc.theta, mg->d32, mg->x32, 2, s);
  cheb_rest();
  // residual to the next level
  spmv0_f32(mg, s);
  hipLaunchKernelGGL(k_f2d, dim3(g), dim3(256), 0, s, n, mg->r32, v.r);
  MGLevel &c = mg->lv[1];
  restrict_to(v, c, s);  // b_c = P^T r
  vcycle(mg, 1, c.b, c.x, s);
  hipLaunchKernelGGL(k_prolong_add32, dim3(g), dim3(256), 0, s, n, v.Pidx, v.Pw, c.x, mg->x32);
  // post-smoothing
  spmv0_f32(mg, s);
  launch_cheb32(n, mg->r32, mg->dinv32, 0.0, 1.0 / cc.theta, mg->d32, mg->x32, 1, s);
  cheb_rest();
  hipLaunchKernelGGL(k_f2d, dim3(g), dim3(256), 0, s, n, mg->x32, x);
}

// one V-cycle: x_0 = M^-1 b_0 on level 0 (b, x: level-0 vectors)
static void vcycle(Multigrid *mg, int l, const double *b, double *x, hipStream_t s) {
  if (l == 0 && mg->f32 && mg->lv.size() > 1) {
    vcycle0_f32(mg, b, x, s);
    return;
  }
  MGLevel &v = mg->lv[l];
  if (l + 1 == (int)mg->lv.size()) {
    hipLaunchKernelGGL(k_dense_matvec, dim3((v.n + 3) / 4), dim3(256), 0, s, v.n, mg->coarse_inv, b, x);
    return;
  }
  double *xs = v.x;
  v.x = x;  // smooth in place in the caller's vector
  mg_smooth(mg, v, b, true, s);
  lv_spmv(mg, v, v.x, v.r, b, s);  // r = b - A x
  MGLevel &c = mg->lv[l + 1];
  restrict_to(v, c, s);  // b_c = P^T r
  vcycle(mg, l + 1, c.b, c.x, s);
  launch_ellP_times(v.n, v.Pidx, v.Pw, c.x, 1, 1, 1.0, v.x, 1, v.x, 1, s);  // x += P x_c
  mg_smooth(mg, v, b, false, s);
  v.x = xs;
}

void mg_apply(Multigrid *mg, const double *b, double *x, hipStream_t s) { vcycle(mg, 0, b, x, s); }

// ------------------------------------------------------------ MG-PCG
// The CG scalars live on the device (sc[]); the host reads back one pair
// (p.q, r.r) per iteration for the breakdown and stopping tests.
// sc layout: [0] p.q, [1] r.r, [2] f.f, [3], [4] alternating r.z slots,
// [5] r_new . z_old.
constexpr int MG_NB = 1024;  // partial-sum blocks of the vector kernels (4 per CU)

// a . b per block (fixed order)
__global__ void __launch_bounds__(256) k_mg_dot(int n, const double *__restrict__ a, const double *__restrict__ b,
                                               double *__restrict__ part) {
  __shared__ double sh[16];
  double v = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v += a[i] * b[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}
// alpha = sc[irz] / sc[0]; x += alpha p; r -= alpha q; per-block r.r
__global__ void __launch_bounds__(256) k_mg_xr(int n, const double *__restrict__ p, const double *__restrict__ q,
                                              double *__restrict__ x, double *__restrict__ r,
                                              const double *__restrict__ sc, int irz, double *__restrict__ part) {
  __shared__ double sh[16];
  const double alpha = sc[irz] / sc[0];
  double v = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    v += ri * ri;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}
// p = z + beta p, beta = (sc[inew] - sc[5]) / sc[iold] = r_new . (z_new - z_old) / (r_old . z_old)
__global__ void k_mg_p(int n, const double *__restrict__ z, double *__restrict__ p, const double *__restrict__ sc,
                       int inew, int iold) {
  const double beta = (sc[inew] - sc[5]) / sc[iold];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = z[i] + beta * p[i];
}
static int mg_nb(int n) { return std::max(1, std::min(MG_NB, (n + 255) / 256)); }
// sc[slot] = a . b (device)
static void dot_dev(int n, const double *a, const double *b, double *part, double *sc, int slot, hipStream_t s) {
  const int nb = mg_nb(n);
  hipLaunchKernelGGL(k_mg_dot, dim3(nb), dim3(256), 0, s, n, a, b, part);
  launch_reduce_cols(part, nb, 1, sc + slot, s);
}
static int read_back(const double *sc, int slot, int cnt, double *h, hipStream_t s) {
  if (hipMemcpyAsync(h, sc + slot, sizeof(double) * cnt, hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
  return hipStreamSynchronize(s) == hipSuccess ? 0 : -1;
}

// CG preconditioned by one V-cycle per iteration on level 0's operator:
// A x = f from the warm start x, stopped at ||f - A x||_2 <= tol ||f||_2.
// part: device scratch (>= 1024 doubles); sc: device scalars (>= 6 doubles).
// Returns 0 converged, 1 iteration limit, -1 launch failure, -2 breakdown
// (p.Ap <= 0).
int mg_pcg(Multigrid *mg, const double *f, double *x, double tol, int max_it, double *part, double *sc,
           int *iters, double *relres, hipStream_t s) {
  MGLevel &v = mg->lv[0];
  const int n = v.n, nb = mg_nb(n);
  double h[2] = {0.0, 0.0};
  lv_spmv(mg, v, x, mg->pr, f, s);  // r = f - A x
  dot_dev(n, f, f, part, sc, 2, s);
  dot_dev(n, mg->pr, mg->pr, part, sc, 1, s);
  double bb = 0.0;
  if (read_back(sc, 1, 2, h, s) < 0) return -1;
  double rr = h[0];
  bb = h[1];
  *iters = 0;
  if (!(bb > 0.0)) {
    launch_fill(n, 0.0, x, s);
    *relres = 0.0;
    return 0;
  }
  *relres = std::sqrt(rr / bb);
  if (rr <= tol * tol * bb) return 0;
  vcycle(mg, 0, mg->pr, mg->pz, s);
  if (hipMemcpyAsync(mg->pp, mg->pz, sizeof(double) * n, hipMemcpyDeviceToDevice, s) != hipSuccess) return -1;
  int irz = 3;
  dot_dev(n, mg->pr, mg->pz, part, sc, irz, s);
  for (int it = 1; it <= max_it; ++it) {
    lv_spmv(mg, v, mg->pp, mg->pq, nullptr, s);  // q = A p
    dot_dev(n, mg->pp, mg->pq, part, sc, 0, s);
    hipLaunchKernelGGL(k_mg_xr, dim3(nb), dim3(256), 0, s, n, mg->pp, mg->pq, x, mg->pr, sc, irz, part);
    launch_reduce_cols(part, nb, 1, sc + 1, s);
    if (read_back(sc, 0, 2, h, s) < 0) return -1;  // p.q, r.r
    // on breakdown x and r already took the (meaningless) step: the caller
    // treats -2 as a failed solve
    if (!(h[0] > 0.0)) return -2;
    rr = h[1];
    *iters = it;
    *relres = std::sqrt(rr / bb);
    if (rr <= tol * tol * bb) return 0;
    // flexible (Polak-Ribiere) beta: the FP32 level-0 smoothing makes the
    // preconditioner vary at rounding level between iterations
    dot_dev(n, mg->pr, mg->pz, part, sc, 5, s);  // r_new . z_old
    vcycle(mg, 0, mg->pr, mg->pz, s);
    const int inew = 7 - irz;  // the other r.z slot (3 <-> 4)
    dot_dev(n, mg->pr, mg->pz, part, sc, inew, s);
    hipLaunchKernelGGL(k_mg_p, dim3(nb), dim3(256), 0, s, n, mg->pz, mg->pp, sc, inew, irz);
    irz = inew;
  }
  return 1;
}

}  // namespace ks
