// The mesh-moving side of Algorithm 2 (Sec. 3.2): the Hessian metric of the
// adaptive function u = sqrt(rho) (eqs. m1, m2), a metric spring node mover
// in place of the remesher, and P1 field interpolation between meshes
// (Algorithm 1) to carry nodal fields to the next mesh.
//
// * u at the nodes: sqrt(sum_i f_i psi_i^2), zero on Dirichlet nodes.
// * recovery: the P1 interpolant's gradient is constant per element; its
//   lumped-mass L2 projection onto P1 is the volume-weighted average over
//   the elements around a node (gathered per node in element order, no
//   atomics).  Applied to u and then to each component of the result, the
//   symmetric part is the recovered Hessian H.
// * metric: H = R Lambda R^T by cyclic Jacobi rotations in registers,
//   lambda~ = min(max(C_d |lambda| / eps, 1 / h_max^2), 1 / h_min^2) with
//   C_d = 9/32 (d = 3), M = R Lambda~ R^T, stored [n_nodes][6] as
//   (xx, yy, zz, xy, xz, yz).
// * mover: damped Jacobi sweeps on the spring energy
//   sum_edges (x_b - x_a)^T (M_a + M_b)/2 (x_b - x_a): every free node moves
//   toward the minimiser over that node, x_a <- (1 - w) x_a + w t_a with
//   (sum_b Mbar_ab) t_a = sum_b Mbar_ab x_b; Dirichlet nodes stay; a sweep
//   whose result has an element with det J <= 0 is redone with w halved.
#include "../../include/ks.h"
#include "common.h"
#include "kernels.h"
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace ks {
namespace {

constexpr double C_D3 = 9.0 / 32.0;  // 1/2 (d / (d + 1))^2, d = 3

__global__ void k_nodal_u(int N, int k, const double *__restrict__ psi, const double *__restrict__ occ,
                          const int32_t *__restrict__ inner, double *__restrict__ u) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  double s = 0.0;
  for (int j = 0; j < k; ++j) {
    const double p = psi[(int64_t)a * k + j];
    s += occ[j] * p * p;
  }
  u[inner[a]] = sqrt(s);
}

// per element: volume and the gradients of the P1 interpolants of m fields
// (F [n_nodes][m]); ge [n_e][m][3]
__global__ void k_elem_grad(int ne, const int32_t *__restrict__ tets, const double *__restrict__ x, int m,
                            const double *__restrict__ F, double *__restrict__ vol, double *__restrict__ ge) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int v[4];
  double X[4][3];
  for (int a = 0; a < 4; ++a) {
    v[a] = tets[4 * (int64_t)e + a];
    for (int d = 0; d < 3; ++d) X[a][d] = x[3 * (int64_t)v[a] + d];
  }
  // J columns X_i - X_0; the rows of J^-1 are the gradients of lambda_1..3
  double J[3][3];
  for (int d = 0; d < 3; ++d)
    for (int i = 0; i < 3; ++i) J[d][i] = X[i + 1][d] - X[0][d];
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  double Ji[3][3];  // inverse: Ji[i][d]
  Ji[0][0] = c00 / det;
  Ji[1][0] = c01 / det;
  Ji[2][0] = c02 / det;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  vol[e] = det / 6.0;
  for (int c = 0; c < m; ++c) {
    const double f0 = F[(int64_t)v[0] * m + c];
    double g[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 3; ++i) {
      const double df = F[(int64_t)v[i + 1] * m + c] - f0;
      for (int d = 0; d < 3; ++d) g[d] += df * Ji[i][d];
    }
    for (int d = 0; d < 3; ++d) ge[((int64_t)e * m + c) * 3 + d] = g[d];
  }
}

// per node: volume-weighted average of ge over its elements (n2e CSR, in
// ascending element order); out [n_nodes][m][3]
__global__ void k_node_avg(int nn, const int32_t *__restrict__ n2e_off, const int32_t *__restrict__ n2e, int m,
                           const double *__restrict__ vol, const double *__restrict__ ge, double *__restrict__ out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nn) return;
  double den = 0.0;
  for (int p = n2e_off[a]; p < n2e_off[a + 1]; ++p) den += vol[n2e[p]];
  for (int c = 0; c < m; ++c)
    for (int d = 0; d < 3; ++d) {
      double s = 0.0;
      for (int p = n2e_off[a]; p < n2e_off[a + 1]; ++p) {
        const int e = n2e[p];
        s += vol[e] * ge[((int64_t)e * m + c) * 3 + d];
      }
      out[((int64_t)a * m + c) * 3 + d] = s / den;
    }
}

// symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations: A is
// overwritten by its eigenvalues on the diagonal, V holds the eigenvectors
// as columns
__device__ void jacobi3(double A[3][3], double V[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    const double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
    const double nrm = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]) + off;
    if (off <= 1e-17 * nrm || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < 3; ++r) {  // A <- A G (columns p, q)
          const double arp = A[r][p], arq = A[r][q];
          A[r][p] = c * arp - s * arq;
          A[r][q] = s * arp + c * arq;
        }
        for (int r = 0; r < 3; ++r) {  // A <- G^T A (rows p, q)
          const double apr = A[p][r], aqr = A[q][r];
          A[p][r] = c * apr - s * aqr;
          A[q][r] = s * apr + c * aqr;
        }
        for (int r = 0; r < 3; ++r) {
          const double vrp = V[r][p], vrq = V[r][q];
          V[r][p] = c * vrp - s * vrq;
          V[r][q] = s * vrp + c * vrq;
        }
      }
  }
}

// D [n][3][3] (component, derivative) -> M [n][6]
__global__ void k_metric(int nn, const double *__restrict__ D, double eps, double lo, double hi,
                         double *__restrict__ M) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nn) return;
  double A[3][3], V[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = 0.5 * (D[(int64_t)a * 9 + i * 3 + j] + D[(int64_t)a * 9 + j * 3 + i]);
  jacobi3(A, V);
  double lt[3];
  for (int i = 0; i < 3; ++i) lt[i] = fmin(fmax(C_D3 * fabs(A[i][i]) / eps, lo), hi);
  const int ij[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  for (int c = 0; c < 6; ++c) {
    const int i = ij[c][0], j = ij[c][1];
    M[(int64_t)a * 6 + c] = V[i][0] * lt[0] * V[j][0] + V[i][1] * lt[1] * V[j][1] + V[i][2] * lt[2] * V[j][2];
  }
}

__device__ __forceinline__ void sym6(const double *m, double S[3][3]) {
  S[0][0] = m[0];
  S[1][1] = m[1];
  S[2][2] = m[2];
  S[0][1] = S[1][0] = m[3];
  S[0][2] = S[2][0] = m[4];
  S[1][2] = S[2][1] = m[5];
}

// per free node: the minimiser t of the spring energy over that node
__global__ void k_move_target(int nn, const int32_t *__restrict__ adj_off, const int32_t *__restrict__ adj,
                              const uint8_t *__restrict__ fixed, const double *__restrict__ x,
                              const double *__restrict__ M, double *__restrict__ t) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nn) return;
  if (fixed[a]) {
    for (int d = 0; d < 3; ++d) t[3 * (int64_t)a + d] = x[3 * (int64_t)a + d];
    return;
  }
  double Ma[3][3];
  sym6(M + (int64_t)a * 6, Ma);
  double S[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, r[3] = {0, 0, 0};
  for (int p = adj_off[a]; p < adj_off[a + 1]; ++p) {
    const int b = adj[p];
    double Mb[3][3];
    sym6(M + (int64_t)b * 6, Mb);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double w = 0.5 * (Ma[i][j] + Mb[i][j]);
        S[i][j] += w;
        r[i] += w * x[3 * (int64_t)b + j];
      }
  }
  // S t = r by Cramer's rule (S is symmetric positive definite)
  const double c00 = S[1][1] * S[2][2] - S[1][2] * S[2][1];
  const double c01 = S[1][2] * S[2][0] - S[1][0] * S[2][2];
  const double c02 = S[1][0] * S[2][1] - S[1][1] * S[2][0];
  const double det = S[0][0] * c00 + S[0][1] * c01 + S[0][2] * c02;
  double inv[3][3];
  inv[0][0] = c00 / det;
  inv[1][0] = c01 / det;
  inv[2][0] = c02 / det;
  inv[0][1] = (S[0][2] * S[2][1] - S[0][1] * S[2][2]) / det;
  inv[1][1] = (S[0][0] * S[2][2] - S[0][2] * S[2][0]) / det;
  inv[2][1] = (S[0][1] * S[2][0] - S[0][0] * S[2][1]) / det;
  inv[0][2] = (S[0][1] * S[1][2] - S[0][2] * S[1][1]) / det;
  inv[1][2] = (S[0][2] * S[1][0] - S[0][0] * S[1][2]) / det;
  inv[2][2] = (S[0][0] * S[1][1] - S[0][1] * S[1][0]) / det;
  for (int i = 0; i < 3; ++i) t[3 * (int64_t)a + i] = inv[i][0] * r[0] + inv[i][1] * r[1] + inv[i][2] * r[2];
}

__global__ void k_move_apply(int64_t n3, double w, const double *__restrict__ x, const double *__restrict__ t,
                             double *__restrict__ xn) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n3) xn[i] = (1.0 - w) * x[i] + w * t[i];
}

// per-block minimum of det J over the elements
__global__ void __launch_bounds__(256) k_min_det(int ne, const int32_t *__restrict__ tets,
                                                 const double *__restrict__ x, double *__restrict__ part) {
  __shared__ double sh[256];
  double mn = INFINITY;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
    double X[4][3];
    for (int a = 0; a < 4; ++a)
      for (int d = 0; d < 3; ++d) X[a][d] = x[3 * (int64_t)tets[4 * (int64_t)e + a] + d];
    double J[3][3];
    for (int d = 0; d < 3; ++d)
      for (int i = 0; i < 3; ++i) J[d][i] = X[i + 1][d] - X[0][d];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    mn = fmin(mn, det);
  }
  sh[threadIdx.x] = mn;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out[i][c] = sum_v w[i][v] F[vid[i][v]][c]
__global__ void k_field_gather(int npts, int m, const int32_t *__restrict__ vid, const double *__restrict__ w,
                               const double *__restrict__ F, double *__restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)npts * m) return;
  const int i = (int)(t / m), c = (int)(t % m);
  double s = 0.0;
  for (int v = 0; v < 4; ++v) s += w[4 * (int64_t)i + v] * F[(int64_t)vid[4 * (int64_t)i + v] * m + c];
  out[t] = s;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// device buffers of one call, freed on every exit path
struct Scratch {
  std::vector<void *> ptrs;
  ~Scratch() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  T *get(size_t n) {
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return static_cast<T *>(p);
  }
};

int check_p1_mesh(const ks_mesh_desc *m) {
  if (!m || !m->coords_host || !m->elems_host || !m->dirichlet_host) return set_error(KS_ERR_ARG, "null mesh array");
  if (m->order != 1) return set_error(KS_ERR_ARG, "the mesh must be P1");
  if (m->n_nodes < 4 || m->n_elems < 1) return set_error(KS_ERR_ARG, "empty mesh");
  for (int64_t i = 0; i < (int64_t)m->n_elems * 4; ++i)
    if (m->elems_host[i] < 0 || m->elems_host[i] >= m->n_nodes) return set_error(KS_ERR_MESH, "node id out of range");
  return KS_OK;
}

// CSR of node -> elements (ascending element order) and node -> neighbours
void node_adjacency(const ks_mesh_desc *m, std::vector<int32_t> &e_off, std::vector<int32_t> &e_idx,
                    std::vector<int32_t> &a_off, std::vector<int32_t> &a_idx) {
  const int nn = m->n_nodes, ne = m->n_elems;
  e_off.assign(nn + 1, 0);
  for (int64_t i = 0; i < (int64_t)ne * 4; ++i) e_off[m->elems_host[i] + 1]++;
  for (int a = 0; a < nn; ++a) e_off[a + 1] += e_off[a];
  e_idx.resize(e_off[nn]);
  std::vector<int32_t> pos(e_off.begin(), e_off.end() - 1);
  for (int e = 0; e < ne; ++e)
    for (int a = 0; a < 4; ++a) e_idx[pos[m->elems_host[4 * (int64_t)e + a]]++] = e;
  a_off.assign(nn + 1, 0);
  a_idx.clear();
  std::vector<int32_t> nb;
  for (int a = 0; a < nn; ++a) {
    nb.clear();
    for (int p = e_off[a]; p < e_off[a + 1]; ++p)
      for (int v = 0; v < 4; ++v) {
        const int b = m->elems_host[4 * (int64_t)e_idx[p] + v];
        if (b != a) nb.push_back(b);
      }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    a_idx.insert(a_idx.end(), nb.begin(), nb.end());
    a_off[a + 1] = (int32_t)a_idx.size();
  }
}

}  // namespace
}  // namespace ks

using namespace ks;

#define MCHK(x)                                                        \
  do {                                                                 \
    hipError_t e_ = (x);                                               \
    if (e_ != hipSuccess) return set_error(KS_ERR_HIP, hipGetErrorString(e_)); \
  } while (0)

extern "C" int ks_mesh_metric(const ks_mesh_desc *mesh, const double *psi, int32_t k, const double *occ_host,
                              const ks_metric_params *prm, double *metric, hipStream_t s) {
  int rc = check_p1_mesh(mesh);
  if (rc < 0) return rc;
  if (!psi || !occ_host || !prm || !metric || k < 1) return set_error(KS_ERR_ARG, "null argument or k < 1");
  if (!(prm->eps > 0.0) || !(prm->h_min > 0.0) || !(prm->h_max >= prm->h_min))
    return set_error(KS_ERR_ARG, "need eps > 0 and 0 < h_min <= h_max");
  const int nn = mesh->n_nodes, ne = mesh->n_elems;
  std::vector<int32_t> inner;
  for (int a = 0; a < nn; ++a)
    if (!mesh->dirichlet_host[a]) inner.push_back(a);
  const int N = (int)inner.size();
  std::vector<int32_t> e_off, e_idx, a_off, a_idx;
  node_adjacency(mesh, e_off, e_idx, a_off, a_idx);
  Scratch sc;
  double *x = sc.get<double>((size_t)nn * 3), *occ = sc.get<double>(k), *u = sc.get<double>(nn);
  double *vol = sc.get<double>(ne), *ge = sc.get<double>((size_t)ne * 9);
  double *G = sc.get<double>((size_t)nn * 3), *D = sc.get<double>((size_t)nn * 9);
  int32_t *tets = sc.get<int32_t>((size_t)ne * 4), *in = sc.get<int32_t>(N);
  int32_t *eo = sc.get<int32_t>(nn + 1), *ei = sc.get<int32_t>(e_idx.size());
  if (!x || !occ || !u || !vol || !ge || !G || !D || !tets || !in || !eo || !ei)
    return set_error(KS_ERR_NOMEM, "ks_mesh_metric: hipMalloc failed");
  MCHK(hipMemcpyAsync(x, mesh->coords_host, sizeof(double) * nn * 3, hipMemcpyHostToDevice, s));
  MCHK(hipMemcpyAsync(occ, occ_host, sizeof(double) * k, hipMemcpyHostToDevice, s));
  MCHK(hipMemcpyAsync(tets, mesh->elems_host, sizeof(int32_t) * ne * 4, hipMemcpyHostToDevice, s));
  MCHK(hipMemcpyAsync(in, inner.data(), sizeof(int32_t) * std::max(N, 1), hipMemcpyHostToDevice, s));
  MCHK(hipMemcpyAsync(eo, e_off.data(), sizeof(int32_t) * (nn + 1), hipMemcpyHostToDevice, s));
  MCHK(hipMemcpyAsync(ei, e_idx.data(), sizeof(int32_t) * e_idx.size(), hipMemcpyHostToDevice, s));
  launch_fill(nn, 0.0, u, s);
  if (N > 0) hipLaunchKernelGGL(k_nodal_u, dim3(blocks_for(N)), dim3(256), 0, s, N, k, psi, occ, in, u);
  // G = recovered gradient of u, D = recovered gradient of each component of G
  hipLaunchKernelGGL(k_elem_grad, dim3(blocks_for(ne)), dim3(256), 0, s, ne, tets, x, 1, u, vol, ge);
  hipLaunchKernelGGL(k_node_avg, dim3(blocks_for(nn)), dim3(256), 0, s, nn, eo, ei, 1, vol, ge, G);
  hipLaunchKernelGGL(k_elem_grad, dim3(blocks_for(ne)), dim3(256), 0, s, ne, tets, x, 3, G, vol, ge);
  hipLaunchKernelGGL(k_node_avg, dim3(blocks_for(nn)), dim3(256), 0, s, nn, eo, ei, 3, vol, ge, D);
  hipLaunchKernelGGL(k_metric, dim3(blocks_for(nn)), dim3(256), 0, s, nn, D, prm->eps,
                     1.0 / (prm->h_max * prm->h_max), 1.0 / (prm->h_min * prm->h_min), metric);
  MCHK(hipGetLastError());
  MCHK(hipStreamSynchronize(s));
  return KS_OK;
}

extern "C" int ks_move_nodes(const ks_mesh_desc *mesh, const double *metric, double omega, int32_t sweeps,
                             double *coords_out_host, int32_t *halvings_host, hipStream_t s) {
  int rc = check_p1_mesh(mesh);
  if (rc < 0) return rc;
  if (!metric || !coords_out_host) return set_error(KS_ERR_ARG, "null argument");
  if (!(omega > 0.0 && omega < 2.0) || sweeps < 0) return set_error(KS_ERR_ARG, "need 0 < omega < 2, sweeps >= 0");
  const int nn = mesh->n_nodes, ne = mesh->n_elems;
  std::vector<int32_t> e_off, e_idx, a_off, a_idx;
  node_adjacency(mesh, e_off, e_idx, a_off, a_idx);
  Scratch sc;
  double *x = sc.get<double>((size_t)nn * 3), *xn = sc.get<double>((size_t)nn * 3);
  double *t = sc.get<double>((size_t)nn * 3);
  const int nb = (int)std::min<int64_t>(blocks_for(ne), 1024);
  double *part = sc.get<double>(nb);
  int32_t *tets = sc.get<int32_t>((size_t)ne * 4), *ao = sc.get<int32_t>(nn + 1), *ai = sc.get<int32_t>(a_idx.size());
  uint8_t *fx = sc.get<uint8_t>(nn);
  if (!x || !xn || !t || !part || !tets || !ao || !ai || !fx)
    return set_error(KS_ERR_NOMEM, "ks_move_nodes: hipMalloc failed");
  MCHK(hipMemcpyAsync(x, mesh->coords_host, sizeof(double) * nn * 3, hipMemcpyHostToDevice, s));
  MCHK(hipMemcpyAsync(tets, mesh->elems_host, sizeof(int32_t) * ne * 4, hipMemcpyHostToDevice, s));
  MCHK(hipMemcpyAsync(ao, a_off.data(), sizeof(int32_t) * (nn + 1), hipMemcpyHostToDevice, s));
  MCHK(hipMemcpyAsync(ai, a_idx.data(), sizeof(int32_t) * a_idx.size(), hipMemcpyHostToDevice, s));
  MCHK(hipMemcpyAsync(fx, mesh->dirichlet_host, nn, hipMemcpyHostToDevice, s));
  std::vector<double> h(nb);
  int halvings = 0;
  for (int sw = 0; sw < sweeps; ++sw) {
    hipLaunchKernelGGL(k_move_target, dim3(blocks_for(nn)), dim3(256), 0, s, nn, ao, ai, fx, x, metric, t);
    double w = omega;
    bool ok = false;
    for (int tries = 0; tries <= 20 && !ok; ++tries) {
      hipLaunchKernelGGL(k_move_apply, dim3(blocks_for((int64_t)nn * 3)), dim3(256), 0, s, (int64_t)nn * 3, w, x, t,
                         xn);
      hipLaunchKernelGGL(k_min_det, dim3(nb), dim3(256), 0, s, ne, tets, xn, part);
      MCHK(hipMemcpyAsync(h.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
      MCHK(hipStreamSynchronize(s));
      const double mn = *std::min_element(h.begin(), h.end());
      ok = mn > 0.0;
      if (!ok) {
        w *= 0.5;
        ++halvings;
      }
    }
    if (!ok) return set_error(KS_ERR_MESH, "ks_move_nodes: every damped move inverts an element");
    std::swap(x, xn);
  }
  MCHK(hipMemcpyAsync(coords_out_host, x, sizeof(double) * nn * 3, hipMemcpyDeviceToHost, s));
  MCHK(hipStreamSynchronize(s));
  if (halvings_host) *halvings_host = halvings;
  return KS_OK;
}

extern "C" int ks_interpolate_field(const ks_mesh_desc *src, const double *field, int32_t m, int32_t n_pts,
                                    const double *pts_host, double *out, hipStream_t s) {
  int rc = check_p1_mesh(src);
  if (rc < 0) return rc;
  if (!field || !pts_host || !out || m < 1 || n_pts < 0) return set_error(KS_ERR_ARG, "null argument or m < 1");
  if (n_pts == 0) return KS_OK;
  Scratch sc;
  int32_t *dv = sc.get<int32_t>((size_t)n_pts * 4);
  double *dw = sc.get<double>((size_t)n_pts * 4), *dp = sc.get<double>((size_t)n_pts * 3);
  if (!dv || !dw || !dp) return set_error(KS_ERR_NOMEM, "ks_interpolate_field: hipMalloc failed");
  MCHK(hipMemcpyAsync(dp, pts_host, sizeof(double) * 3 * (size_t)n_pts, hipMemcpyHostToDevice, s));
  const int r = nonnested_weights_device(src->n_nodes, src->coords_host, src->n_elems, src->elems_host, n_pts, dp, dv,
                                         dw, s);
  if (r == -1) return set_error(KS_ERR_MESH, "source mesh: bad element vertex ids");
  if (r == -2) return set_error(KS_ERR_MESH, "point location: degenerate weights");
  if (r == -3) return set_error(KS_ERR_NOMEM, "ks_interpolate_field: hipMalloc failed");
  if (r < 0) return set_error(KS_ERR_HIP, "point location failed");
  hipLaunchKernelGGL(k_field_gather, dim3(blocks_for((int64_t)n_pts * m)), dim3(256), 0, s, n_pts, m, dv, dw, field,
                     out);
  MCHK(hipGetLastError());
  MCHK(hipStreamSynchronize(s));
  return KS_OK;
}
