// Quadrature-point fields: external potential, density, nodal fields
// evaluated at the points, LDA exchange-correlation, density moments and the
// multipole boundary values of the Hartree problem (Sec. 2 and Sec. 3.1).
#include "common.h"
#include "kernels.h"

namespace ks {

static inline dim3 grid_for(int64_t n, int bs = 256, int64_t cap = 8192) {
  int64_t b = (n + bs - 1) / bs;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

// V_ext(x) = -sum_k Z_k / |x - R_k| at x_eq = sum_v lambda_v(q) X_v
__global__ void k_vext(const double *__restrict__ coords, const int32_t *__restrict__ elems,
                       int n_loc, int n_e, int n_q, const double *__restrict__ bary, int n_atoms,
                       const double *__restrict__ Z, const double *__restrict__ R,
                       double *__restrict__ out) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_e * n_q) return;
  int e = (int)(t / n_q), q = (int)(t % n_q);
  double x[3] = {0, 0, 0};
  for (int v = 0; v < 4; ++v) {
    const double l = bary[q * 4 + v];
    const int64_t nd = elems[(int64_t)e * n_loc + v];
    for (int d = 0; d < 3; ++d) x[d] += l * coords[3 * nd + d];
  }
  double V = 0.0;
  for (int a = 0; a < n_atoms; ++a) {
    double dx = x[0] - R[3 * a], dy = x[1] - R[3 * a + 1], dz = x[2] - R[3 * a + 2];
    V -= Z[a] / sqrt(dx * dx + dy * dy + dz * dz);
  }
  out[t] = V;
}
void launch_vext(const double *coords, const int32_t *elems, int n_loc, int n_e, int n_q,
                 const double *bary, int n_atoms, const double *Z, const double *R, double *out,
                 hipStream_t s) {
  int64_t n = (int64_t)n_e * n_q;
  if (n > 0)
    hipLaunchKernelGGL(k_vext, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, coords, elems,
                       n_loc, n_e, n_q, bary, n_atoms, Z, R, out);
}

// rho_q = sum_i f_i (sum_a phi_qa X[node_a][i])^2 = sum_{a,b} phi_qa phi_qb G_ab
// with G_ab = sum_i f_i X[node_a][i] X[node_b][i], the element's occupied
// Gram matrix.  A block first stages its elements' nodal rows (all k orbitals
// of each node, coalesced) in LDS, rows padded to an odd number of doubles so
// that the ten rows of an element sit in distinct banks; the LPE lanes of an
// element then form the NLOC (NLOC + 1) / 2 entries of G (lane l: pairs l,
// l + LPE, ...), and lane q evaluates the quadratic form at point q:
// (NP k + NP NQ) multiply-adds per element instead of NQ NLOC k.
// EPB = 256 / LPE elements per block, LPE >= NQ.
template <int NLOC, int NQ, int LPE>
__global__ void __launch_bounds__(256) k_density(const int32_t *__restrict__ edof, int n_e,
                                                 const double *__restrict__ phi,
                                                 const double *__restrict__ X, int ldx, int k,
                                                 const double *__restrict__ occ,
                                                 double *__restrict__ rho) {
  constexpr int EPB = 256 / LPE, NP = NLOC * (NLOC + 1) / 2;
  extern __shared__ double s_x[];  // [EPB][NLOC][kp], occ [k], G [EPB][NP]
  const int kp = k | 1;
  const int nk = NLOC * kp;
  __shared__ int s_dof[EPB * NLOC];
  const int e0 = blockIdx.x * EPB;
  // the block's node indices in one coalesced read, then each thread's
  // orbital values in batches of eight loads in flight before any store;
  // idx -> (staged row, orbital) without an integer division by k: the float
  // quotient is exact to far better than 1/(2k) for idx < EPB NLOC 64
  for (int t = threadIdx.x; t < EPB * NLOC; t += blockDim.x)
    s_dof[t] = e0 + t / NLOC < n_e ? edof[(int64_t)e0 * NLOC + t] : -1;
  __syncthreads();
  const float rk = 1.0f / (float)k;
  const int total = EPB * NLOC * k;
  for (int c0 = 0; c0 < total; c0 += 8 * 256) {
    double v[8];
    int dst[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = c0 + u * 256 + (int)threadIdx.x;
      v[u] = 0.0;
      dst[u] = -1;
      if (idx < total) {
        const int row = (int)(((float)idx + 0.5f) * rk), i = idx - row * k;
        const int d = s_dof[row];
        if (d >= 0) v[u] = X[(int64_t)d * ldx + i];
        dst[u] = row * kp + i;  // row = el NLOC + a
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (dst[u] >= 0) s_x[dst[u]] = v[u];
  }
  double *s_occ = s_x + EPB * nk;
  double *s_g = s_occ + k;
  for (int i = threadIdx.x; i < k; i += blockDim.x) s_occ[i] = occ[i];
  __syncthreads();
  const int el = threadIdx.x / LPE, l = threadIdx.x - el * LPE, e = e0 + el;
  const double *xe = s_x + el * nk;
  for (int p = l; p < NP; p += LPE) {
    int a = 0, rem = p;  // p -> (a, b), a <= b, upper triangle row by row
    while (rem >= NLOC - a) {
      rem -= NLOC - a;
      ++a;
    }
    const double *xa = xe + a * kp, *xb = xe + (a + rem) * kp;
    double g0 = 0.0, g1 = 0.0;
    int i = 0;
    for (; i + 1 < k; i += 2) {
      g0 += (s_occ[i] * xa[i]) * xb[i];
      g1 += (s_occ[i + 1] * xa[i + 1]) * xb[i + 1];
    }
    if (i < k) g0 += (s_occ[i] * xa[i]) * xb[i];
    s_g[el * NP + p] = rem == 0 ? g0 + g1 : 2.0 * (g0 + g1);
  }
  __syncthreads();
  if (l >= NQ || e >= n_e) return;
  double ph[NLOC];
#pragma unroll
  for (int a = 0; a < NLOC; ++a) ph[a] = phi[l * NLOC + a];
  const double *ge = s_g + el * NP;
  double r0 = 0.0, r1 = 0.0;
  int p = 0;
#pragma unroll
  for (int a = 0; a < NLOC; ++a) {
    double t = 0.0;
#pragma unroll
    for (int b = a; b < NLOC; ++b, ++p) t += ge[p] * ph[b];
    if (a & 1) r1 += ph[a] * t;
    else r0 += ph[a] * t;
  }
  rho[(int64_t)e * NQ + l] = r0 + r1;
}
template <int NLOC, int NQ>
static void density_t(const int32_t *edof, int n_e, const double *phi, const double *X, int ldx, int k,
                      const double *occ, double *rho, hipStream_t s) {
  // 32 lanes per element for the 27-point rule or 10-node elements (the
  // staged block stays under 48 KB at k = 64), else 16
  constexpr int LPE = (NQ > 16 || NLOC == 10) ? 32 : 16;
  constexpr int EPB = 256 / LPE;
  const size_t lds = sizeof(double) * ((size_t)EPB * NLOC * (k | 1) + k + (size_t)EPB * NLOC * (NLOC + 1) / 2);
  hipLaunchKernelGGL((k_density<NLOC, NQ, LPE>), dim3((n_e + EPB - 1) / EPB), dim3(256), lds, s, edof, n_e, phi,
                     X, ldx, k, occ, rho);
}
void launch_density(const int32_t *edof, int n_loc, int n_e, int n_q, const double *phi,
                    const double *X, int ldx, int k, const double *occ, double *rho,
                    hipStream_t s) {
  if (n_e <= 0 || k < 1 || k > 64) return;
  if (n_loc == 4 && n_q == 8) density_t<4, 8>(edof, n_e, phi, X, ldx, k, occ, rho, s);
  else if (n_loc == 10 && n_q == 27) density_t<10, 27>(edof, n_e, phi, X, ldx, k, occ, rho, s);
  else if (n_loc == 4 && n_q == 27) density_t<4, 27>(edof, n_e, phi, X, ldx, k, occ, rho, s);
  else if (n_loc == 10 && n_q == 8) density_t<10, 8>(edof, n_e, phi, X, ldx, k, occ, rho, s);
}

// u_q = sum_a phi_qa U[node_a] for a nodal field over all nodes
template <int NLOC, int NQ>
__global__ void __launch_bounds__(256) k_eval_nodal(const int32_t *__restrict__ elems, int n_e,
                                                    const double *__restrict__ phi,
                                                    const double *__restrict__ U,
                                                    double *__restrict__ out) {
  __shared__ double s_phi[NQ * NLOC];
  for (int i = threadIdx.x; i < NQ * NLOC; i += blockDim.x) s_phi[i] = phi[i];
  __syncthreads();
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_e) return;
  double ua[NLOC];
#pragma unroll
  for (int a = 0; a < NLOC; ++a) ua[a] = U[elems[(int64_t)e * NLOC + a]];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < NLOC; ++a) v += s_phi[q * NLOC + a] * ua[a];
    out[(int64_t)e * NQ + q] = v;
  }
}
void launch_eval_nodal(const int32_t *elems, int n_loc, int n_e, int n_q, const double *phi,
                       const double *U, double *out, hipStream_t s) {
  if (n_e <= 0) return;
  dim3 g((n_e + 255) / 256), b(256);
  if (n_loc == 4 && n_q == 8)
    hipLaunchKernelGGL((k_eval_nodal<4, 8>), g, b, 0, s, elems, n_e, phi, U, out);
  else if (n_loc == 10 && n_q == 27)
    hipLaunchKernelGGL((k_eval_nodal<10, 27>), g, b, 0, s, elems, n_e, phi, U, out);
  else if (n_loc == 4 && n_q == 27)
    hipLaunchKernelGGL((k_eval_nodal<4, 27>), g, b, 0, s, elems, n_e, phi, U, out);
  else if (n_loc == 10 && n_q == 8)
    hipLaunchKernelGGL((k_eval_nodal<10, 8>), g, b, 0, s, elems, n_e, phi, U, out);
}

// LDA (Sec. 3.1): Slater exchange and Perdew-Zunger correlation with the
// constants printed in the paper; r_s = 1 belongs to the low-density branch;
// densities at or below 1e-30 give zero.
__global__ void k_xc(int64_t n, const double *__restrict__ rho, int mode, double *__restrict__ eps,
                     double *__restrict__ v) {
  const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
  const double G = -0.1423, B1 = 1.0529, B2 = 0.3334;
  const double PI = 3.141592653589793238462643;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double r = rho[i];
    double e = 0.0, vv = 0.0;
    if (mode != 0 && r > 1e-30) {
      const double c3 = cbrt(r);
      e = -0.75 * cbrt(3.0 / PI) * c3;
      vv = -cbrt(3.0 / PI) * c3;
      if (mode == 2) {
        const double rs = cbrt(3.0 / (4.0 * PI * r));
        double ec, vc;
        if (rs < 1.0) {
          const double lr = log(rs);
          ec = A * lr + B + C * rs * lr + D * rs;
          vc = A * lr + (B - A / 3.0) + (2.0 / 3.0) * C * rs * lr + (2.0 * D - C) * rs / 3.0;
        } else {
          const double sq = sqrt(rs);
          const double den = 1.0 + B1 * sq + B2 * rs;
          ec = G / den;
          vc = ec * (1.0 + (7.0 / 6.0) * B1 * sq + (4.0 / 3.0) * B2 * rs) / den;
        }
        e += ec;
        vv += vc;
      }
    }
    eps[i] = e;
    v[i] = vv;
  }
}
void launch_xc(int64_t n, const double *rho, int mode, double *eps, double *v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_xc, grid_for(n), dim3(256), 0, s, n, rho, mode, eps, v);
}

// ---------------------------------------------------------------- moments
int moments_blocks(int n_e) {
  int b = (n_e + 255) / 256;
  return b > 1024 ? 1024 : (b < 1 ? 1 : b);
}
__global__ void __launch_bounds__(256) k_moments(const double *__restrict__ coords,
                                                 const int32_t *__restrict__ elems, int n_loc,
                                                 int n_e, int n_q, const double *__restrict__ bary,
                                                 const double *__restrict__ w,
                                                 const double *__restrict__ absdet,
                                                 const double *__restrict__ rho,
                                                 const double *__restrict__ center,
                                                 double *__restrict__ part, int nvals) {
  __shared__ double sh[16];
  double acc[9];
  for (int j = 0; j < 9; ++j) acc[j] = 0.0;
  double c[3] = {0, 0, 0};
  if (center)
    for (int d = 0; d < 3; ++d) c[d] = center[d];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_e; e += gridDim.x * blockDim.x) {
    double X[4][3];
    for (int v = 0; v < 4; ++v)
      for (int d = 0; d < 3; ++d) X[v][d] = coords[3 * (int64_t)elems[(int64_t)e * n_loc + v] + d];
    const double dj = absdet[e];
    for (int q = 0; q < n_q; ++q) {
      double x[3] = {0, 0, 0};
      for (int v = 0; v < 4; ++v)
        for (int d = 0; d < 3; ++d) x[d] += bary[q * 4 + v] * X[v][d];
      const double m = w[q] * dj * rho[(int64_t)e * n_q + q];
      if (!center) {
        acc[0] += m;
        acc[1] += m * x[0];
        acc[2] += m * x[1];
        acc[3] += m * x[2];
      } else {
        const double dx = x[0] - c[0], dy = x[1] - c[1], dz = x[2] - c[2];
        acc[0] += m * dx;
        acc[1] += m * dy;
        acc[2] += m * dz;
        acc[3] += m * dx * dx;
        acc[4] += m * dx * dy;
        acc[5] += m * dx * dz;
        acc[6] += m * dy * dy;
        acc[7] += m * dy * dz;
        acc[8] += m * dz * dz;
      }
    }
  }
  for (int j = 0; j < nvals; ++j) {
    double s = block_sum(acc[j], sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nvals + j] = s;
  }
}
void launch_moments(const double *coords, const int32_t *elems, int n_loc, int n_e, int n_q,
                    const double *bary, const double *w, const double *absdet, const double *rho,
                    const double *center, double *part, int nvals, hipStream_t s) {
  hipLaunchKernelGGL(k_moments, dim3(moments_blocks(n_e)), dim3(256), 0, s, coords, elems, n_loc,
                     n_e, n_q, bary, w, absdet, rho, center, part, nvals);
}

// out[j] = sum_b part[b][j]: all columns at once (threads t = g W + c take
// rows b = g, g + G, ... of column c, eight loads in flight), then the G
// group sums of each column by a tree; W = min(nvals, 1024) columns per pass
__global__ void __launch_bounds__(1024) k_reduce_cols(const double *__restrict__ part, int nblk,
                                                      int nvals, double *__restrict__ out) {
  __shared__ double sh[1024];
  const int t = threadIdx.x;
  for (int c0 = 0; c0 < nvals; c0 += 1024) {
    const int W = min(1024, nvals - c0);
    const int G = 1024 / W;
    double a = 0.0;
    if (t < G * W) {
      const int c = c0 + t % W, g = t / W;
      for (int b = g; b < nblk; b += 8 * G) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = (b + u * G < nblk) ? part[(int64_t)(b + u * G) * nvals + c] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) a += v[u];
      }
    }
    sh[t] = a;
    __syncthreads();
    // the G group sums of each column by a fixed-order tree
    int span = 1;
    while (span < G) span <<= 1;
    for (int st = span >> 1; st >= 1; st >>= 1) {
      if (t < G * W) {
        const int g = t / W;
        if (g < st && g + st < G) sh[t] += sh[t + st * W];
      }
      __syncthreads();
    }
    if (t < W) out[c0 + t] = sh[t];
    __syncthreads();
  }
}
void launch_reduce_cols(const double *part, int nblk, int nvals, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(1024), 0, s, part, nblk, nvals, out);
}

// w_D = Q/|d| + p.d/|d|^3 + f sum q_ij (3 d_i d_j - delta_ij |d|^2)/|d|^5  (eq. bd)
// mom: [0] Q, [1..3] centre, [4..6] p, [7..12] q_xx q_xy q_xz q_yy q_yz q_zz
__global__ void k_multipole(const double *__restrict__ coords, const int32_t *__restrict__ bnodes,
                            int nb, const double *__restrict__ mom, double f,
                            double *__restrict__ wB) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int64_t nd = bnodes[i];
  const double dx = coords[3 * nd] - mom[1], dy = coords[3 * nd + 1] - mom[2],
               dz = coords[3 * nd + 2] - mom[3];
  const double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
  const double qxx = mom[7], qxy = mom[8], qxz = mom[9], qyy = mom[10], qyz = mom[11],
               qzz = mom[12];
  const double dqd = qxx * dx * dx + qyy * dy * dy + qzz * dz * dz +
                     2.0 * (qxy * dx * dy + qxz * dx * dz + qyz * dy * dz);
  const double tr = qxx + qyy + qzz;
  wB[i] = mom[0] / r + (mom[4] * dx + mom[5] * dy + mom[6] * dz) / (r2 * r) +
          f * (3.0 * dqd - tr * r2) / (r2 * r2 * r);
}
void launch_multipole(const double *coords, const int32_t *bnodes, int nb, const double *mom,
                      double quad_factor, double *wB, hipStream_t s) {
  if (nb > 0)
    hipLaunchKernelGGL(k_multipole, dim3((nb + 255) / 256), dim3(256), 0, s, coords, bnodes, nb, mom,
                       quad_factor, wB);
}

__global__ void k_scatter_nodes(int n_nodes, const int32_t *__restrict__ node2int,
                                const int32_t *__restrict__ node2bnd,
                                const double *__restrict__ vint, const double *__restrict__ vbnd,
                                double *__restrict__ V) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_nodes) return;
  const int a = node2int[i];
  V[i] = a >= 0 ? (vint ? vint[a] : 0.0) : (vbnd ? vbnd[node2bnd[i]] : 0.0);
}
void launch_scatter_nodes(int n_nodes, const int32_t *node2int, const int32_t *node2bnd,
                          const double *vint, const double *vbnd, double *V, hipStream_t s) {
  if (n_nodes > 0)
    hipLaunchKernelGGL(k_scatter_nodes, dim3((n_nodes + 255) / 256), dim3(256), 0, s, n_nodes,
                       node2int, node2bnd, vint, vbnd, V);
}

// ---------------------------------------------------------- weighted dots
struct DotArgs {
  const double *a[8];
  const double *b[8];
};
int wdot_blocks(int64_t npts) {
  int64_t b = (npts + 255) / 256;
  return (int)(b > 1024 ? 1024 : (b < 1 ? 1 : b));
}
__global__ void __launch_bounds__(256) k_wdots(int64_t npts, int n_q,
                                               const double *__restrict__ absdet,
                                               const double *__restrict__ w, int nd, DotArgs args,
                                               double *__restrict__ part) {
  __shared__ double sh[16];
  double acc[8];
  for (int j = 0; j < 8; ++j) acc[j] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npts;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double dv = absdet[i / n_q] * w[i % n_q];
    for (int j = 0; j < nd; ++j) acc[j] += dv * args.a[j][i] * (args.b[j] ? args.b[j][i] : 1.0);
  }
  for (int j = 0; j < nd; ++j) {
    double s = block_sum(acc[j], sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nd + j] = s;
  }
}
void launch_wdots(int64_t npts, int n_q, const double *absdet, const double *w, int ndots,
                  const double *const *a, const double *const *b, double *part, hipStream_t s) {
  DotArgs args;
  for (int j = 0; j < 8; ++j) {
    args.a[j] = j < ndots ? a[j] : nullptr;
    args.b[j] = j < ndots ? b[j] : nullptr;
  }
  hipLaunchKernelGGL(k_wdots, dim3(wdot_blocks(npts)), dim3(256), 0, s, npts, n_q, absdet, w,
                     ndots, args, part);
}

struct CombArgs {
  const double *x[12];
};
__global__ void k_lincomb(int64_t n, int nv, const double *__restrict__ coef, CombArgs args,
                          double *__restrict__ out) {
  double c[12];
  for (int j = 0; j < 12; ++j) c[j] = j < nv ? coef[j] : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double r = 0.0;
    for (int j = 0; j < nv; ++j) r += c[j] * args.x[j][i];
    out[i] = r;
  }
}
void launch_lincomb(int64_t n, int nvec, const double *coef_dev, const double *const *x,
                    double *out, hipStream_t s) {
  CombArgs args;
  for (int j = 0; j < 12; ++j) args.x[j] = j < nvec ? x[j] : nullptr;
  if (n > 0) hipLaunchKernelGGL(k_lincomb, grid_for(n), dim3(256), 0, s, n, nvec, coef_dev, args, out);
}

}  // namespace ks

namespace ks {
// Per-column sums of X[i][c] * Y[i][c] over [N][k] row-major blocks (Y null:
// squares of X), per block of rows: thread t owns column t % k of rows
// t / k, t / k + R, ... (R = 256 / k rows per pass), so the reads of a pass are
// one contiguous, coalesced run; the R partial sums of a column are added in a
// fixed order.  k <= 256.
__global__ void __launch_bounds__(256) k_colsums(int N, int k, const double *__restrict__ X,
                                                 const double *__restrict__ Y, double *__restrict__ part) {
  __shared__ double s[256];
  const int R = 256 / k, t = threadIdx.x, c = t % k, r0 = t / k;
  double a = 0.0;
  if (r0 < R) {
    // four passes in flight per iteration
    const int64_t step = (int64_t)gridDim.x * R;
    int64_t i = (int64_t)blockIdx.x * R + r0;
    for (; i + 3 * step < N; i += 4 * step) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = X[(i + u * step) * k + c];
#pragma unroll
      for (int u = 0; u < 4; ++u) y[u] = Y ? Y[(i + u * step) * k + c] : x[u];
#pragma unroll
      for (int u = 0; u < 4; ++u) a += x[u] * y[u];
    }
    for (; i < N; i += step) {
      const double x = X[i * k + c];
      a += x * (Y ? Y[i * k + c] : x);
    }
  }
  s[t] = a;
  __syncthreads();
  if (t < k) {
    double sum = 0.0;
    for (int r = 0; r < R; ++r) sum += s[r * k + t];
    part[(int64_t)blockIdx.x * k + t] = sum;
  }
}
int launch_colsums(int N, int k, const double *X, const double *Y, double *part, hipStream_t s) {
  const int R = 256 / k;
  int nb = (N + R - 1) / R;
  nb = nb > 512 ? 512 : (nb < 1 ? 1 : nb);  // part: <= 512 k doubles
  hipLaunchKernelGGL(k_colsums, dim3(nb), dim3(256), 0, s, N, k, X, Y, part);
  return nb;
}
int launch_colnorms(int N, int k, const double *X, double *part, hipStream_t s) {
  return launch_colsums(N, k, X, nullptr, part, s);
}

struct FjArgs {
  const double *f[4];
};
// NH history differences (compile-time, so the accumulators stay in
// registers); part[b][21]: [0] <F,F>, [1 + j] <D_j,F>, [5 + 4j + l] <D_j,D_l>
template <int NH>
__global__ void __launch_bounds__(256) k_anderson_gram(int64_t npts, int n_q,
                                                       const double *__restrict__ absdet,
                                                       const double *__restrict__ w,
                                                       const double *__restrict__ Fm, FjArgs fj,
                                                       double *__restrict__ part) {
  __shared__ double sh[16];
  double a0 = 0.0, a1[NH > 0 ? NH : 1], a2[NH > 0 ? NH * NH : 1];
#pragma unroll
  for (int j = 0; j < NH; ++j) a1[j] = 0.0;
#pragma unroll
  for (int j = 0; j < NH * NH; ++j) a2[j] = 0.0;
  const bool small = npts < 2147483647LL;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npts;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t e;
    int q;
    if (small) {
      const unsigned ui = (unsigned)i, un = (unsigned)n_q;
      e = ui / un;
      q = (int)(ui - (unsigned)e * un);
    } else {
      e = i / n_q;
      q = (int)(i - e * n_q);
    }
    const double dv = absdet[e] * w[q];
    const double fm = Fm[i];
    double d[NH > 0 ? NH : 1];
#pragma unroll
    for (int j = 0; j < NH; ++j) d[j] = fm - fj.f[j][i];
    a0 += dv * fm * fm;
#pragma unroll
    for (int j = 0; j < NH; ++j) {
      const double dj = dv * d[j];
      a1[j] += dj * fm;
#pragma unroll
      for (int l = 0; l < NH; ++l) a2[j * NH + l] += dj * d[l];
    }
  }
  double s = block_sum(a0, sh);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 21] = s;
  for (int j = 0; j < 4; ++j) {
    double v = 0.0;
#pragma unroll
    for (int jj = 0; jj < NH; ++jj) if (jj == j) v = a1[jj];
    s = block_sum(v, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 21 + 1 + j] = s;
    for (int l = 0; l < 4; ++l) {
      double u = 0.0;
#pragma unroll
      for (int jj = 0; jj < NH; ++jj)
#pragma unroll
        for (int ll = 0; ll < NH; ++ll) if (jj == j && ll == l) u = a2[jj * NH + ll];
      s = block_sum(u, sh);
      if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 21 + 5 + 4 * j + l] = s;
    }
  }
}
int launch_anderson_gram(int64_t npts, int n_q, const double *absdet, const double *w,
                         const double *Fm, int nh, const double *const *Fj, double *part,
                         hipStream_t s) {
  FjArgs a;
  for (int j = 0; j < 4; ++j) a.f[j] = j < nh ? Fj[j] : nullptr;
  int nb = wdot_blocks(npts);
  switch (nh) {
    case 0: hipLaunchKernelGGL(k_anderson_gram<0>, dim3(nb), dim3(256), 0, s, npts, n_q, absdet, w, Fm, a, part); break;
    case 1: hipLaunchKernelGGL(k_anderson_gram<1>, dim3(nb), dim3(256), 0, s, npts, n_q, absdet, w, Fm, a, part); break;
    case 2: hipLaunchKernelGGL(k_anderson_gram<2>, dim3(nb), dim3(256), 0, s, npts, n_q, absdet, w, Fm, a, part); break;
    case 3: hipLaunchKernelGGL(k_anderson_gram<3>, dim3(nb), dim3(256), 0, s, npts, n_q, absdet, w, Fm, a, part); break;
    default: hipLaunchKernelGGL(k_anderson_gram<4>, dim3(nb), dim3(256), 0, s, npts, n_q, absdet, w, Fm, a, part); break;
  }
  return nb;
}

__global__ void k_fill_pencil(int m, int nH, const double *__restrict__ PP,
                              const double *__restrict__ tail, double *__restrict__ F) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * m) return;
  const int i = t / m, j = t % m, kt = m - nH;
  double v;
  if (i < nH && j < nH) v = PP[i * nH + j];
  else if (j >= nH && i < nH) v = tail[i * kt + (j - nH)];
  else if (i >= nH && j < nH) v = tail[j * kt + (i - nH)];
  else v = 0.5 * (tail[i * kt + (j - nH)] + tail[j * kt + (i - nH)]);
  F[t] = v;
}
void launch_fill_pencil(int m, int nH, const double *PP, const double *tail, double *F,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_fill_pencil, dim3((m * m + 255) / 256), dim3(256), 0, s, m, nH, PP, tail, F);
}
__global__ void k_add(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                      double *__restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a[i] + b[i];
}
// Row permutations between the API's natural numbering and the storage
// order: to storage dst[r] = src[int2nat[r]]; to API dst[int2nat[r]] = src[r]
// (k contiguous values per row).
__global__ void k_rows_perm(int N, int k, const double *__restrict__ src, double *__restrict__ dst,
                            const int32_t *__restrict__ int2nat, int to_api) {
  const int64_t n = (int64_t)N * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / k, c = i - r * k;
    const int64_t o = (int64_t)int2nat[r] * k + c;
    if (to_api) dst[o] = src[i];
    else dst[i] = src[o];
  }
}
void launch_rows_to_storage(int N, int k, const double *src_api, double *dst, const int32_t *int2nat,
                            hipStream_t s) {
  const int64_t n = (int64_t)N * k;
  if (n > 0)
    hipLaunchKernelGGL(k_rows_perm, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0,
                       s, N, k, src_api, dst, int2nat, 0);
}
void launch_rows_to_api(int N, int k, const double *src, double *dst_api, const int32_t *int2nat,
                        hipStream_t s) {
  const int64_t n = (int64_t)N * k;
  if (n > 0)
    hipLaunchKernelGGL(k_rows_perm, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0,
                       s, N, k, src, dst_api, int2nat, 1);
}

void launch_add(int64_t n, const double *a, const double *b, double *out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_add, grid_for(n), dim3(256), 0, s, n, a, b, out);
}
}  // namespace ks
