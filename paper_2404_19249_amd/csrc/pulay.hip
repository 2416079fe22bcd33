// Derivative of one step's Kohn-Sham energy with respect to the vertex
// coordinates of the fine mesh (mesh-motion, or Pulay, terms of the forces).
//
// The step's inputs (Psi^l, lambda^l, rho^l, the Hartree boundary data and
// the matrix of I_H^h) are held fixed and the vertices move.  The chain rule
// through the converged inner iteration, the M-orthogonalisation of the BVP
// solutions and the BVPs themselves (one adjoint BVP solve, two adjoint
// Poisson solves, done by the caller) leaves a sum over elements of
//   * stiffness forms  sum_i wK_i u_i^T K_e v_i     (pairs of vector blocks),
//   * mass forms       sum_i wM_i u_i^T M_e v_i,
//   * sum_q dV_q F_q          (fixed quadrature values F),
//   * sum_q dV_q G_q V_ext(x_q)   (the quadrature points move with the mesh),
// differentiated with respect to the element's four vertices in closed form
// for the affine map x = X0 + J xi:
//   u^T K_e v = |J| tr(B A),  B = J^-1 J^-T,  A = sum_q w_q (grad_xi u)(grad_xi v)^T,
//   d(|J| tr(B A_s))/dJ = |J| (tr(B A_s) J^-T - 2 (B A_s J^-1)^T),  A_s = sym(A),
//   d|J|/dJ = |J| J^-T,   dx_q/dX_v = lambda_v(xi_q),
// with J's columns X1 - X0, X2 - X0, X3 - X0.  One element per thread; the
// per-element results are gathered per vertex in a fixed order.
#include "common.h"
#include "kernels.h"

namespace ks {

static inline dim3 grid_1d(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

// out_q = sum_i A_i(x_q) B_i(x_q) over interior blocks A [N][lda], B [N][ldb]
template <int NLOC, int NQ>
__global__ void __launch_bounds__(256) k_pair_q(const int32_t *__restrict__ edof, int n_e,
                                                const double *__restrict__ phi, const double *__restrict__ A,
                                                int lda, const double *__restrict__ Bm, int ldb, int k,
                                                double *__restrict__ out) {
  __shared__ double s_phi[NQ * NLOC];
  for (int i = threadIdx.x; i < NQ * NLOC; i += blockDim.x) s_phi[i] = phi[i];
  __syncthreads();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_e) return;
  int dof[NLOC];
#pragma unroll
  for (int a = 0; a < NLOC; ++a) dof[a] = edof[(int64_t)e * NLOC + a];
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int i = 0; i < k; ++i) {
    double xa[NLOC], ya[NLOC];
#pragma unroll
    for (int a = 0; a < NLOC; ++a) {
      xa[a] = dof[a] >= 0 ? A[(int64_t)dof[a] * lda + i] : 0.0;
      ya[a] = dof[a] >= 0 ? Bm[(int64_t)dof[a] * ldb + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double u = 0.0, v = 0.0;
#pragma unroll
      for (int a = 0; a < NLOC; ++a) {
        u += s_phi[q * NLOC + a] * xa[a];
        v += s_phi[q * NLOC + a] * ya[a];
      }
      acc[q] += u * v;
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) out[(int64_t)e * NQ + q] = acc[q];
}

// F = rho eps - gam vxc_l [+ rho V0 + (rho - rho_l / 2) Vbc - gam VHl - 4 pi rho_l W2]
// G = rho - gam        (the Hartree fields are null when the step has none)
__global__ void k_pulay_fields(int64_t n, const double *__restrict__ rho, const double *__restrict__ rho_l,
                               const double *__restrict__ eps, const double *__restrict__ vxc_l,
                               const double *__restrict__ gam, const double *__restrict__ V0,
                               const double *__restrict__ Vbc, const double *__restrict__ VHl,
                               const double *__restrict__ W2, double *__restrict__ F, double *__restrict__ G) {
  const double FOUR_PI = 4.0 * 3.141592653589793238462643;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double r = rho[i], rl = rho_l[i], g = gam[i];
    double f = r * eps[i] - g * vxc_l[i];
    if (V0) f += r * V0[i] + (r - 0.5 * rl) * Vbc[i] - g * VHl[i] - FOUR_PI * rl * W2[i];
    F[i] = f;
    G[i] = r - g;
  }
}

template <int NLOC, int NQ>
__global__ void __launch_bounds__(128) k_mesh_grad(const double *__restrict__ coords, const int32_t *__restrict__ elems,
                                                   const int32_t *__restrict__ edof, int n_e,
                                                   const double *__restrict__ phi, const double *__restrict__ dphi,
                                                   const double *__restrict__ w, const double *__restrict__ bary,
                                                   MeshGradPairs pr, const double *__restrict__ coef, int k,
                                                   const double *__restrict__ F, const double *__restrict__ G,
                                                   int n_atoms, const double *__restrict__ Zn,
                                                   const double *__restrict__ Rn, double scale,
                                                   double *__restrict__ out) {
  __shared__ double s_phi[NQ * NLOC];
  __shared__ double s_gx[NQ * NLOC * 3];  // d phi_a / d xi_c at q
  __shared__ double s_w[NQ];
  __shared__ double s_bary[NQ * 4];
  for (int i = threadIdx.x; i < NQ * NLOC; i += blockDim.x) {
    s_phi[i] = phi[i];
    const double *d = dphi + (int64_t)i * 4;
    for (int c = 0; c < 3; ++c) s_gx[i * 3 + c] = d[c + 1] - d[0];
  }
  for (int i = threadIdx.x; i < NQ; i += blockDim.x) s_w[i] = w[i];
  for (int i = threadIdx.x; i < NQ * 4; i += blockDim.x) s_bary[i] = bary[i];
  __syncthreads();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_e) return;
  double X[4][3];
  for (int v = 0; v < 4; ++v)
    for (int d = 0; d < 3; ++d) X[v][d] = coords[3 * (int64_t)elems[(int64_t)e * NLOC + v] + d];
  double J[3][3];
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 3; ++c) J[d][c] = X[c + 1][d] - X[0][d];
  const double C00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], C01 = J[1][2] * J[2][0] - J[1][0] * J[2][2],
               C02 = J[1][0] * J[2][1] - J[1][1] * J[2][0], C10 = J[0][2] * J[2][1] - J[0][1] * J[2][2],
               C11 = J[0][0] * J[2][2] - J[0][2] * J[2][0], C12 = J[0][1] * J[2][0] - J[0][0] * J[2][1],
               C20 = J[0][1] * J[1][2] - J[0][2] * J[1][1], C21 = J[0][2] * J[1][0] - J[0][0] * J[1][2],
               C22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * C00 + J[0][1] * C01 + J[0][2] * C02;  // > 0 (checked at set-up)
  const double id = 1.0 / det;
  const double Ji[3][3] = {{C00 * id, C10 * id, C20 * id}, {C01 * id, C11 * id, C21 * id},
                           {C02 * id, C12 * id, C22 * id}};
  double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double s = 0.0;         // everything proportional to |J|
  double pv[4][3] = {};   // moving quadrature points
  int dof[NLOC], node[NLOC];
#pragma unroll
  for (int a = 0; a < NLOC; ++a) {
    dof[a] = edof[(int64_t)e * NLOC + a];
    node[a] = elems[(int64_t)e * NLOC + a];
  }
  // pairs of interior blocks: stiffness and mass forms with per-column weights
  for (int p = 0; p < pr.n; ++p) {
    const double *U = pr.u[p], *V = pr.v[p];
    const int lu = pr.ldu[p], lv = pr.ldv[p];
    for (int i = 0; i < k; ++i) {
      const double wk = coef[(p * k + i) * 2], wm = coef[(p * k + i) * 2 + 1];
      if (wk == 0.0 && wm == 0.0) continue;
      double ua[NLOC], va[NLOC];
#pragma unroll
      for (int a = 0; a < NLOC; ++a) {
        ua[a] = dof[a] >= 0 ? U[(int64_t)dof[a] * lu + i] : 0.0;
        va[a] = dof[a] >= 0 ? V[(int64_t)dof[a] * lv + i] : 0.0;
      }
      for (int q = 0; q < NQ; ++q) {
        if (wk != 0.0) {
          double gu[3] = {0, 0, 0}, gv[3] = {0, 0, 0};
#pragma unroll
          for (int a = 0; a < NLOC; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              gu[c] += s_gx[(q * NLOC + a) * 3 + c] * ua[a];
              gv[c] += s_gx[(q * NLOC + a) * 3 + c] * va[a];
            }
          const double f = wk * s_w[q];
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) A[r][c] += f * gu[r] * gv[c];
        }
        if (wm != 0.0) {
          double uq = 0.0, vq = 0.0;
#pragma unroll
          for (int a = 0; a < NLOC; ++a) {
            uq += s_phi[q * NLOC + a] * ua[a];
            vq += s_phi[q * NLOC + a] * va[a];
          }
          s += wm * s_w[q] * det * uq * vq;
        }
      }
    }
  }
  // pairs of nodal fields over all nodes: stiffness forms only
  for (int p = 0; p < pr.n_nodal; ++p) {
    const double *U = pr.nu[p], *V = pr.nv[p];
    const double wk = pr.nw[p];
    double ua[NLOC], va[NLOC];
#pragma unroll
    for (int a = 0; a < NLOC; ++a) {
      ua[a] = U[node[a]];
      va[a] = V[node[a]];
    }
    for (int q = 0; q < NQ; ++q) {
      double gu[3] = {0, 0, 0}, gv[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < NLOC; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          gu[c] += s_gx[(q * NLOC + a) * 3 + c] * ua[a];
          gv[c] += s_gx[(q * NLOC + a) * 3 + c] * va[a];
        }
      const double f = wk * s_w[q];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) A[r][c] += f * gu[r] * gv[c];
    }
  }
  // quadrature fields: fixed F, and G V_ext at the moving points
  for (int q = 0; q < NQ; ++q) {
    const int64_t iq = (int64_t)e * NQ + q;
    const double dV = s_w[q] * det;
    double x[3] = {0, 0, 0};
    for (int v = 0; v < 4; ++v)
      for (int d = 0; d < 3; ++d) x[d] += s_bary[q * 4 + v] * X[v][d];
    double ve = 0.0, gr[3] = {0, 0, 0};
    for (int a = 0; a < n_atoms; ++a) {
      const double dx = x[0] - Rn[3 * a], dy = x[1] - Rn[3 * a + 1], dz = x[2] - Rn[3 * a + 2];
      const double r2 = dx * dx + dy * dy + dz * dz, ir = 1.0 / sqrt(r2);
      const double z = Zn[a];
      ve -= z * ir;
      const double c3 = z * ir * ir * ir;  // grad (-Z / r) = Z (x - R) / r^3
      gr[0] += c3 * dx;
      gr[1] += c3 * dy;
      gr[2] += c3 * dz;
    }
    const double gq = G[iq] * dV;
    s += dV * F[iq] + gq * ve;
    for (int v = 0; v < 4; ++v) {
      const double l = s_bary[q * 4 + v] * gq;
      for (int d = 0; d < 3; ++d) pv[v][d] += l * gr[d];
    }
  }
  // d/dJ of |J| tr(B A_s) + s, B = Ji Ji^T
  double As[3][3], B[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      As[r][c] = 0.5 * (A[r][c] + A[c][r]);
      B[r][c] = Ji[r][0] * Ji[c][0] + Ji[r][1] * Ji[c][1] + Ji[r][2] * Ji[c][2];
    }
  double BA[3][3], tr = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) BA[r][c] = B[r][0] * As[0][c] + B[r][1] * As[1][c] + B[r][2] * As[2][c];
  for (int r = 0; r < 3; ++r) tr += BA[r][r];
  double Gm[3][3];  // Gm[d][c] = d phi / d J[d][c]
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) {
      const double M1 = BA[c][0] * Ji[0][d] + BA[c][1] * Ji[1][d] + BA[c][2] * Ji[2][d];  // (B A_s J^-1)[c][d]
      Gm[d][c] = det * (tr * Ji[c][d] - 2.0 * M1) + s * Ji[c][d];
    }
  double *o = out + (int64_t)e * 12;
  for (int d = 0; d < 3; ++d) {
    o[d] = scale * (pv[0][d] - Gm[d][0] - Gm[d][1] - Gm[d][2]);
    for (int c = 0; c < 3; ++c) o[3 * (c + 1) + d] = scale * (pv[c + 1][d] + Gm[d][c]);
  }
}

void launch_pair_q(const int32_t *edof, int n_loc, int n_e, int n_q, const double *phi, const double *A, int lda,
                   const double *B, int ldb, int k, double *out, hipStream_t s) {
  if (n_e <= 0) return;
  dim3 gr((n_e + 255) / 256), b(256);
  if (n_loc == 4 && n_q == 8)
    hipLaunchKernelGGL((k_pair_q<4, 8>), gr, b, 0, s, edof, n_e, phi, A, lda, B, ldb, k, out);
  else if (n_loc == 10 && n_q == 27)
    hipLaunchKernelGGL((k_pair_q<10, 27>), gr, b, 0, s, edof, n_e, phi, A, lda, B, ldb, k, out);
  else if (n_loc == 4 && n_q == 27)
    hipLaunchKernelGGL((k_pair_q<4, 27>), gr, b, 0, s, edof, n_e, phi, A, lda, B, ldb, k, out);
  else if (n_loc == 10 && n_q == 8)
    hipLaunchKernelGGL((k_pair_q<10, 8>), gr, b, 0, s, edof, n_e, phi, A, lda, B, ldb, k, out);
}

void launch_pulay_fields(int64_t n, const double *rho, const double *rho_l, const double *eps, const double *vxc_l,
                         const double *gam, const double *V0, const double *Vbc, const double *VHl, const double *W2,
                         double *F, double *G, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_pulay_fields, grid_1d(n), dim3(256), 0, s, n, rho, rho_l, eps, vxc_l, gam, V0, Vbc, VHl,
                       W2, F, G);
}

bool launch_mesh_grad(const double *coords, const int32_t *elems, const int32_t *edof, int n_loc, int n_e, int n_q,
                      const double *phi, const double *dphi, const double *w, const double *bary,
                      const MeshGradPairs &pr, const double *coef, int k, const double *F, const double *G,
                      int n_atoms, const double *Z, const double *R, double scale, double *out, hipStream_t s) {
  if (n_e <= 0) return true;
  dim3 gr((n_e + 127) / 128), b(128);
#define KS_MG(NL, NQ)                                                                                         \
  hipLaunchKernelGGL((k_mesh_grad<NL, NQ>), gr, b, 0, s, coords, elems, edof, n_e, phi, dphi, w, bary, pr, coef, \
                     k, F, G, n_atoms, Z, R, scale, out)
  if (n_loc == 4 && n_q == 8) KS_MG(4, 8);
  else if (n_loc == 10 && n_q == 27) KS_MG(10, 27);
  else if (n_loc == 4 && n_q == 27) KS_MG(4, 27);
  else if (n_loc == 10 && n_q == 8) KS_MG(10, 8);
  else return false;
#undef KS_MG
  return true;
}

// dEdX[n][d] = sum over the (element, local vertex) records of node n of
// the element results, in the order of the records (zero for edge nodes)
__global__ void k_vertex_gather(int n_nodes, const int32_t *__restrict__ ptr, const int32_t *__restrict__ rec,
                                const double *__restrict__ per_elem, double *__restrict__ out) {
  for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < n_nodes; n += gridDim.x * blockDim.x) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int j = ptr[n]; j < ptr[n + 1]; ++j) {
      const int64_t r = rec[j];  // 4 * element + local vertex
      const double *p = per_elem + (r >> 2) * 12 + 3 * (r & 3);
      a0 += p[0];
      a1 += p[1];
      a2 += p[2];
    }
    out[3 * (int64_t)n] = a0;
    out[3 * (int64_t)n + 1] = a1;
    out[3 * (int64_t)n + 2] = a2;
  }
}
void launch_vertex_gather(int n_nodes, const int32_t *ptr, const int32_t *rec, const double *per_elem, double *out,
                          hipStream_t s) {
  if (n_nodes > 0)
    hipLaunchKernelGGL(k_vertex_gather, grid_1d(n_nodes), dim3(256), 0, s, n_nodes, ptr, rec, per_elem, out);
}

// part[blk][3 a + d] = block sums of Wm[n][a0 + a] dEdX[n][d], a < na <= 8
int motion_blocks(int n) {
  int b = (n + 255) / 256;
  return b > 1024 ? 1024 : (b < 1 ? 1 : b);
}
__global__ void __launch_bounds__(256) k_motion_partials(int n_nodes, const double *__restrict__ Wm, int n_atoms,
                                                         int a0, int na, const double *__restrict__ g,
                                                         double *__restrict__ part) {
  __shared__ double sh[16];
  double acc[24];
  for (int j = 0; j < 24; ++j) acc[j] = 0.0;
  for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < n_nodes; n += gridDim.x * blockDim.x) {
    const double g0 = g[3 * (int64_t)n], g1 = g[3 * (int64_t)n + 1], g2 = g[3 * (int64_t)n + 2];
    for (int a = 0; a < na; ++a) {
      const double wv = Wm[(int64_t)n * n_atoms + a0 + a];
      acc[3 * a] += wv * g0;
      acc[3 * a + 1] += wv * g1;
      acc[3 * a + 2] += wv * g2;
    }
  }
  for (int j = 0; j < 3 * na; ++j) {
    const double t = block_sum(acc[j], sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 24 + j] = t;
  }
}
void launch_motion_partials(int n_nodes, const double *Wm, int n_atoms, int a0, int na, const double *g, double *part,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_motion_partials, dim3(motion_blocks(n_nodes)), dim3(256), 0, s, n_nodes, Wm, n_atoms, a0, na,
                     g, part);
}

}  // namespace ks
