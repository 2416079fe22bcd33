// Kernels of the adjoint of one augmented-subspace step: the gradient of the
// step's Kohn-Sham energy with respect to the external potential at the
// quadrature points, and the nuclear forces.
//
// With the inner iteration converged the new orbitals are a stationary point
// of E_KS over the augmented space, so only the explicit V_ext term and the
// dependence of the augmented basis on V_ext (through the boundary value
// problems S psi_hat = b) contribute:
//   g_q = w_q |J| ( rho_q - sum_i Y_i(x_q) psi_hat_i(x_q) ),  S Y = psi_bar_hat.
#include "common.h"
#include "kernels.h"

namespace ks {

static inline dim3 grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

// R[i][j] = Y1[i][j] + (Y2 ? Y2[i][j] : 0) - theta[j] * Y3[i][j]
__global__ void k_residual_cols(int64_t n, int k, const double *__restrict__ Y1,
                                const double *__restrict__ Y2, const double *__restrict__ Y3,
                                const double *__restrict__ theta, double *__restrict__ R) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = Y1[i] - theta[i % k] * Y3[i];
    if (Y2) v += Y2[i];
    R[i] = v;
  }
}
void launch_residual_cols(int N, int k, const double *Y1, const double *Y2, const double *Y3,
                          const double *theta, double *R, hipStream_t s) {
  int64_t n = (int64_t)N * k;
  if (n > 0) hipLaunchKernelGGL(k_residual_cols, grid_for(n), dim3(256), 0, s, n, k, Y1, Y2, Y3, theta, R);
}

// Out = X Mk with X [N][k], Mk [k][k] (row-major), Out [N][k]
__global__ void k_right_mult(int N, int k, const double *__restrict__ X, const double *__restrict__ Mk,
                             double *__restrict__ Out) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * k) return;
  const int64_t i = t / k;
  const int j = (int)(t % k);
  double s = 0.0;
  for (int l = 0; l < k; ++l) s += X[i * k + l] * Mk[l * k + j];
  Out[t] = s;
}
void launch_right_mult(int N, int k, const double *X, const double *Mk, double *Out, hipStream_t s) {
  int64_t n = (int64_t)N * k;
  if (n > 0)
    hipLaunchKernelGGL(k_right_mult, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, k, X, Mk, Out);
}

// g_q = scale * w_q |J| (rho_q - sum_i A_i(x_q) B_i(x_q)), A, B [N][k] over
// interior nodes (zero on the boundary), one element per thread
template <int NLOC, int NQ>
__global__ void __launch_bounds__(256) k_grad_q(const int32_t *__restrict__ edof, int n_e,
                                                const double *__restrict__ phi,
                                                const double *__restrict__ w,
                                                const double *__restrict__ absdet,
                                                const double *__restrict__ A,
                                                const double *__restrict__ Bm, int k,
                                                const double *__restrict__ rho, double scale,
                                                double *__restrict__ g) {
  __shared__ double s_phi[NQ * NLOC];
  __shared__ double s_w[NQ];
  for (int i = threadIdx.x; i < NQ * NLOC; i += blockDim.x) s_phi[i] = phi[i];
  for (int i = threadIdx.x; i < NQ; i += blockDim.x) s_w[i] = w[i];
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
      xa[a] = dof[a] >= 0 ? A[(int64_t)dof[a] * k + i] : 0.0;
      ya[a] = dof[a] >= 0 ? Bm[(int64_t)dof[a] * k + i] : 0.0;
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
  const double dj = absdet[e];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int64_t idx = (int64_t)e * NQ + q;
    g[idx] = scale * s_w[q] * dj * (rho[idx] - acc[q]);
  }
}
void launch_grad_q(const int32_t *edof, int n_loc, int n_e, int n_q, const double *phi,
                   const double *w, const double *absdet, const double *A, const double *B, int k,
                   const double *rho, double scale, double *g, hipStream_t s) {
  if (n_e <= 0) return;
  dim3 gr((n_e + 255) / 256), b(256);
  if (n_loc == 4 && n_q == 8)
    hipLaunchKernelGGL((k_grad_q<4, 8>), gr, b, 0, s, edof, n_e, phi, w, absdet, A, B, k, rho, scale, g);
  else if (n_loc == 10 && n_q == 27)
    hipLaunchKernelGGL((k_grad_q<10, 27>), gr, b, 0, s, edof, n_e, phi, w, absdet, A, B, k, rho, scale, g);
  else if (n_loc == 4 && n_q == 27)
    hipLaunchKernelGGL((k_grad_q<4, 27>), gr, b, 0, s, edof, n_e, phi, w, absdet, A, B, k, rho, scale, g);
  else if (n_loc == 10 && n_q == 8)
    hipLaunchKernelGGL((k_grad_q<10, 8>), gr, b, 0, s, edof, n_e, phi, w, absdet, A, B, k, rho, scale, g);
}

// Reverse mode through the truncated PCG (per-column coefficients).
// Y = a o X + b o Y column by column (a, b device [k]; X may be null)
__global__ void k_col_axpby(int64_t n, int k, const double *__restrict__ a, const double *__restrict__ X,
                            const double *__restrict__ b, double *__restrict__ Y) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int c = (int)(t % k);
  const double y = b[c] == 0.0 ? 0.0 : b[c] * Y[t];  // b = 0 never reads Y
  Y[t] = (X ? a[c] * X[t] : 0.0) + y;
}
void launch_col_axpby(int N, int k, const double *a, const double *X, const double *b, double *Y, hipStream_t s) {
  const int64_t n = (int64_t)N * k;
  if (n > 0) hipLaunchKernelGGL(k_col_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, k, a, X, b, Y);
}
// Rbar += Zbar / d row by row, and dbar[i] -= sum_c Zbar[i][c] Z[i][c] / d[i]
__global__ void k_zbar_back(int N, int k, const double *__restrict__ Zbar, const double *__restrict__ Z,
                            const double *__restrict__ d, double *__restrict__ Rbar, double *__restrict__ dbar) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double di = d[i];
  double acc = 0.0;
  for (int c = 0; c < k; ++c) {
    const double zb = Zbar[(int64_t)i * k + c];
    Rbar[(int64_t)i * k + c] += zb / di;
    acc += zb * Z[(int64_t)i * k + c];
  }
  dbar[i] -= acc / di;
}
void launch_zbar_back(int N, int k, const double *Zbar, const double *Z, const double *d, double *Rbar, double *dbar,
                      hipStream_t s) {
  if (N > 0) hipLaunchKernelGGL(k_zbar_back, dim3((N + 255) / 256), dim3(256), 0, s, N, k, Zbar, Z, d, Rbar, dbar);
}
// g_q += scale w_q |J| sum_c A_c(x_q) B_c(x_q) (A, B [N][k] over interior nodes),
// and with A = null: g_q += w_q |J| sum_a dbar[dof a] phi_a(x_q)^2 (B = dbar)
template <int NLOC, int NQ>
__global__ void __launch_bounds__(256) k_pair_accum(const int32_t *__restrict__ edof, int n_e,
                                                    const double *__restrict__ phi, const double *__restrict__ w,
                                                    const double *__restrict__ absdet, const double *__restrict__ A,
                                                    const double *__restrict__ Bm, int k, double scale,
                                                    double *__restrict__ g) {
  __shared__ double s_phi[NQ * NLOC];
  __shared__ double s_w[NQ];
  for (int i = threadIdx.x; i < NQ * NLOC; i += blockDim.x) s_phi[i] = phi[i];
  for (int i = threadIdx.x; i < NQ; i += blockDim.x) s_w[i] = w[i];
  __syncthreads();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_e) return;
  int dof[NLOC];
#pragma unroll
  for (int a = 0; a < NLOC; ++a) dof[a] = edof[(int64_t)e * NLOC + a];
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  if (A) {
    for (int i = 0; i < k; ++i) {
      double xa[NLOC], ya[NLOC];
#pragma unroll
      for (int a = 0; a < NLOC; ++a) {
        xa[a] = dof[a] >= 0 ? A[(int64_t)dof[a] * k + i] : 0.0;
        ya[a] = dof[a] >= 0 ? Bm[(int64_t)dof[a] * k + i] : 0.0;
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
  } else {
    double da[NLOC];
#pragma unroll
    for (int a = 0; a < NLOC; ++a) da[a] = dof[a] >= 0 ? Bm[dof[a]] : 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double u = 0.0;
#pragma unroll
      for (int a = 0; a < NLOC; ++a) u += da[a] * s_phi[q * NLOC + a] * s_phi[q * NLOC + a];
      acc[q] = u;
    }
  }
  const double dj = absdet[e];
#pragma unroll
  for (int q = 0; q < NQ; ++q) g[(int64_t)e * NQ + q] += scale * s_w[q] * dj * acc[q];
}
void launch_pair_accum(const int32_t *edof, int n_loc, int n_e, int n_q, const double *phi, const double *w,
                       const double *absdet, const double *A, const double *B, int k, double scale, double *g,
                       hipStream_t s) {
  if (n_e <= 0) return;
  dim3 gr((n_e + 255) / 256), b(256);
  if (n_loc == 4 && n_q == 8)
    hipLaunchKernelGGL((k_pair_accum<4, 8>), gr, b, 0, s, edof, n_e, phi, w, absdet, A, B, k, scale, g);
  else if (n_loc == 10 && n_q == 27)
    hipLaunchKernelGGL((k_pair_accum<10, 27>), gr, b, 0, s, edof, n_e, phi, w, absdet, A, B, k, scale, g);
  else if (n_loc == 4 && n_q == 27)
    hipLaunchKernelGGL((k_pair_accum<4, 27>), gr, b, 0, s, edof, n_e, phi, w, absdet, A, B, k, scale, g);
  else if (n_loc == 10 && n_q == 8)
    hipLaunchKernelGGL((k_pair_accum<10, 8>), gr, b, 0, s, edof, n_e, phi, w, absdet, A, B, k, scale, g);
}

// Partial sums over the quadrature points of g_q dV_ext(x_q)/dR_a for up to 8
// nuclei (atoms a0 .. a0+na-1): dV/dR_a = -Z_a (x - R_a) / |x - R_a|^3.
int force_blocks(int n_e) {
  int b = (n_e + 255) / 256;
  return b > 1024 ? 1024 : (b < 1 ? 1 : b);
}
__global__ void __launch_bounds__(256) k_force_partials(const double *__restrict__ coords,
                                                        const int32_t *__restrict__ elems, int n_loc,
                                                        int n_e, int n_q,
                                                        const double *__restrict__ bary,
                                                        const double *__restrict__ g, int a0, int na,
                                                        const double *__restrict__ Z,
                                                        const double *__restrict__ R,
                                                        double *__restrict__ part) {
  __shared__ double sh[16];
  double acc[24];
  for (int j = 0; j < 24; ++j) acc[j] = 0.0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_e; e += gridDim.x * blockDim.x) {
    double X[4][3];
    for (int v = 0; v < 4; ++v)
      for (int d = 0; d < 3; ++d) X[v][d] = coords[3 * (int64_t)elems[(int64_t)e * n_loc + v] + d];
    for (int q = 0; q < n_q; ++q) {
      double x[3] = {0, 0, 0};
      for (int v = 0; v < 4; ++v)
        for (int d = 0; d < 3; ++d) x[d] += bary[q * 4 + v] * X[v][d];
      const double gq = g[(int64_t)e * n_q + q];
      for (int a = 0; a < na; ++a) {
        const double dx = x[0] - R[3 * (a0 + a)], dy = x[1] - R[3 * (a0 + a) + 1],
                     dz = x[2] - R[3 * (a0 + a) + 2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double c = -gq * Z[a0 + a] / (r2 * sqrt(r2));
        acc[3 * a] += c * dx;
        acc[3 * a + 1] += c * dy;
        acc[3 * a + 2] += c * dz;
      }
    }
  }
  for (int j = 0; j < 3 * na; ++j) {
    const double s = block_sum(acc[j], sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 24 + j] = s;
  }
}
void launch_force_partials(const double *coords, const int32_t *elems, int n_loc, int n_e, int n_q,
                           const double *bary, const double *g, int a0, int na, const double *Z,
                           const double *R, double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_force_partials, dim3(force_blocks(n_e)), dim3(256), 0, s, coords, elems, n_loc,
                     n_e, n_q, bary, g, a0, na, Z, R, part);
}

// per-column dot products of two [N][k] blocks: part[blk][k]
int launch_coldots(int N, int k, const double *X, const double *Y, double *part, hipStream_t s) {
  return launch_colsums(N, k, X, Y, part, s);
}

}  // namespace ks
