// Dense parts of the augmented subspace step (Sec. 3.3, eqs. st1-st7):
//  * tall-skinny products C = Z^T Y (N ~ 1e6 rows, <= 256 columns) on the
//    FP64 matrix cores (v_mfma_f64_16x16x4f64), rows staged through LDS,
//    split over workgroups and reduced in a fixed order;
//  * products with the coarse interpolation I_H^h stored as ELL-4 (every fine
//    node lies in one coarse tetrahedron: at most four weights);
//  * the small generalised eigenproblem F_A u = lambda F_B u solved in one
//    workgroup: diagonal scaling, canonical orthogonalisation of F_B and
//    cyclic Jacobi (round-robin parallel ordering) for both symmetric
//    eigenproblems.
#include "common.h"
#include "kernels.h"
#include <algorithm>

namespace ks {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- GEMM TN
constexpr int GT_ROWS = 16;        // rows staged per LDS slab (multiple of 4)
constexpr int GT_THREADS = 512;    // 8 waves
constexpr int GT_MAXC = 256;       // max padded columns per operand

static inline int pad16(int x) { return (x + 15) / 16 * 16; }

static int gemm_blocks(int N) {
  int b = (N + 1023) / 1024;  // at least 1024 rows per workgroup
  return std::max(1, std::min(b, 512));
}
size_t gemm_tn_work_doubles(int N, int ma, int nb) {
  return (size_t)gemm_blocks(N) * pad16(ma) * pad16(nb);
}

// work[blk][ma_p][nb_p] = sum over the block's rows of Z^T Y.  Wave w owns
// the 16x16 output tiles w, w + 8, ...; MAXT bounds the tiles per wave so
// the accumulators stay in registers (static indexing after unrolling).
// SYM: Z^T Y is symmetric (Y = H Z for a symmetric H): only the tiles on and
// above the diagonal are computed
__device__ __forceinline__ void gemm_tile(int t, int tb_n, bool sym, int &ta, int &tb) {
  if (!sym) {
    ta = t / tb_n;
    tb = t - ta * tb_n;
    return;
  }
  // t-th tile of the upper triangle, row by row: row ta holds tb_n - ta tiles
  ta = 0;
  int rem = t;
  while (rem >= tb_n - ta) {
    rem -= tb_n - ta;
    ++ta;
  }
  tb = ta + rem;
}
template <int MAXT, bool SYM>
__global__ void __launch_bounds__(GT_THREADS) k_gemm_tn(int N, int ma, int nb, int ma_p, int nb_p,
                                                       const double *__restrict__ Z, int ldz,
                                                       const double *__restrict__ Y, int ldy,
                                                       double *__restrict__ work, int rows_per_blk) {
  extern __shared__ double sm[];
  double *sZ = sm;                       // [GT_ROWS][ma_p]
  double *sY = sm + GT_ROWS * ma_p;      // [GT_ROWS][nb_p]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = GT_THREADS / 64;
  const int tb_n = nb_p / 16, ntiles = SYM ? tb_n * (tb_n + 1) / 2 : (ma_p / 16) * tb_n;
  f64x4 acc[MAXT];
#pragma unroll
  for (int ti = 0; ti < MAXT; ++ti) acc[ti] = (f64x4){0.0, 0.0, 0.0, 0.0};
  const int r0 = blockIdx.x * rows_per_blk;
  const int r1 = min(N, r0 + rows_per_blk);
  for (int base = r0; base < r1; base += GT_ROWS) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < GT_ROWS * ma_p; idx += GT_THREADS) {
      const int rr = idx / ma_p, c = idx % ma_p, row = base + rr;
      sZ[idx] = (row < r1 && c < ma) ? Z[(int64_t)row * ldz + c] : 0.0;
    }
    for (int idx = threadIdx.x; idx < GT_ROWS * nb_p; idx += GT_THREADS) {
      const int rr = idx / nb_p, c = idx % nb_p, row = base + rr;
      sY[idx] = (row < r1 && c < nb) ? Y[(int64_t)row * ldy + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ti = 0; ti < MAXT; ++ti) {
      const int t = wave + ti * nwaves;
      if (t < ntiles) {
        int ta, tb;
        gemm_tile(t, tb_n, SYM, ta, tb);
        f64x4 c = acc[ti];
#pragma unroll
        for (int kk = 0; kk < GT_ROWS; kk += 4) {
          const int rr = kk + (lane >> 4);
          const double a = sZ[rr * ma_p + ta * 16 + (lane & 15)];
          const double b = sY[rr * nb_p + tb * 16 + (lane & 15)];
          c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
        }
        acc[ti] = c;
      }
    }
  }
  // accumulator layout of v_mfma_f64_16x16x4f64 (measured): lane l, item r
  // holds D[l/16 + 4 r][l % 16]; A and B lanes hold A[l%16][l/16], B[l/16][l%16]
  double *out = work + (int64_t)blockIdx.x * ma_p * nb_p;
#pragma unroll
  for (int ti = 0; ti < MAXT; ++ti) {
    const int t = wave + ti * nwaves;
    if (t < ntiles) {
      int ta, tb;
      gemm_tile(t, tb_n, SYM, ta, tb);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ta * 16 + (lane >> 4) + 4 * r, col = tb * 16 + (lane & 15);
        out[(int64_t)row * nb_p + col] = acc[ti][r];
      }
    }
  }
}

// sym: entries below the diagonal tiles come from their mirror
__global__ void k_gemm_reduce(int nblk, int ma, int nb, int ma_p, int nb_p,
                              const double *__restrict__ work, double *__restrict__ C, int ldc, int sym) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ma * nb) return;
  int a = idx / nb, b = idx % nb;
  const int ca = a, cb = b;
  if (sym && a / 16 > b / 16) {
    const int t = a;
    a = b;
    b = t;
  }
  double s = 0.0;
  for (int k = 0; k < nblk; ++k) s += work[(int64_t)k * ma_p * nb_p + a * nb_p + b];
  C[(int64_t)ca * ldc + cb] = s;
}

template <bool SYM>
static void gemm_tn_t(int N, int ma, int nb, const double *Z, int ldz, const double *Y, int ldy, double *C,
                      int ldc, double *work, hipStream_t s) {
  const int ma_p = pad16(ma), nb_p = pad16(nb);
  const int nblk = gemm_blocks(N);
  int rows_per_blk = (N + nblk - 1) / nblk;
  rows_per_blk = (rows_per_blk + GT_ROWS - 1) / GT_ROWS * GT_ROWS;
  const size_t shm = sizeof(double) * GT_ROWS * (ma_p + nb_p);
  const int tn = nb_p / 16, ntiles = SYM ? tn * (tn + 1) / 2 : (ma_p / 16) * tn;
  const int per_wave = (ntiles + 7) / 8;
  dim3 g(nblk), b(GT_THREADS);
#define KS_GT(T) \
  hipLaunchKernelGGL((k_gemm_tn<T, SYM>), g, b, shm, s, N, ma, nb, ma_p, nb_p, Z, ldz, Y, ldy, work, rows_per_blk)
  if (per_wave <= 2) KS_GT(2);
  else if (per_wave <= 4) KS_GT(4);
  else if (per_wave <= 8) KS_GT(8);
  else if (per_wave <= 16) KS_GT(16);
  else KS_GT(32);
#undef KS_GT
  hipLaunchKernelGGL(k_gemm_reduce, dim3((ma * nb + 255) / 256), dim3(256), 0, s, nblk, ma, nb, ma_p,
                     nb_p, work, C, ldc, SYM ? 1 : 0);
}
void launch_gemm_tn(int N, int ma, int nb, const double *Z, int ldz, const double *Y, int ldy,
                    double *C, int ldc, double *work, size_t work_doubles, hipStream_t s) {
  (void)work_doubles;
  gemm_tn_t<false>(N, ma, nb, Z, ldz, Y, ldy, C, ldc, work, s);
}
void launch_gemm_tn_sym(int N, int m, const double *Z, int ldz, const double *Y, int ldy, double *C, int ldc,
                        double *work, hipStream_t s) {
  gemm_tn_t<true>(N, m, m, Z, ldz, Y, ldy, C, ldc, work, s);
}

// ------------------------------------------------------------ ELL-4 P
__global__ void k_ellP_times(int N, const int32_t *__restrict__ Pidx, const double *__restrict__ Pw,
                             const double *__restrict__ T, int ldt, int k, double alpha,
                             const double *__restrict__ Y, int ldy, double *__restrict__ Out, int ldo) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * k) return;
  const int i = (int)(t / k), j = (int)(t % k);
  double s = 0.0;
  for (int c = 0; c < 4; ++c) {
    const int id = Pidx[4 * (int64_t)i + c];
    if (id >= 0) s += Pw[4 * (int64_t)i + c] * T[(int64_t)id * ldt + j];
  }
  s *= alpha;
  if (Y) s += Y[(int64_t)i * ldy + j];
  Out[(int64_t)i * ldo + j] = s;
}
void launch_ellP_times(int N, const int32_t *Pidx, const double *Pw, const double *T, int ldt, int k,
                       double alpha, const double *Y, int ldy, double *Out, int ldo, hipStream_t s) {
  int64_t n = (int64_t)N * k;
  if (n > 0)
    hipLaunchKernelGGL(k_ellP_times, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, Pidx, Pw,
                       T, ldt, k, alpha, Y, ldy, Out, ldo);
}

// Psi = Z U with Z = [P | tail]: P part through the ELL form
__global__ void k_zu(int N, const int32_t *__restrict__ Pidx, const double *__restrict__ Pw, int n_H,
                     const double *__restrict__ Z, int ldz, int kt, const double *__restrict__ U,
                     int k, double *__restrict__ Psi) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * k) return;
  const int i = (int)(t / k), j = (int)(t % k);
  double s = 0.0;
  for (int c = 0; c < 4; ++c) {
    const int id = Pidx[4 * (int64_t)i + c];
    if (id >= 0) s += Pw[4 * (int64_t)i + c] * U[(int64_t)id * k + j];
  }
  const double *zr = Z + (int64_t)i * ldz + n_H;
  for (int a = 0; a < kt; ++a) s += zr[a] * U[(int64_t)(n_H + a) * k + j];
  Psi[t] = s;
}
// The same with U staged in LDS and four output columns per lane (k % 4 == 0,
// (n_H + kt) k doubles <= 64 KB): the Z row a lane group shares is read once
// per four columns.
__global__ void __launch_bounds__(256) k_zu4(int N, const int32_t *__restrict__ Pidx, const double *__restrict__ Pw,
                                             int n_H, const double *__restrict__ Z, int ldz, int kt,
                                             const double *__restrict__ U, int k, double *__restrict__ Psi) {
  extern __shared__ double s_u[];  // [(n_H + kt)][k]
  const int m = n_H + kt;
  for (int idx = threadIdx.x; idx < m * k; idx += blockDim.x) s_u[idx] = U[idx];
  __syncthreads();
  const int CG = k / 4;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * CG) return;
  const int i = (int)(t / CG), c0 = (int)(t - (int64_t)i * CG) * 4;
  f64x4 acc = (f64x4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int id = Pidx[4 * (int64_t)i + c];
    if (id >= 0) {
      const double w = Pw[4 * (int64_t)i + c];
      const f64x4 u = *reinterpret_cast<const f64x4 *>(s_u + id * k + c0);
      acc += w * u;
    }
  }
  const double *zr = Z + (int64_t)i * ldz + n_H;
  for (int a = 0; a < kt; ++a) {
    const double z = zr[a];
    const f64x4 u = *reinterpret_cast<const f64x4 *>(s_u + (n_H + a) * k + c0);
    acc += z * u;
  }
  *reinterpret_cast<f64x4 *>(Psi + (int64_t)i * k + c0) = acc;
}
void launch_zu(int N, const int32_t *Pidx, const double *Pw, int n_H, const double *Z, int ldz, int kt,
               const double *U, int k, double *Psi, hipStream_t s) {
  int64_t n = (int64_t)N * k;
  if (n <= 0) return;
  const size_t lds = sizeof(double) * (size_t)(n_H + kt) * k;
  if (k % 4 == 0 && lds <= 65536) {
    const int64_t nt = (int64_t)N * (k / 4);
    hipLaunchKernelGGL(k_zu4, dim3((unsigned)((nt + 255) / 256)), dim3(256), lds, s, N, Pidx, Pw, n_H, Z, ldz,
                       kt, U, k, Psi);
    return;
  }
  hipLaunchKernelGGL(k_zu, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, Pidx, Pw, n_H, Z,
                     ldz, kt, U, k, Psi);
}

// Out[i][j] (row stride ldo) = sum_{a < m} S[i][a] C[a][j] for j < k: a tall
// block times a small matrix, C (m x k, row-major) staged in LDS, four output
// columns per lane when k % 4 == 0.
__global__ void __launch_bounds__(256) k_tsmm(int N, int m, const double *__restrict__ S, int lds,
                                              const double *__restrict__ C, int k, double *__restrict__ Out,
                                              int ldo) {
  extern __shared__ double s_c[];  // [m][k]
  for (int idx = threadIdx.x; idx < m * k; idx += blockDim.x) s_c[idx] = C[idx];
  __syncthreads();
  const int VW = (k % 4 == 0) ? 4 : 1, CG = k / VW;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * CG) return;
  const int i = (int)(t / CG), c0 = (int)(t - (int64_t)i * CG) * VW;
  const double *sr = S + (int64_t)i * lds;
  if (VW == 4) {
    f64x4 acc = (f64x4){0.0, 0.0, 0.0, 0.0};
    for (int a = 0; a < m; ++a) acc += sr[a] * *reinterpret_cast<const f64x4 *>(s_c + a * k + c0);
    double *o = Out + (int64_t)i * ldo + c0;
    o[0] = acc.x; o[1] = acc.y; o[2] = acc.z; o[3] = acc.w;
  } else {
    double acc = 0.0;
    for (int a = 0; a < m; ++a) acc += sr[a] * s_c[a * k + c0];
    Out[(int64_t)i * ldo + c0] = acc;
  }
}
int launch_tsmm(int N, int m, const double *S, int lds, const double *C, int k, double *Out, int ldo,
                hipStream_t s) {
  const size_t lb = sizeof(double) * (size_t)m * k;
  if (lb > 64 * 1024) return -1;
  const int CG = (k % 4 == 0) ? k / 4 : k;
  const int64_t nt = (int64_t)N * CG;
  if (nt > 0)
    hipLaunchKernelGGL(k_tsmm, dim3((unsigned)((nt + 255) / 256)), dim3(256), lb, s, N, m, S, lds, C, k, Out, ldo);
  return 0;
}

// LOBPCG residual block (rows of stride ld): R = HX - MX diag(theta); W =
// D^-1 R (stride ldw); per-block column sums of R^2 (part[b][j]) and MX^2
// (part[b][k + j]) in a fixed order.  blockDim = (256 / k) k threads: thread
// t owns column t % k of every (256 / k)-th row of the block's rows.
__global__ void __launch_bounds__(256) k_lobpcg_resid(int N, int k, int ld, const double *__restrict__ HX,
                                                      const double *__restrict__ MX,
                                                      const double *__restrict__ theta,
                                                      const double *__restrict__ dinv, double *__restrict__ W,
                                                      int ldw, double *__restrict__ part) {
  __shared__ double s_r[256], s_m[256];
  const int rpi = blockDim.x / k;
  const int j = threadIdx.x % k, r0 = threadIdx.x / k;
  const double th = theta[j];
  double sr = 0.0, sm = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * rpi + r0; i < N; i += (int64_t)gridDim.x * rpi) {
    const double mx = MX[i * ld + j];
    const double r = HX[i * ld + j] - th * mx;
    W[i * ldw + j] = r * dinv[i];
    sr += r * r;
    sm += mx * mx;
  }
  s_r[threadIdx.x] = sr;
  s_m[threadIdx.x] = sm;
  __syncthreads();
  if ((int)threadIdx.x < k) {
    double a = 0.0, b = 0.0;
    for (int u = 0; u < rpi; ++u) {
      a += s_r[u * k + threadIdx.x];
      b += s_m[u * k + threadIdx.x];
    }
    part[(int64_t)blockIdx.x * 2 * k + threadIdx.x] = a;
    part[(int64_t)blockIdx.x * 2 * k + k + threadIdx.x] = b;
  }
}
int launch_lobpcg_resid(int N, int k, int ld, const double *HX, const double *MX, const double *theta,
                        const double *dinv, double *W, int ldw, double *part, int max_blocks, hipStream_t s) {
  if (k < 1 || k > 256) return -1;
  const int rpi = 256 / k, tpb = rpi * k;
  int nb = (int)std::min<int64_t>(((int64_t)N + rpi - 1) / rpi, max_blocks);
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_lobpcg_resid, dim3(nb), dim3(tpb), 0, s, N, k, ld, HX, MX, theta, dinv, W, ldw, part);
  return nb;
}
// dinv[i] = 1 / (a dK[i] + b dM[i])
__global__ void k_prec_diag(int N, double a, const double *__restrict__ dK, double b, const double *__restrict__ dM,
                            double *__restrict__ dinv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dinv[i] = 1.0 / (a * dK[i] + b * dM[i]);
}
void launch_prec_diag(int N, double a, const double *dK, double b, const double *dM, double *dinv, hipStream_t s) {
  if (N > 0) hipLaunchKernelGGL(k_prec_diag, dim3((N + 255) / 256), dim3(256), 0, s, N, a, dK, b, dM, dinv);
}

// Coarse blocks of the projection F = Z^T H Z, Z = [P | T], P the coarse
// interpolation in ELL form (4 (index, weight) per fine row, the valid
// indices of a row distinct: the vertices of one coarse tetrahedron).  One wavefront
// per block of CP_ROWS consecutive rows; the block's own coarse indices
// (those of its rows' P rows, list `own`) and its neighbours' (those of the
// P rows of its rows' columns, list `nbr`) are given.  Partials (fixed
// order, no atomics):
//   pp[u][v] = sum_{i in block} P[i][own_u] (H P)[i][nbr_v]
//   pt[u][j] = sum_{i in block} P[i][own_u] Y[i][j]      (Y = H T, [N][k])
__global__ void __launch_bounds__(CP_ROWS) k_proj_coarse(int N, int n_H, int k, int kmax,
                                                         const int32_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ col,
                                                         const double *__restrict__ H,
                                                         const int32_t *__restrict__ Pidx,
                                                         const double *__restrict__ Pw,
                                                         const double *__restrict__ Y,
                                                         const int32_t *__restrict__ uoff,
                                                         const int32_t *__restrict__ ulist,
                                                         const int32_t *__restrict__ noff,
                                                         const int32_t *__restrict__ nlist,
                                                         const int64_t *__restrict__ ppoff,
                                                         const int64_t *__restrict__ ptoff, double *__restrict__ pp,
                                                         double *__restrict__ pt, int ldt, int ldo) {
  extern __shared__ double s_dyn[];
  // (H P)[i][nbr_v] at pitch lt = ldt + 1: slot ldt takes the products of
  // absent (-1) P entries and is never read
  const int lt = ldt + 1;
  double *s_t = s_dyn;                           // [CP_ROWS][lt]
  double *s_p = s_dyn + CP_ROWS * lt;            // [CP_ROWS][ldo]: P[i][own_u]
  double *s_y = s_p + CP_ROWS * ldo;             // [CP_ROWS][k]: Y[i][j]
  __shared__ int16_t s_map[256];                 // coarse index -> position in nbr (-1)
  __shared__ int16_t s_umap[256];                // coarse index -> position in own (-1)
  const int b = blockIdx.x, r0 = b * CP_ROWS, nr = min(CP_ROWS, N - r0);
  const int u0 = uoff[b], nu = uoff[b + 1] - u0, v0 = noff[b], nv = noff[b + 1] - v0;
  const int t = threadIdx.x;
  for (int i = t; i < n_H; i += CP_ROWS) {
    s_map[i] = -1;
    s_umap[i] = -1;
  }
  for (int i = t; i < CP_ROWS * (lt + ldo); i += CP_ROWS) s_dyn[i] = 0.0;
  __syncthreads();
  for (int v = t; v < nv; v += CP_ROWS) s_map[nlist[v0 + v]] = (int16_t)v;
  for (int u = t; u < nu; u += CP_ROWS) s_umap[ulist[u0 + u]] = (int16_t)u;
  // Y rows of the block (coalesced)
  for (int i = t; i < nr * k; i += CP_ROWS) s_y[i] = Y[(int64_t)r0 * k + i];
  __syncthreads();
  if (t < nr) {
    const int i = r0 + t;
    for (int c = 0; c < 4; ++c) {
      const int I = Pidx[4 * (int64_t)i + c];
      if (I >= 0) s_p[t * ldo + s_umap[I]] = Pw[4 * (int64_t)i + c];
    }
    double *ti = s_t + t * lt;
    const int jb = rowptr[i], je = rowptr[i + 1];
    // four nonzeros at a time: their columns, values and P rows are loaded
    // before any of them is accumulated
    for (int jj = jb; jj < je; jj += 4) {
      int j4[4];
      double h4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool ok = jj + u < je;
        j4[u] = ok ? col[jj + u] : i;
        h4[u] = ok ? H[jj + u] : 0.0;
      }
      int4 pi[4];
      double2 pa[4], pb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        pi[u] = *reinterpret_cast<const int4 *>(Pidx + 4 * (int64_t)j4[u]);
        pa[u] = *reinterpret_cast<const double2 *>(Pw + 4 * (int64_t)j4[u]);
        pb[u] = *reinterpret_cast<const double2 *>(Pw + 4 * (int64_t)j4[u] + 2);
      }
      // a P row's valid slots are distinct, so its four accumulators are
      // read together, then written (one LDS round trip per nonzero, not
      // four); nonzeros follow one another, as their slots may repeat
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a0 = pi[u].x >= 0 ? s_map[pi[u].x] : ldt, a1 = pi[u].y >= 0 ? s_map[pi[u].y] : ldt;
        const int a2 = pi[u].z >= 0 ? s_map[pi[u].z] : ldt, a3 = pi[u].w >= 0 ? s_map[pi[u].w] : ldt;
        const double v0 = ti[a0], v1 = ti[a1], v2 = ti[a2], v3 = ti[a3];
        ti[a0] = v0 + h4[u] * pa[u].x;
        ti[a1] = v1 + h4[u] * pa[u].y;
        ti[a2] = v2 + h4[u] * pb[u].x;
        ti[a3] = v3 + h4[u] * pb[u].y;
      }
    }
  }
  __syncthreads();
  double *ppb = pp + ppoff[b];
  for (int o = t; o < nu * nv; o += CP_ROWS) {
    const int u = o / nv, v = o - u * nv;
    double acc = 0.0;
    for (int r = 0; r < nr; ++r) acc += s_p[r * ldo + u] * s_t[r * lt + v];
    ppb[o] = acc;
  }
  double *ptb = pt + ptoff[b];
  for (int o = t; o < nu * k; o += CP_ROWS) {
    const int u = o / k, j = o - u * k;
    double acc = 0.0;
    for (int r = 0; r < nr; ++r) acc += s_p[r * ldo + u] * s_y[r * k + j];
    ptb[u * kmax + j] = acc;
  }
}
// F[I][J] = sum of the pp partials listed for (I, J), ascending; F[I][n_H + j]
// = F[n_H + j][I] = sum of the pt partials listed for I (at offset j).  One
// wavefront per output: lane l sums the entries l, l + 64, ... in order, then
// a fixed butterfly combines the lanes.
__global__ void __launch_bounds__(256) k_proj_gather(int n_H, int k, int m, const int32_t *__restrict__ gpp_ptr,
                                                     const int64_t *__restrict__ gpp_idx,
                                                     const double *__restrict__ pp,
                                                     const int32_t *__restrict__ gpt_ptr,
                                                     const int64_t *__restrict__ gpt_idx,
                                                     const double *__restrict__ pt, double *__restrict__ F) {
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (o < n_H * n_H) {
    double acc = 0.0;
    for (int q = gpp_ptr[o] + lane; q < gpp_ptr[o + 1]; q += 64) acc += pp[gpp_idx[q]];
    acc = wave_sum(acc);
    if (lane == 0) F[(int64_t)(o / n_H) * m + (o % n_H)] = acc;
  } else if (o < n_H * n_H + n_H * k) {
    const int p = o - n_H * n_H, I = p / k, j = p - I * k;
    double acc = 0.0;
    for (int q = gpt_ptr[I] + lane; q < gpt_ptr[I + 1]; q += 64) acc += pt[gpt_idx[q] + j];
    acc = wave_sum(acc);
    if (lane == 0) {
      F[(int64_t)I * m + n_H + j] = acc;
      F[(int64_t)(n_H + j) * m + I] = acc;
    }
  }
}
int launch_proj_coarse(int N, int n_H, int k, int kmax, int nblk, int ldt, int ldo, const int32_t *rowptr,
                       const int32_t *col,
                       const double *H, const int32_t *Pidx, const double *Pw, const double *Y, const int32_t *uoff,
                       const int32_t *ulist, const int32_t *noff, const int32_t *nlist, const int64_t *ppoff,
                       const int64_t *ptoff, double *pp, double *pt, const int32_t *gpp_ptr, const int64_t *gpp_idx,
                       const int32_t *gpt_ptr, const int64_t *gpt_idx, double *F, int m, hipStream_t s) {
  if (n_H > 256 || k > kmax) return -1;
  const size_t lds = sizeof(double) * (size_t)CP_ROWS * (ldt + 1 + ldo + k);
  if (lds > 60 * 1024) return -1;
  hipLaunchKernelGGL(k_proj_coarse, dim3(nblk), dim3(CP_ROWS), lds, s, N, n_H, k, kmax, rowptr, col, H, Pidx, Pw,
                     Y, uoff, ulist, noff, nlist, ppoff, ptoff, pp, pt, ldt, ldo);
  const int nout = n_H * n_H + n_H * k;
  hipLaunchKernelGGL(k_proj_gather, dim3((nout + 3) / 4), dim3(256), 0, s, n_H, k, m, gpp_ptr, gpp_idx, pp,
                     gpt_ptr, gpt_idx, pt, F);
  return 0;
}

__global__ void k_small_gemm(int m, int n, int p, const double *__restrict__ A, int lda,
                             const double *__restrict__ B, int ldb, double *__restrict__ C, int ldc,
                             double beta) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * n) return;
  const int i = t / n, j = t % n;
  double s = 0.0;
  for (int a = 0; a < p; ++a) s += A[(int64_t)i * lda + a] * B[(int64_t)a * ldb + j];
  C[(int64_t)i * ldc + j] = (beta == 0.0 ? 0.0 : beta * C[(int64_t)i * ldc + j]) + s;
}
void launch_small_gemm(int m, int n, int p, const double *A, int lda, const double *B, int ldb,
                       double *C, int ldc, double beta, hipStream_t s) {
  if (m * n > 0)
    hipLaunchKernelGGL(k_small_gemm, dim3((m * n + 255) / 256), dim3(256), 0, s, m, n, p, A, lda, B,
                       ldb, C, ldc, beta);
}

__global__ void k_dense_P(int N, const int32_t *__restrict__ Pidx, const double *__restrict__ Pw,
                          int n_H, double *__restrict__ Z, int ldz) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * n_H) return;
  const int i = (int)(t / n_H), c = (int)(t % n_H);
  double s = 0.0;
  for (int a = 0; a < 4; ++a)
    if (Pidx[4 * (int64_t)i + a] == c) s += Pw[4 * (int64_t)i + a];
  Z[(int64_t)i * ldz + c] = s;
}
void launch_dense_P(int N, const int32_t *Pidx, const double *Pw, int n_H, double *Z, int ldz,
                    hipStream_t s) {
  int64_t n = (int64_t)N * n_H;
  if (n > 0)
    hipLaunchKernelGGL(k_dense_P, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, Pidx, Pw, n_H,
                       Z, ldz);
}
__global__ void k_copy_cols(int N, int k, const double *__restrict__ X, int ldx,
                            double *__restrict__ Z, int ldz, int c0) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * k) return;
  const int i = (int)(t / k), j = (int)(t % k);
  Z[(int64_t)i * ldz + c0 + j] = X[(int64_t)i * ldx + j];
}
void launch_copy_cols(int N, int k, const double *X, int ldx, double *Z, int ldz, int c0,
                      hipStream_t s) {
  int64_t n = (int64_t)N * k;
  if (n > 0)
    hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, k, X, ldx, Z,
                       ldz, c0);
}
__global__ void k_zero_cols(int N, int c0, int c1, double *__restrict__ Z, int ldz) {
  const int w = c1 - c0;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * w) return;
  Z[(t / w) * ldz + c0 + (t % w)] = 0.0;
}
void launch_zero_cols(int N, int c0, int c1, double *Z, int ldz, hipStream_t s) {
  int64_t n = (int64_t)N * (c1 - c0);
  if (n > 0)
    hipLaunchKernelGGL(k_zero_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, c0, c1, Z,
                       ldz);
}

// ----------------------------------------------------- small eigensolver
constexpr int EIG_THREADS = 1024;
constexpr int EIG_MAXN = 256;

size_t small_eig_work_doubles(int m) { return (size_t)6 * m * m + 8 * m + 64; }

// Cyclic Jacobi on the symmetric n x n matrix A (ld n, global memory),
// accumulating eigenvectors in V (V := V J).  Round-robin ordering: n/2
// disjoint pairs rotated per round, n-1 rounds per sweep.  A pair is
// rotated only while |a_pq| exceeds 1e-15 sqrt(|a_pp a_qq|) (and an absolute
// floor); the sweep loop ends when a whole sweep rotates nothing.
__device__ int jacobi_eig(int n, double *A, double *V, int *s_top, int *s_bot, int *s_p, int *s_q,
                          double *s_c, double *s_s, int *s_cnt, double *s_red) {
  const int tid = threadIdx.x;
  const int ne = (n + 1) & ~1, h = ne / 2;
  for (int idx = tid; idx < n * n; idx += blockDim.x) V[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
  // Frobenius norm for the absolute floor
  double loc = 0.0;
  for (int idx = tid; idx < n * n; idx += blockDim.x) loc += A[idx] * A[idx];
  double fro2 = block_sum(loc, s_red);
  if (tid == 0) s_red[16] = sqrt(fro2);
  for (int t = tid; t < h; t += blockDim.x) {
    s_top[t] = 2 * t;
    s_bot[t] = 2 * t + 1;
  }
  __syncthreads();
  const double floor_abs = 1e-300 + 1e-18 * s_red[16];
  int sweeps = 0;
  for (; sweeps < 60; ++sweeps) {
    if (tid == 0) *s_cnt = 0;
    __syncthreads();
    for (int round = 0; round < ne - 1; ++round) {
      for (int t = tid; t < h; t += blockDim.x) {
        int p = s_top[t], q = s_bot[t];
        if (p > q) { int x = p; p = q; q = x; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          const double app = A[p * n + p], aqq = A[q * n + q];
          if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs) {
            const double th = (aqq - app) / (2.0 * apq);
            double tt;
            if (fabs(th) > 1e150) tt = 0.5 / th;
            else tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            s = tt * c;
            atomicAdd(s_cnt, 1);
          }
        }
        s_p[t] = p; s_q[t] = q; s_c[t] = c; s_s[t] = s;
      }
      __syncthreads();
      // rows p, q of A
      for (int idx = tid; idx < h * n; idx += blockDim.x) {
        const int t = idx / n, j = idx % n;
        const double s = s_s[t];
        if (s == 0.0 || s_q[t] >= n) continue;
        const int p = s_p[t], q = s_q[t];
        const double c = s_c[t];
        const double ap = A[p * n + j], aq = A[q * n + j];
        A[p * n + j] = c * ap - s * aq;
        A[q * n + j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns p, q of A and V
      for (int idx = tid; idx < h * n; idx += blockDim.x) {
        const int t = idx / n, i = idx % n;
        const double s = s_s[t];
        if (s == 0.0 || s_q[t] >= n) continue;
        const int p = s_p[t], q = s_q[t];
        const double c = s_c[t];
        const double ap = A[i * n + p], aq = A[i * n + q];
        A[i * n + p] = c * ap - s * aq;
        A[i * n + q] = s * ap + c * aq;
        const double vp = V[i * n + p], vq = V[i * n + q];
        V[i * n + p] = c * vp - s * vq;
        V[i * n + q] = s * vp + c * vq;
      }
      __syncthreads();
      // next round-robin arrangement (player top[0] fixed)
      if (tid == 0) {
        const int lt = s_top[h - 1], b0 = s_bot[0];
        for (int t = h - 1; t >= 2; --t) s_top[t] = s_top[t - 1];
        if (h > 1) s_top[1] = b0;
        for (int t = 0; t < h - 1; ++t) s_bot[t] = s_bot[t + 1];
        s_bot[h - 1] = (h > 1) ? lt : b0;
      }
      __syncthreads();
    }
    const int cnt = *s_cnt;
    __syncthreads();
    if (cnt == 0) break;
  }
  return sweeps;
}

// Lowest k eigenpairs of (FA, FB); see the header for the method.
// work: D[m], A[m*m], V[m*m], X[m*m], T1[m*m], W[m*m], s[m], idx[m] ...
__global__ void __launch_bounds__(EIG_THREADS) k_small_eig(int m, int k, const double *__restrict__ FA,
                                                           int ldfa, const double *__restrict__ FB,
                                                           int ldfb, double *__restrict__ work,
                                                           double *__restrict__ theta,
                                                           double *__restrict__ U, int *info) {
  __shared__ int s_top[EIG_MAXN / 2 + 1], s_bot[EIG_MAXN / 2 + 1], s_p[EIG_MAXN / 2 + 1],
      s_q[EIG_MAXN / 2 + 1];
  __shared__ double s_c[EIG_MAXN / 2 + 1], s_s[EIG_MAXN / 2 + 1];
  __shared__ double s_red[32];
  __shared__ int s_cnt, s_rank, s_keep[EIG_MAXN], s_sel[EIG_MAXN];
  __shared__ double s_sv[EIG_MAXN];
  const int tid = threadIdx.x;
  double *D = work;
  double *A = D + m;
  double *V = A + m * m;
  double *X = V + m * m;
  double *T1 = X + m * m;
  double *W = T1 + m * m;
  // 1. scaling
  for (int i = tid; i < m; i += blockDim.x) {
    const double b = FB[(int64_t)i * ldfb + i];
    D[i] = b > 0.0 ? 1.0 / sqrt(b) : 0.0;
    if (!(b > 0.0)) info[2] = 1;
  }
  __syncthreads();
  for (int idx = tid; idx < m * m; idx += blockDim.x) {
    const int i = idx / m, j = idx % m;
    A[idx] = D[i] * D[j] * 0.5 * (FB[(int64_t)i * ldfb + j] + FB[(int64_t)j * ldfb + i]);
  }
  __syncthreads();
  // 2. eigen-decomposition of the scaled F_B
  const int sw1 = jacobi_eig(m, A, V, s_top, s_bot, s_p, s_q, s_c, s_s, &s_cnt, s_red);
  // 3. keep s > 1e-12 s_max (ascending index order)
  for (int i = tid; i < m; i += blockDim.x) s_sv[i] = A[i * m + i];
  __syncthreads();
  if (tid == 0) {
    double smax = 0.0;
    for (int i = 0; i < m; ++i) smax = fmax(smax, s_sv[i]);
    int r = 0;
    for (int i = 0; i < m; ++i)
      if (s_sv[i] > 1e-12 * smax) s_keep[r++] = i;
    s_rank = r;
  }
  __syncthreads();
  const int r = s_rank;
  // X[i][a] = V[i][keep_a] / sqrt(s_keep_a), ld r
  for (int idx = tid; idx < m * r; idx += blockDim.x) {
    const int i = idx / r, a = idx % r;
    const int c = s_keep[a];
    X[idx] = V[i * m + c] / sqrt(s_sv[c]);
  }
  // scaled F_A into A
  __syncthreads();
  for (int idx = tid; idx < m * m; idx += blockDim.x) {
    const int i = idx / m, j = idx % m;
    A[idx] = D[i] * D[j] * 0.5 * (FA[(int64_t)i * ldfa + j] + FA[(int64_t)j * ldfa + i]);
  }
  __syncthreads();
  // T1 = A X  (m x r)
  for (int idx = tid; idx < m * r; idx += blockDim.x) {
    const int i = idx / r, a = idx % r;
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += A[i * m + j] * X[j * r + a];
    T1[idx] = s;
  }
  __syncthreads();
  // C = X^T T1 (r x r), symmetrised, stored in A (ld r)
  for (int idx = tid; idx < r * r; idx += blockDim.x) {
    const int a = idx / r, b = idx % r;
    if (b < a) continue;
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < m; ++i) {
      s1 += X[i * r + a] * T1[i * r + b];
      s2 += X[i * r + b] * T1[i * r + a];
    }
    const double v = 0.5 * (s1 + s2);
    V[a * r + b] = v;
    V[b * r + a] = v;
  }
  __syncthreads();
  for (int idx = tid; idx < r * r; idx += blockDim.x) A[idx] = V[idx];
  __syncthreads();
  // 4. eigen-decomposition of C; eigenvectors in W (ld r)
  const int sw2 = jacobi_eig(r, A, W, s_top, s_bot, s_p, s_q, s_c, s_s, &s_cnt, s_red);
  // 5. ascending order by rank (ties by index)
  for (int i = tid; i < r; i += blockDim.x) s_sv[i] = A[i * r + i];
  __syncthreads();
  for (int i = tid; i < r; i += blockDim.x) {
    const double v = s_sv[i];
    int rk = 0;
    for (int j = 0; j < r; ++j) rk += (s_sv[j] < v) || (s_sv[j] == v && j < i);
    s_sel[rk] = i;
  }
  __syncthreads();
  for (int i = tid; i < r; i += blockDim.x) theta[i] = s_sv[s_sel[i]];
  // 6. U = D X W_sel (m x k)
  for (int idx = tid; idx < m * k; idx += blockDim.x) {
    const int i = idx / k, j = idx % k;
    double s = 0.0;
    if (j < r) {
      const int c = s_sel[j];
      for (int a = 0; a < r; ++a) s += X[i * r + a] * W[a * r + c];
    }
    U[idx] = D[i] * s;
  }
  __syncthreads();
  // 7. sign: largest-magnitude entry of each column positive (first max)
  for (int j = tid; j < k; j += blockDim.x) {
    int im = 0;
    double vm = -1.0;
    for (int i = 0; i < m; ++i) {
      const double a = fabs(U[i * k + j]);
      if (a > vm) { vm = a; im = i; }
    }
    if (U[im * k + j] < 0.0)
      for (int i = 0; i < m; ++i) U[i * k + j] = -U[i * k + j];
  }
  if (tid == 0) {
    info[0] = r;
    info[1] = sw1 + sw2;
  }
}

// ------------------------------------------- packed-LDS Jacobi (m <= 190)
// The symmetric matrix (padded to even order ne with a zero row/column) is
// kept as its packed upper triangle in LDS.  A sweep is ne - 1 rounds of the
// circle method (player ne - 1 stays, the others turn), each round rotating
// ne/2 disjoint pairs at once: every 2x2 block (pair t1 rows, pair t2
// columns), t1 <= t2, is transformed by J1^T B J2 by one thread, so a round
// has no read/write conflicts.  The eigenvectors are not accumulated here:
// each round's (cos, sin) per pair goes to a log in global memory (written,
// never read back by this kernel), and k_apply_rot replays the log on the
// rows of a matrix over many workgroups.  A pair is rotated while
// |a_pq| > 1e-15 sqrt(|a_pp a_qq|) and above an absolute floor; the sweep
// loop stops after a sweep without rotations.
constexpr int PJ_MAXN = 190;  // packed (190*191/2) doubles = 145 KB of the 160 KB LDS
constexpr int PJ_PACK = (PJ_MAXN * (PJ_MAXN + 1)) / 2;
constexpr int JAC_MAX_SWEEPS = 60;

// doubles of the rotation log for order n: (cos, sin) per pair, round, sweep
__host__ __device__ inline size_t jacobi_log_doubles(int n) {
  const size_t ne = (size_t)((n + 1) & ~1);
  return 2 * (size_t)JAC_MAX_SWEEPS * (ne - 1) * (ne / 2);
}
size_t jacobi_work_doubles(int m) { return jacobi_log_doubles(m) + 2 * (size_t)m + 64; }

__device__ __forceinline__ int pk(int i, int j, int ne) {
  if (i > j) { int t = i; i = j; j = t; }
  return i * ne - (i * (i - 1)) / 2 + (j - i);
}

// pair t of round rho of the circle method over ne players (p < q)
__device__ __forceinline__ void circle_pair(int t, int rho, int ne, int &p, int &q) {
  const int M = ne - 1;
  int x, y;
  if (t == 0) {
    x = rho;
    y = M;
  } else {
    x = rho + t;
    if (x >= M) x -= M;
    y = rho - t;
    if (y < 0) y += M;
  }
  p = min(x, y);
  q = max(x, y);
}

// a rotation of pair (p, q) is due: |a_pq| above the relative threshold and
// the absolute floor
__device__ __forceinline__ bool rot_due(double apq, double app, double aqq, double floor_abs) {
  return fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs;
}

// Returns the number of sweeps run (all of them rotated and are in the log).
// Before each sweep every pair is tested at once: a sweep starting with no
// pair due would rotate nothing, so the loop ends there without running it.
constexpr int JB_MAX = 5;  // 2x2 blocks per thread of the 1024-thread workgroup
static_assert((PJ_MAXN / 2) * (PJ_MAXN / 2 + 1) / 2 <= JB_MAX * EIG_THREADS, "2x2 blocks per thread");
__device__ int jacobi_packed(int n, double *sA, double2 *__restrict__ rot, double2 *s_cs, int2 *s_pq, int *s_cnt,
                             double *s_red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ne = (n + 1) & ~1, h = ne / 2, nblk2 = h * (h + 1) / 2;
  double loc = 0.0;
  for (int idx = tid; idx < ne * (ne + 1) / 2; idx += nt) loc += sA[idx] * sA[idx];
  const double fro2 = block_sum(loc, s_red);
  if (tid == 0) s_red[16] = sqrt(fro2);
  // this thread's 2x2 blocks (t1 <= t2), enumerated over the upper triangle
  int nb = 0, bt1[JB_MAX], bt2[JB_MAX];
  for (int idx = tid; idx < nblk2 && nb < JB_MAX; idx += nt) {
    int t2 = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);  // fixed up below
    while (t2 * (t2 + 1) / 2 > idx) --t2;
    while ((t2 + 1) * (t2 + 2) / 2 <= idx) ++t2;
    bt1[nb] = idx - t2 * (t2 + 1) / 2;
    bt2[nb] = t2;
    ++nb;
  }
  __syncthreads();
  const double floor_abs = 1e-300 + 1e-18 * s_red[16];
  int sweeps = 0;
  for (; sweeps < JAC_MAX_SWEEPS; ++sweeps) {
    // any pair due?
    if (tid == 0) *s_cnt = 0;
    __syncthreads();
    bool any = false;
    for (int idx = tid; idx < n * n && !any; idx += nt) {
      const int p = idx / n, q = idx - p * n;
      if (q > p) any = rot_due(sA[pk(p, q, ne)], sA[pk(p, p, ne)], sA[pk(q, q, ne)], floor_abs);
    }
    if (any) *s_cnt = 1;
    __syncthreads();
    const int cnt = *s_cnt;
    if (cnt == 0) break;
    for (int round = 0; round < ne - 1; ++round) {
      double2 *lg = rot + ((size_t)sweeps * (ne - 1) + round) * h;
      // rotation of each pair of this round
      for (int t = tid; t < h; t += nt) {
        int p, q;
        circle_pair(t, round, ne, p, q);
        double c = 1.0, sn = 0.0;
        if (q < n) {
          const double apq = sA[pk(p, q, ne)], app = sA[pk(p, p, ne)], aqq = sA[pk(q, q, ne)];
          if (rot_due(apq, app, aqq, floor_abs)) {
            const double th = (aqq - app) / (2.0 * apq);
            const double tt = fabs(th) > 1e150 ? 0.5 / th
                                               : (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            sn = tt * c;
          }
        }
        s_cs[t] = make_double2(c, sn);
        s_pq[t] = make_int2(p, q);
        lg[t] = make_double2(c, sn);
      }
      __syncthreads();
      for (int b = 0; b < nb; ++b) {
        const int t1 = bt1[b], t2 = bt2[b];
        const double2 r1 = s_cs[t1], r2 = s_cs[t2];
        const int2 i1 = s_pq[t1], i2 = s_pq[t2];
        const double c1 = r1.x, s1 = r1.y, c2 = r2.x, s2 = r2.y;
        if (s1 == 0.0 && s2 == 0.0) continue;
        const int p1 = i1.x, q1 = i1.y, p2 = i2.x, q2 = i2.y;
        if (t1 == t2) {
          const int ipp = pk(p1, p1, ne), iqq = pk(q1, q1, ne), ipq = pk(p1, q1, ne);
          const double app = sA[ipp], aqq = sA[iqq], apq = sA[ipq];
          sA[ipp] = c1 * c1 * app - 2.0 * c1 * s1 * apq + s1 * s1 * aqq;
          sA[iqq] = s1 * s1 * app + 2.0 * c1 * s1 * apq + c1 * c1 * aqq;
          sA[ipq] = 0.0;
        } else {
          const int i00 = pk(p1, p2, ne), i01 = pk(p1, q2, ne), i10 = pk(q1, p2, ne),
                    i11 = pk(q1, q2, ne);
          const double b00 = sA[i00], b01 = sA[i01], b10 = sA[i10], b11 = sA[i11];
          // rows (p1, q1) by J1^T, then columns (p2, q2) by J2
          const double r00 = c1 * b00 - s1 * b10, r01 = c1 * b01 - s1 * b11;
          const double r10 = s1 * b00 + c1 * b10, r11 = s1 * b01 + c1 * b11;
          sA[i00] = c2 * r00 - s2 * r01;
          sA[i01] = s2 * r00 + c2 * r01;
          sA[i10] = c2 * r10 - s2 * r11;
          sA[i11] = s2 * r10 + c2 * r11;
        }
      }
      __syncthreads();
    }
  }
  return sweeps;
}

// W <- W J_1 J_2 ... : the first nsw logged sweeps of rotations, in order,
// applied to the columns of W (n x n, row-major; the identity first when
// init).  Rows are independent, so each workgroup rotates its own block of
// R = 1024 / (ne/2) rows in LDS; per round, thread (row slot, pair) updates
// two entries, and the next round's (cos, sin) is loaded ahead.
constexpr int AR_THREADS = 1024;
__global__ void __launch_bounds__(AR_THREADS) k_apply_rot(int n, const int *__restrict__ nsw_ptr,
                                                          const double2 *__restrict__ rot, double *__restrict__ W,
                                                          int init) {
  __shared__ double sW[2 * AR_THREADS];  // R n <= (1024 / h) 2h
  const int ne = (n + 1) & ~1, h = ne / 2, R = AR_THREADS / h;
  const int row0 = blockIdx.x * R, tid = threadIdx.x;
  for (int idx = tid; idx < R * n; idx += blockDim.x) {
    const int i = row0 + idx / n, j = idx % n;
    double v = 0.0;
    if (i < n) v = init ? (i == j ? 1.0 : 0.0) : W[(int64_t)i * n + j];
    sW[idx] = v;
  }
  __syncthreads();
  const int slot = tid / h, t = tid - slot * h;
  const bool act = slot < R && row0 + slot < n;
  const int nrounds = min(*nsw_ptr, JAC_MAX_SWEEPS) * (ne - 1);
  double *w = sW + slot * n;
  double2 cs = make_double2(1.0, 0.0);
  if (act && nrounds > 0) cs = rot[t];
  int round = 0;
  for (int g = 0; g < nrounds; ++g) {
    double2 nx = make_double2(1.0, 0.0);
    if (act && g + 1 < nrounds) nx = rot[(size_t)(g + 1) * h + t];
    if (act && cs.y != 0.0) {
      int p, q;
      circle_pair(t, round, ne, p, q);  // q < n whenever the sine is nonzero
      const double wp = w[p], wq = w[q];
      w[p] = cs.x * wp - cs.y * wq;
      w[q] = cs.y * wp + cs.x * wq;
    }
    __syncthreads();
    cs = nx;
    if (++round == ne - 1) round = 0;
  }
  for (int idx = tid; idx < R * n; idx += blockDim.x) {
    const int i = row0 + idx / n;
    if (i < n) W[(int64_t)i * n + idx % n] = sW[idx];
  }
}
static void apply_rot(int n, const int *nsw, const double *rot, double *W, int init, hipStream_t s) {
  const int h = ((n + 1) & ~1) / 2, R = AR_THREADS / h;
  hipLaunchKernelGGL(k_apply_rot, dim3((n + R - 1) / R), dim3(AR_THREADS), 0, s, n, nsw,
                     reinterpret_cast<const double2 *>(rot), W, init);
}

// Canonical orthogonalisation of F_B (once per augmented space):
// D = diag(F_B)^{-1/2}, D F_B D = V s V^T, X = V_keep s_keep^{-1/2} (keep
// s > 1e-12 s_max), X stored [m][r] with ld m.  k_orth (one workgroup) runs
// the Jacobi and selects the kept pairs (s and the kept indices to the tail
// of work); k_apply_rot forms V; k_orth_x forms X.  info[0] = r, info[2] = 1
// on a non-positive diagonal, info[3] = sweeps.
__global__ void __launch_bounds__(EIG_THREADS) k_orth(int m, const double *__restrict__ FB, int ldfb,
                                                      double *__restrict__ D, double *__restrict__ work,
                                                      int *info) {
  extern __shared__ double sA[];
  __shared__ double2 s_cs[PJ_MAXN / 2 + 1];
  __shared__ int2 s_pq[PJ_MAXN / 2 + 1];
  __shared__ double s_red[32], s_sv[PJ_MAXN];
  __shared__ int s_cnt;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ne = (m + 1) & ~1;
  for (int i = tid; i < m; i += nt) {
    const double b = FB[(int64_t)i * ldfb + i];
    D[i] = b > 0.0 ? 1.0 / sqrt(b) : 0.0;
    if (!(b > 0.0)) info[2] = 1;
  }
  __syncthreads();
  for (int idx = tid; idx < ne * ne; idx += nt) {
    const int i = idx / ne, j = idx % ne;
    if (j < i) continue;
    double v = 0.0;
    if (i < m && j < m) v = D[i] * D[j] * 0.5 * (FB[(int64_t)i * ldfb + j] + FB[(int64_t)j * ldfb + i]);
    sA[pk(i, j, ne)] = v;
  }
  __syncthreads();
  const int sw = jacobi_packed(m, sA, reinterpret_cast<double2 *>(work), s_cs, s_pq, &s_cnt, s_red);
  for (int i = tid; i < m; i += nt) s_sv[i] = sA[pk(i, i, ne)];
  __syncthreads();
  double *sv = work + jacobi_log_doubles(m);
  int *keep = reinterpret_cast<int *>(sv + m);
  for (int i = tid; i < m; i += nt) sv[i] = s_sv[i];
  if (tid == 0) {
    double smax = 0.0;
    for (int i = 0; i < m; ++i) smax = fmax(smax, s_sv[i]);
    int r = 0;
    for (int i = 0; i < m; ++i)
      if (s_sv[i] > 1e-12 * smax) keep[r++] = i;
    info[0] = r;
    info[3] = sw;
  }
}
// X[i][a] = V[i][keep[a]] / sqrt(s[keep[a]]) for a < r = info[0]
__global__ void k_orth_x(int m, const double *__restrict__ V, const double *__restrict__ work,
                         const int *__restrict__ info, double *__restrict__ X) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = info[0];
  if (idx >= m * r) return;
  const double *sv = work + jacobi_log_doubles(m);
  const int *keep = reinterpret_cast<const int *>(sv + m);
  const int i = idx / r, a = idx % r, c = keep[a];
  X[(int64_t)i * m + a] = V[(int64_t)i * m + c] / sqrt(sv[c]);
}

size_t orth_shared_bytes(int m) {
  const int ne = (m + 1) & ~1;
  return sizeof(double) * (size_t)ne * (ne + 1) / 2;
}
int packed_eig_supported(int m) { return m <= PJ_MAXN; }
static int lds_ready = 0;
// the packed matrix needs more than the default 64 KB of dynamic LDS
static int enable_big_lds() {
  if (lds_ready) return 0;
  const int bytes = (int)orth_shared_bytes(PJ_MAXN);
  if (hipFuncSetAttribute((const void *)k_orth, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) !=
      hipSuccess)
    return -1;
  lds_ready = 1;
  return 0;
}
int launch_orth(int m, const double *FB, int ldfb, double *D, double *V, double *X, double *work, int *info,
                hipStream_t s) {
  if (enable_big_lds() < 0) return -1;
  hipLaunchKernelGGL(k_orth, dim3(1), dim3(EIG_THREADS), orth_shared_bytes(m), s, m, FB, ldfb, D, work, info);
  apply_rot(m, info + 3, work, V, 1, s);
  hipLaunchKernelGGL(k_orth_x, dim3((m * m + 255) / 256), dim3(256), 0, s, m, V, work, info, X);
  return 0;
}

// ---------------------------------------- reduced eigensolve, split form
// The dense products around the Jacobi iteration (r <= 190) run as
// one-thread-per-entry kernels over many workgroups, the eigenvector
// accumulation as the rotation replay; only the Jacobi iteration on the
// matrix itself is one workgroup.

// C = op(A) op(B) + beta C, op = transpose when t* != 0 (row-major, small)
__global__ void k_gemm_small(int m, int n, int p, const double *__restrict__ A, int lda, int ta,
                             const double *__restrict__ B, int ldb, int tb, double *__restrict__ C,
                             int ldc, double beta) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int i = idx / n, j = idx % n;
  double s = 0.0;
  for (int l = 0; l < p; ++l) {
    const double a = ta ? A[(int64_t)l * lda + i] : A[(int64_t)i * lda + l];
    const double b = tb ? B[(int64_t)j * ldb + l] : B[(int64_t)l * ldb + j];
    s += a * b;
  }
  C[(int64_t)i * ldc + j] = beta != 0.0 ? s + beta * C[(int64_t)i * ldc + j] : s;
}
static void gemm_small(int m, int n, int p, const double *A, int lda, int ta, const double *B, int ldb, int tb,
                       double *C, int ldc, hipStream_t s) {
  if (m * n > 0)
    hipLaunchKernelGGL(k_gemm_small, dim3((m * n + 127) / 128), dim3(128), 0, s, m, n, p, A, lda, ta, B, ldb, tb,
                       C, ldc, 0.0);
}
// S = D sym(FA) D  (m x m, ld m)
__global__ void k_scale_sym(int m, const double *__restrict__ FA, int ldfa, const double *__restrict__ D,
                            double *__restrict__ S) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  const int i = idx / m, j = idx % m;
  S[idx] = D[i] * D[j] * 0.5 * (FA[(int64_t)i * ldfa + j] + FA[(int64_t)j * ldfa + i]);
}
// eigenvalues (unsorted, lam) of the symmetric C; rotations to the log
__global__ void __launch_bounds__(EIG_THREADS) k_jacobi_only(int r, const double *__restrict__ C,
                                                             double *__restrict__ rot, double *__restrict__ lam,
                                                             int *info) {
  extern __shared__ double sA[];
  __shared__ double2 s_cs[PJ_MAXN / 2 + 1];
  __shared__ int2 s_pq[PJ_MAXN / 2 + 1];
  __shared__ double s_red[32];
  __shared__ int s_cnt;
  const int ne = (r + 1) & ~1;
  for (int idx = threadIdx.x; idx < ne * ne; idx += blockDim.x) {
    const int a = idx / ne, b = idx % ne;
    if (b < a) continue;
    sA[pk(a, b, ne)] = (a < r && b < r) ? 0.5 * (C[a * r + b] + C[b * r + a]) : 0.0;
  }
  __syncthreads();
  const int sw = jacobi_packed(r, sA, reinterpret_cast<double2 *>(rot), s_cs, s_pq, &s_cnt, s_red);
  for (int i = threadIdx.x; i < r; i += blockDim.x) lam[i] = sA[pk(i, i, ne)];
  if (threadIdx.x == 0) {
    info[0] = r;
    info[1] = sw;
  }
}
// ascending theta; U[:, j] = D .* XW[:, sel_j] for the k lowest, largest-
// magnitude entry of each column positive (one workgroup)
__global__ void __launch_bounds__(256) k_eig_select(int m, int k, int r, const double *__restrict__ lam,
                                                    const double *__restrict__ XW, const double *__restrict__ D,
                                                    double *__restrict__ theta, double *__restrict__ U) {
  __shared__ int s_sel[PJ_MAXN];
  for (int i = threadIdx.x; i < r; i += blockDim.x) {
    const double v = lam[i];
    int rk = 0;
    for (int j = 0; j < r; ++j) rk += (lam[j] < v) || (lam[j] == v && j < i);
    s_sel[rk] = i;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < r; i += blockDim.x) theta[i] = lam[s_sel[i]];
  for (int idx = threadIdx.x; idx < m * k; idx += blockDim.x) {
    const int i = idx / k, j = idx % k;
    U[idx] = j < r ? D[i] * XW[(int64_t)i * r + s_sel[j]] : 0.0;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    int im = 0;
    double vm = -1.0;
    for (int i = 0; i < m; ++i) {
      const double a = fabs(U[i * k + j]);
      if (a > vm) { vm = a; im = i; }
    }
    if (U[im * k + j] < 0.0)
      for (int i = 0; i < m; ++i) U[i * k + j] = -U[i * k + j];
  }
}
int launch_reduced_eig_split(int m, int k, int r, const double *FA, int ldfa, const double *D, const double *X,
                             double *W, int warm, double *S, double *T1, double *T2, double *work, double *lam,
                             double *theta, double *U, int *info, hipStream_t s) {
  if (enable_big_lds() < 0) return -1;
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void *)k_jacobi_only, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)orth_shared_bytes(PJ_MAXN)) != hipSuccess)
      return -1;
    attr = true;
  }
  hipLaunchKernelGGL(k_scale_sym, dim3((m * m + 255) / 256), dim3(256), 0, s, m, FA, ldfa, D, S);
  gemm_small(m, r, m, S, m, 0, X, m, 0, T1, r, s);   // T1 = S X      (m x r)
  gemm_small(r, r, m, X, m, 1, T1, r, 0, T2, r, s);  // T2 = X^T T1   (r x r)
  if (warm) {
    gemm_small(r, r, r, T2, r, 0, W, r, 0, T1, r, s);  // T1 = C W
    gemm_small(r, r, r, W, r, 1, T1, r, 0, T2, r, s);  // T2 = W^T C W
  }
  hipLaunchKernelGGL(k_jacobi_only, dim3(1), dim3(EIG_THREADS), orth_shared_bytes(r), s, r, T2, work, lam, info);
  apply_rot(r, info + 1, work, W, warm ? 0 : 1, s);  // W <- W V (or V)
  gemm_small(m, r, r, X, m, 0, W, r, 0, T1, r, s);  // X W (m x r)
  hipLaunchKernelGGL(k_eig_select, dim3(1), dim3(256), 0, s, m, k, r, lam, T1, D, theta, U);
  return 0;
}

void launch_small_eig(int m, int k, const double *FA, int ldfa, const double *FB, int ldfb,
                      double *work, double *theta, double *U, int *info, hipStream_t s) {
  hipLaunchKernelGGL(k_small_eig, dim3(1), dim3(EIG_THREADS), 0, s, m, k, FA, ldfa, FB, ldfb, work,
                     theta, U, info);
}

// Z[i][j] = R[i][j] / d[i] (the Jacobi preconditioner applied to a block)
__global__ void k_row_div(int64_t n, int k, const double *__restrict__ R, const double *__restrict__ d,
                          double *__restrict__ Z) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) Z[t] = R[t] / d[t / k];
}
void launch_row_div(int N, int k, const double *R, const double *d, double *Z, hipStream_t s) {
  const int64_t n = (int64_t)N * k;
  if (n > 0) hipLaunchKernelGGL(k_row_div, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, k, R, d, Z);
}

}  // namespace ks
