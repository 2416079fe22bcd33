// Launchers of the device kernels (all enqueue on `s`, no synchronisation).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

namespace ks {

// ---------------------------------------------------------------- geometry
// absdet[e] = |det J_e|, gl[e][4][3] = barycentric gradients; bad[0] counts
// elements with det J <= 0.
void launch_geometry(const double *coords, const int32_t *elems, int n_loc, int n_e,
                     double *absdet, double *gl, int32_t *bad, hipStream_t s);

// ---------------------------------------------------------------- assembly
// Element tables in device memory: phi [n_q][n_loc], dphi [n_q][n_loc][4],
// w [n_q].  `list` holds the element ids of one colour.
void launch_assemble_KM(const int32_t *list, int count, int n_loc, int n_q,
                        const int32_t *slot, const double *absdet, const double *gl,
                        const double *phi, const double *dphi, const double *w,
                        double *K, double *M, hipStream_t s);
// out[slot] += sum_q w_q |J| V_q phi_a phi_b (one colour).  pairtab: [n_q][n_pairs]
// products phi_a phi_b for a <= b.
void launch_assemble_potential(const int32_t *list, int count, int n_loc, int n_q,
                               const int32_t *slot, const double *absdet, const double *pairtab,
                               const double *w, const double *V_q, double *out, hipStream_t s);
// Row form of the potential assembly: one record per incidence (element e,
// local node a) of an interior row, grouped by row (incptr) in ascending
// element order: ea = e << 4 | a, off[b] = position of local node b's
// column in the row's CSR column list (255: a boundary column, skipped).
constexpr int ASM_ROWS = 128;  // rows (threads) per workgroup of the row-form assembly
template <int NLOC> struct IncRec;
template <> struct __align__(16) IncRec<10> { uint32_t ea; uint8_t off[12]; };
template <> struct __align__(8) IncRec<4> { uint32_t ea; uint8_t off[4]; };
// out = base + M[V] over the interior pattern (base may be null; out32 =
// (float) out, may be null).  Row blocks of ASM_ROWS rows: rperm [N] holds each
// block's local rows in visiting order; lds_bytes = 8 x the largest block's
// value count (<= assemble_rows_lds_limit()).  Returns -1 when the shape has
// no kernel or the LDS attribute cannot be set.
size_t assemble_rows_lds_limit();
// out[r] = scale sum_(e,a) |J_e| sum_q w_q f_eq phi_a(q) over the incidence
// records of each interior row (the load vector, all of out written), via
// per-element values in be [n_e][n_loc] (device scratch); -1 when the shape
// has no kernel
int launch_load_rows(int N, int n_e, int n_loc, int n_q, const int32_t *incptr, const void *inc,
                     const double *absdet, const double *phi, const double *w, const double *f_q, double scale,
                     double *be, double *out, hipStream_t s);
// phi: [n_q][n_loc] basis values at the quadrature points; phib: the same
// table b-major [n_loc][n_q]
int launch_assemble_rows(int N, int n_loc, int n_q, const int32_t *rowptr, const int32_t *incptr, const void *inc,
                         const uint8_t *rperm, size_t lds_bytes, const double *absdet, const double *phi,
                         const double *phib, const double *w, const double *V_q, const double *base, double *out,
                         float *out32, hipStream_t s);
// out[dof_a] += sum_q w_q |J| f_q phi_a (one colour; dof = interior index or -1).
void launch_load_vector(const int32_t *list, int count, int n_loc, int n_q,
                        const int32_t *edof, const double *absdet, const double *phi,
                        const double *w, const double *f_q, double scale, double *out,
                        hipStream_t s);

// y = a*x + b*y on n doubles; also used for copies (a=1,b=0).
void launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
void launch_fill(int64_t n, double v, double *y, hipStream_t s);
void launch_combine3(int64_t n, double a, const double *x, double b, const double *y, double c,
                     const double *z, double *out, hipStream_t s);
void launch_to_float(int64_t n, const double *x, float *y, hipStream_t s);
// diag[i] = val[slot of (i,i)]
void launch_extract_diag(int N, const int32_t *rowptr, const int32_t *col, const double *val,
                         double *diag, hipStream_t s);

// ------------------------------------------------------------------ fields
void launch_vext(const double *coords, const int32_t *elems, int n_loc, int n_e, int n_q,
                 const double *bary, int n_atoms, const double *Z, const double *R, double *out,
                 hipStream_t s);
// rho_q = sum_i occ_i (sum_a phi_qa X[dof_a][i])^2
void launch_density(const int32_t *edof, int n_loc, int n_e, int n_q, const double *phi,
                    const double *X, int ldx, int k, const double *occ, double *rho, hipStream_t s);
// u_q = sum_a phi_qa U[node_a]  (U over all nodes)
void launch_eval_nodal(const int32_t *elems, int n_loc, int n_e, int n_q, const double *phi,
                       const double *U, double *out, hipStream_t s);
void launch_xc(int64_t n, const double *rho, int mode, double *eps, double *v, hipStream_t s);
// partial sums over (e,q) of dV rho * {1, x, y, z} (stage 1) -> part[nblk][4]
// or of dV rho * {dx, dy, dz, dxdx, dxdy, dxdz, dydy, dydz, dzdz} about c.
int moments_blocks(int n_e);
void launch_moments(const double *coords, const int32_t *elems, int n_loc, int n_e, int n_q,
                    const double *bary, const double *w, const double *absdet, const double *rho,
                    const double *center /*device [3] or null*/, double *part, int nvals,
                    hipStream_t s);
// out[j] = sum_b part[b][j], j < nvals (single block, fixed order)
void launch_reduce_cols(const double *part, int nblk, int nvals, double *out, hipStream_t s);
// multipole boundary values (eq. bd) from mom = {Q, cx, cy, cz, px, py, pz, qxx..qzz}
void launch_multipole(const double *coords, const int32_t *bnodes, int nb, const double *mom,
                      double quad_factor, double *wB, hipStream_t s);
// V[node] = interior value or boundary value
void launch_scatter_nodes(int n_nodes, const int32_t *node2int, const int32_t *node2bnd,
                          const double *vint, const double *vbnd, double *V, hipStream_t s);
// multi weighted dot: out_part[blk][j] = sum dV a_j b_j over the block's points
int wdot_blocks(int64_t npts);
void launch_wdots(int64_t npts, int n_q, const double *absdet, const double *w, int ndots,
                  const double *const *a, const double *const *b, double *part, hipStream_t s);
// out = sum_j c_j x_j  (nvec <= 12)
void launch_lincomb(int64_t n, int nvec, const double *coef_dev, const double *const *x,
                    double *out, hipStream_t s);

// ------------------------------------------------------ nonnested meshes
// Interpolation weights of npts points in a coarse P1 tetrahedral mesh
// (Algorithm 1, host): vid/w [npts][4] = the containing element's vertices
// and barycentric coordinates.  Returns 0, -1 on a bad mesh, -2 if some
// point could not be placed (its weights are then those of the nearest
// element's projection).
int nonnested_weights(int ncv, const double *cv, int nct, const int32_t *ctet, int npts, const double *pts,
                      int32_t *vid, double *w);
// the same location on the GPU for device points pts_dev [npts][3]; vid_dev,
// w_dev device [npts][4]; the search index is built on the host from the
// host mesh arrays.  0, -1 bad vertex ids, -2 degenerate weights, -3 device
// allocation, -4 HIP error
int nonnested_weights_device(int ncv, const double *cv, int nct, const int32_t *ctet, int npts, const double *pts_dev,
                             int32_t *vid_dev, double *w_dev, hipStream_t s);
void launch_interior_coords(int nn, const int32_t *node2int, const double *coords, double *pts, hipStream_t s);
void launch_ell_from_vertices(int npts, const int32_t *vid, const double *w, const int32_t *sint, int32_t *idx,
                              double *wo, hipStream_t s);

// ------------------------------------------------------------- sparse / CG
struct ColState;  // per-column PCG scalars, defined in spmm_cg.hip

// Y = A X (mode 0) or Y = B - A X (mode 1) for [N][k] blocks, row stride ldx/ldy.
// `ord`: device [N] schedule (permutation) in which rows are processed, or
// nullptr for the natural order.  A spatially local schedule keeps the
// gathered rows of X in L2; the results do not depend on it.
void launch_spmm(int N, const int32_t *rowptr, const int32_t *col, const double *val,
                 const double *X, int ldx, double *Y, int ldy, int k, const double *B, int ldb,
                 int mode, const int32_t *ord, hipStream_t s);
void launch_spmm_f32(int N, const int32_t *rowptr, const int32_t *col, const float *val,
                     const float *X, float *Y, int k, const int32_t *ord, hipStream_t s);
// Y[i][j] *= scale[j]
void launch_scale_cols(int N, int k, double *Y, const double *scale_dev, hipStream_t s);

// PCG driver (device-side per-column scalars; host polls every `chunk`
// iterations).  Solves S X = B for k columns from X (in/out) to tol.
// Halo tiling of a CSR pattern for the LDS-staged SpMM: row block b is
// rows [b*BR, min(N, (b+1)*BR)); its halo is the sorted set of columns its
// rows reference (halo_col[halo_ptr[b] .. halo_ptr[b+1])), and lcol[j] is
// the position of col[j] in its row block's halo.
struct Tiling {
  int BR = 0, nblk = 0, max_halo = 0, max_nnz = 0;  // max_nnz: most nonzeros in one block
  int max_pnz = 0;           // most padded local indices in one block
  int32_t *halo_ptr = nullptr, *halo_col = nullptr;
  int32_t *hself = nullptr;  // [nblk] position of the block's first row in its halo
  // local (halo) column indices, each row's run padded to a multiple of 8
  // entries with index max_halo (a halo row the kernel keeps at zero), so
  // that every run starts on a 16-byte boundary; pptr [nblk + 1]: start of
  // each block's runs
  uint16_t *lcol = nullptr;
  // the same runs as LDS byte offsets lcol[j] * lb_rowbytes, for halo rows
  // of lb_rowbytes bytes (present when max_halo * lb_rowbytes < 2^16)
  uint16_t *lbyte = nullptr;
  int lb_rowbytes = 0;
  int32_t *pptr = nullptr;
  // [N][2] per row slot of each block, rows with more nonzeros first (so
  // that the rows one wavefront walks together have similar lengths): word 0
  // bits 0-15 the row's first nonzero relative to the block's first, 16-23
  // its nonzero count, 24-31 its offset inside the block; word 1 the start of
  // its padded index run relative to the block's
  uint32_t *rmeta = nullptr;
};
// LDS bytes the tiled SpMM needs for k columns of elem-byte values (0 if the
// tiling cannot serve this shape).  The kernel reads the value and index
// arrays in whole 16-byte chunks: each must extend 16 bytes past its last
// entry.
size_t tiled_lds_bytes(const Tiling &t, int k, size_t elem);
// Y = S X (B null) or Y = B - S X through the halo tiles (FP64); -1 when the
// tiling cannot serve k columns (the caller uses launch_spmm)
int launch_spmm_tiled(int N, int k, const Tiling &t, int tb, const int32_t *rowptr, const double *val,
                      const double *X, double *Y, const double *B, hipStream_t s);
// FP32 values and vectors; tiled_fits_f32: whether the tiling serves k FP32 columns
int launch_spmm_tiled_f32(int N, int k, const Tiling &t, int tb, const int32_t *rowptr, const float *val,
                          const float *X, float *Y, const float *B, hipStream_t s);
bool tiled_fits_f32(int N, int k, const Tiling &t, int tb);
// the same over column chunks of width kc, X / Y / B with row pitches ldx / ldy
// (B: ldy); -1 (nothing launched) when the tiling cannot serve a chunk
int launch_spmm_tiled_cols(int N, int k, int ldx, int ldy, int kc, const Tiling &t, int tb, const int32_t *rowptr,
                           const double *val, const double *X, double *Y, const double *B, hipStream_t s);

struct PCGWork {
  void *R, *P, *Q;       // [N][k] of T
  void *P2;              // [N][k] of T: directions alternate between P and P2
  void *part;            // block partials, up to [nblk_max][3k] doubles
  void *state;           // device ColState[k] + control
  unsigned int *counter; // last-block counters
  int nblk_max;
  const Tiling *til;     // SpMM phase: LDS-staged halo tiles (nullptr = row kernel)
  int til_tb;            // threads per workgroup of the tiled kernel (256, 512, 1024)
  int last_iters = 0;    // iterations of the previous solve (first host poll)
  int prep_nblk = 0;     // partial rows written by launch_refine_prep
};
template <typename T>
int pcg_solve(int N, int k, const int32_t *rowptr, const int32_t *col, const T *val,
              const int32_t *ord, const T *diag, const T *B, T *X, double tol, int max_iter,
              PCGWork &w, int *iters_out, double *relres_out, int *converged_out,
              int *breakdown_out, hipStream_t s, int ng = 0, int x_zero = 0);
// x_zero: 1 = X is 0 on entry; 2 = R, P, X and the start partials were
// written by launch_refine_prep (B unused)
// FP32 correction-solve start of the mixed-precision refinement from the
// FP64 residual W [N][k] and column scales sc (device, [2k]: the scales,
// then per-column factors >= 1 on the solve's tolerance): R = float(W sc),
// P = D^{-1} R, X = 0 and the start partials, in w; then pcg_solve<float>
// with x_zero = 2
int launch_refine_prep(int N, int k, const double *W, const double *sc, const float *diag, float *X, PCGWork &w,
                       hipStream_t s);
// Y = B - S X through the halo tiles with per-workgroup column partials of
// the squared residual in part [returned count][k]; -1 when the tiling
// cannot serve k (nothing launched)
int launch_residual_tiled_norms(int N, int k, const Tiling &t, int tb, const int32_t *rowptr, const double *val,
                                const double *X, double *Y, const double *B, double *part, hipStream_t s);
size_t pcg_state_bytes(int k);
// autotuner check of the SpMM phase on the work buffers of w: mode 0 fills
// p with a fixed pattern, 1 copies q to ref ([N][k] of T), 2 returns
// max|q - ref| / max|ref| in *dev_host (NaN in q: infinite)
template <typename T>
int pcg_phase_check(PCGWork &w, int N, int k, int mode, void *ref, double *dev_host, hipStream_t s);
template <typename T>
int pcg_time_phase(int N, int k, int phase, const int32_t *rowptr, const int32_t *col, const T *val,
                   const int32_t *ord, const T *diag, T *X, PCGWork &w, int reps, float *ms,
                   hipStream_t s, int ng = 0);

// ------------------------------------------------------------------- dense
// C[a][b] = sum_i Z[i][a] Y[i][b] for a < ma, b < nb (tall-skinny, FP64
// MFMA), Z row stride ldz, Y row stride ldy, C row stride ldc.
void launch_gemm_tn(int N, int ma, int nb, const double *Z, int ldz, const double *Y, int ldy,
                    double *C, int ldc, double *work, size_t work_doubles, hipStream_t s);
// the same for a symmetric product (Y = H Z, H symmetric; m x m): only the
// 16x16 tiles on and above the diagonal are computed, the rest mirrored
void launch_gemm_tn_sym(int N, int m, const double *Z, int ldz, const double *Y, int ldy, double *C, int ldc,
                        double *work, hipStream_t s);
size_t gemm_tn_work_doubles(int N, int ma, int nb);
// Out[i][j] = sum_{c<4} Pw[i][c] T[Pidx[i][c]][j] (+ Y[i][j] if Y) ; T row stride ldt
void launch_ellP_times(int N, const int32_t *Pidx, const double *Pw, const double *T, int ldt,
                       int k, double alpha, const double *Y, int ldy, double *Out, int ldo,
                       hipStream_t s);
// Psi[i][j] = sum_c Pw Ut[Pidx][j] + sum_a Zt[i][a] Ut2[a][j]  (Zt: tail block of Z)
void launch_zu(int N, const int32_t *Pidx, const double *Pw, int n_H, const double *Z, int ldz,
               int kt, const double *U, int k, double *Psi, hipStream_t s);
// Out[i][j] (row stride ldo) = sum_{a < m} S[i][a] C[a][j], j < k (S row stride
// lds, C m x k row-major, m k doubles <= 64 KB; -1 otherwise)
int launch_tsmm(int N, int m, const double *S, int lds, const double *C, int k, double *Out, int ldo,
                hipStream_t s);
// Z = D^-1 R row by row (d: the diagonal), [N][k] row-major
void launch_row_div(int N, int k, const double *R, const double *d, double *Z, hipStream_t s);
// LOBPCG residual block: R = HX - MX diag(theta) (row stride ld), W = D^-1 R
// (row stride ldw), per-block column sums of R^2 and MX^2 in part[b][2k];
// returns the number of blocks (<= max_blocks), -1 if k > 256
int launch_lobpcg_resid(int N, int k, int ld, const double *HX, const double *MX, const double *theta,
                        const double *dinv, double *W, int ldw, double *part, int max_blocks, hipStream_t s);
// dinv = 1 / (a dK + b dM)
void launch_prec_diag(int N, double a, const double *dK, double b, const double *dM, double *dinv, hipStream_t s);
// Coarse blocks of the projection F = Z^T H Z with Z = [P | T] (P in ELL
// form): F[:n_H][:n_H] = P^T H P and F[:n_H][n_H:] = P^T Y (mirrored), Y = H T
// [N][k], from per-row-block partials (pp, pt; blocks of CP_ROWS rows, own and
// neighbour coarse index lists) gathered in a fixed order.  ldt, ldo >= the
// largest neighbour / own list; -1 when n_H > 256, k > kmax or the LDS does
// not fit.  Pidx / Pw rows are 16- / 32-byte aligned (4 entries per row).
constexpr int CP_ROWS = 64;
int launch_proj_coarse(int N, int n_H, int k, int kmax, int nblk, int ldt, int ldo, const int32_t *rowptr,
                       const int32_t *col,
                       const double *H, const int32_t *Pidx, const double *Pw, const double *Y, const int32_t *uoff,
                       const int32_t *ulist, const int32_t *noff, const int32_t *nlist, const int64_t *ppoff,
                       const int64_t *ptoff, double *pp, double *pt, const int32_t *gpp_ptr, const int64_t *gpp_idx,
                       const int32_t *gpt_ptr, const int64_t *gpt_idx, double *F, int m, hipStream_t s);
// C (m x n) = A (m x p) * B (p x n), small dense, row-major
void launch_small_gemm(int m, int n, int p, const double *A, int lda, const double *B, int ldb,
                       double *C, int ldc, double beta, hipStream_t s);
// Lowest k eigenpairs of (FA, FB), m <= 256: see ks_small_eig.
// out_theta[m], out_U[m][k], info[0] = rank, info[1] = sweeps
void launch_small_eig(int m, int k, const double *FA, int ldfa, const double *FB, int ldfb,
                      double *work, double *theta, double *U, int *info, hipStream_t s);
size_t small_eig_work_doubles(int m);
// Two-stage small eigensolver (m <= 190, packed symmetric matrices in LDS):
// launch_orth once per augmented space, launch_reduced_eig_split per F_A.
// work: jacobi_work_doubles(m) device doubles (the Jacobi rotation log).  The
// launchers return -1 if the large-LDS attribute cannot be set.
int packed_eig_supported(int m);
size_t orth_shared_bytes(int m);
size_t jacobi_work_doubles(int m);
int launch_orth(int m, const double *FB, int ldfb, double *D, double *V, double *X, double *work, int *info,
                hipStream_t s);
// the dense products run as multi-workgroup kernels; S (m x m), T1 (m x r),
// T2 (r x r), lam [r] are work buffers
int launch_reduced_eig_split(int m, int k, int r, const double *FA, int ldfa, const double *D, const double *X,
                             double *W, int warm, double *S, double *T1, double *T2, double *work, double *lam,
                             double *theta, double *U, int *info, hipStream_t s);
// Record msg as ks_last_error() of the calling thread; returns code.
int set_error(int code, const char *msg);
// Dense P (first n_H columns of Z) from the ELL form
void launch_dense_P(int N, const int32_t *Pidx, const double *Pw, int n_H, double *Z, int ldz,
                    hipStream_t s);
// copy [N][k] block into columns [c0, c0+k) of Z
void launch_copy_cols(int N, int k, const double *X, int ldx, double *Z, int ldz, int c0,
                      hipStream_t s);
void launch_zero_cols(int N, int c0, int c1, double *Z, int ldz, hipStream_t s);

}  // namespace ks

namespace ks {
// per-column sums of X .* Y (Y null: X .* X) over [N][k] rows, k <= 256:
// part[blk][k] with at most 512 blocks; returns the number of blocks
int launch_colsums(int N, int k, const double *X, const double *Y, double *part, hipStream_t s);
// per-column sums of squares (launch_colsums with Y null)
int launch_colnorms(int N, int k, const double *X, double *part, hipStream_t s);
// X[i][j] += scale[j] * (double)D[i][j]   (mixed-precision refinement update)
void launch_refine_update(int N, int k, const float *D, const double *scale, double *X, hipStream_t s);
// Anderson normal equations in one pass: with D_j = Fm - F_j (j < nh <= 4):
// out[0] = <Fm,Fm>, out[1+j] = <D_j, Fm>, out[5 + 4j + l] = <D_j, D_l>
// (block partials of 21 values: part[blk][21]); returns nblk
int launch_anderson_gram(int64_t npts, int n_q, const double *absdet, const double *w,
                         const double *Fm, int nh, const double *const *Fj, double *part,
                         hipStream_t s);
// F = A (m x m) assembled from blocks: PP [nH][nH] (ld nH), tail [m][kt] (ld kt)
void launch_fill_pencil(int m, int nH, const double *PP, const double *tail, double *F,
                        hipStream_t s);
// out = a + b  (n doubles)
void launch_add(int64_t n, const double *a, const double *b, double *out, hipStream_t s);
void launch_rows_to_storage(int N, int k, const double *src_api, double *dst, const int32_t *int2nat,
                            hipStream_t s);
void launch_rows_to_api(int N, int k, const double *src, double *dst_api, const int32_t *int2nat,
                        hipStream_t s);
}  // namespace ks

namespace ks {
// ------------------------------------------------------------------ adjoint
void launch_residual_cols(int N, int k, const double *Y1, const double *Y2, const double *Y3,
                          const double *theta, double *R, hipStream_t s);
void launch_right_mult(int N, int k, const double *X, const double *Mk, double *Out, hipStream_t s);
void launch_grad_q(const int32_t *edof, int n_loc, int n_e, int n_q, const double *phi,
                   const double *w, const double *absdet, const double *A, const double *B, int k,
                   const double *rho, double scale, double *g, hipStream_t s);
int force_blocks(int n_e);
void launch_force_partials(const double *coords, const int32_t *elems, int n_loc, int n_e, int n_q,
                           const double *bary, const double *g, int a0, int na, const double *Z,
                           const double *R, double *part, hipStream_t s);
int launch_coldots(int N, int k, const double *X, const double *Y, double *part, hipStream_t s);
// reverse mode through the truncated PCG
void launch_col_axpby(int N, int k, const double *a, const double *X, const double *b, double *Y, hipStream_t s);
void launch_zbar_back(int N, int k, const double *Zbar, const double *Z, const double *d, double *Rbar, double *dbar,
                      hipStream_t s);
void launch_pair_accum(const int32_t *edof, int n_loc, int n_e, int n_q, const double *phi, const double *w,
                       const double *absdet, const double *A, const double *B, int k, double scale, double *g,
                       hipStream_t s);

// ------------------------------------------- mesh-vertex derivative (pulay.hip)
// pairs of the element forms: n interior block pairs (u[p], v[p]) [N][ld]
// with per-column weights coef[p][i] = {wK, wM}; n_nodal pairs of nodal
// fields over all nodes with stiffness weight nw[p]
struct MeshGradPairs {
  int n = 0, n_nodal = 0;
  const double *u[4] = {}, *v[4] = {};
  int ldu[4] = {}, ldv[4] = {};
  const double *nu[3] = {}, *nv[3] = {};
  double nw[3] = {};
};
void launch_pair_q(const int32_t *edof, int n_loc, int n_e, int n_q, const double *phi, const double *A, int lda,
                   const double *B, int ldb, int k, double *out, hipStream_t s);
void launch_pulay_fields(int64_t n, const double *rho, const double *rho_l, const double *eps, const double *vxc_l,
                         const double *gam, const double *V0, const double *Vbc, const double *VHl, const double *W2,
                         double *F, double *G, hipStream_t s);
// per element [n_e][4 vertices][3]: scale * d/dX of the element forms
bool launch_mesh_grad(const double *coords, const int32_t *elems, const int32_t *edof, int n_loc, int n_e, int n_q,
                      const double *phi, const double *dphi, const double *w, const double *bary,
                      const MeshGradPairs &pr, const double *coef, int k, const double *F, const double *G,
                      int n_atoms, const double *Z, const double *R, double scale, double *out, hipStream_t s);
void launch_vertex_gather(int n_nodes, const int32_t *ptr, const int32_t *rec, const double *per_elem, double *out,
                          hipStream_t s);
int motion_blocks(int n);
void launch_motion_partials(int n_nodes, const double *Wm, int n_atoms, int a0, int na, const double *g, double *part,
                            hipStream_t s);
}  // namespace ks

namespace ks {
// ------------------------------------------------------------------ batch
size_t batch_sys_bytes();
size_t batch_part_stride();
int batch_resident_grid();
// dynamic LDS (bytes) the batched kernel can take with `grid` workgroups resident
int64_t batch_lds_budget(int grid);
// til: the system's halo tiling (nullptr: row products from the CSR arrays)
void pack_batch_sys(void *dst, const int32_t *rowptr, const int32_t *col, const double *val,
                    const double *diag, const double *B, double *X, double *R, double *P, double *Q,
                    double *part, unsigned int *bar, int N, int k, int ng, int team0, int team,
                    int max_iter, double tol, int *iters, double *relres,
                    unsigned long long *t_done, int *status, const Tiling *til);
void launch_batch_reset(void *systems, int n, unsigned long long *t0, hipStream_t s);
// lds: dynamic LDS bytes, at least max_halo * k * 8 of every tiled system
void launch_batch_pcg(int grid, const void *systems, const int *wg_sys, size_t lds, hipStream_t s);
}  // namespace ks

namespace ks {
// ------------------------------------------------------------ multigrid
struct Multigrid;
void kuhn_interp(const double *x, double L, int nH, int32_t *idx, double *w);
// An optional first coarse level given by the caller: nc unknowns at
// coordinates X [nc][3], reached from level 0 by the ELL-4 interpolation
// Pi/Pw [n0][4] (-1: no entry).  For P2 meshes this is P1 on the mesh's own
// vertices (nested, exact Galerkin operator: the P1 stiffness).
struct MGFirst {
  int nc = 0;
  std::vector<int32_t> Pi;
  std::vector<double> Pw, X;
};
Multigrid *mg_build(int n0, const int32_t *rp_d, const int32_t *ci_d, const double *val_d, const Tiling *til0,
                    int tb0,
                    const std::vector<int32_t> &rp_h, const std::vector<int32_t> &ci_h,
                    const std::vector<double> &val_h, const std::vector<double> &coords, double L, int n1,
                    hipStream_t s, const MGFirst *first = nullptr);
void mg_destroy(Multigrid *mg);
void mg_set_tiling(Multigrid *mg, const Tiling *til0, int tb0);
int mg_levels(const Multigrid *mg);
// part: >= 1024 doubles of device scratch; sc: >= 6 device doubles (CG scalars)
int mg_pcg(Multigrid *mg, const double *f, double *x, double tol, int max_it, double *part, double *sc,
           int *iters, double *relres, hipStream_t s);
}  // namespace ks
