/*
 * ks.h -- C ABI of the MI355X library for one step of the augmented subspace
 * method for the Kohn-Sham equation (Xu, Xie et al., "A Nonnested Augmented
 * Subspace Method for Kohn-Sham Equation", arXiv 2404.19249).
 *
 * Conventions
 *  - Pointers whose name ends in _host are host memory; every other array
 *    pointer is HIP device memory.  The caller owns all buffers it passes; the
 *    library owns the context and every workspace inside it.
 *  - Unknowns are numbered by the interior (non-Dirichlet) nodes in ascending
 *    node order: row i of an orbital block is the i-th node whose dirichlet
 *    flag is 0.  Orbital blocks are row-major [N][k] (node-major, the k
 *    right-hand sides contiguous), FP64.
 *  - Quadrature-point arrays are [n_elems][n_q], FP64.
 *  - All work is enqueued on the stream given to ks_create.  Entry points
 *    that return results in _host memory synchronise that stream before they
 *    return.
 *  - Every entry point returns a ks_status; negative values are errors (the
 *    outputs are then undefined) and ks_last_error() describes the last one on
 *    the calling thread.  Positive values are usable results with a warning.
 *  - A context is not thread safe; separate contexts on separate streams may
 *    be used concurrently.
 *  - Two environment variables print diagnostics and change no result:
 *    KS_DEBUG=1 synchronises after each stage and reports launch errors and
 *    buffer summaries on stderr; KS_TRACE_INNER=1 prints the residual of
 *    every inner (nonlinear) iteration of ks_scf_step.
 */
#ifndef KS_H
#define KS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ks_ctx ks_ctx;

typedef enum {
  KS_OK = 0,
  KS_NOT_CONVERGED = 1,     /* iteration limit reached; stats hold the residuals */
  KS_WARN_DEGENERATE = 2,   /* lambda_{k+1} - lambda_k < 1e-8: occupied set ambiguous */
  KS_ERR_ARG = -1,          /* invalid argument (null pointer, size out of range) */
  KS_ERR_HIP = -2,          /* a HIP runtime call failed */
  KS_ERR_NOMEM = -3,        /* device allocation failed */
  KS_ERR_MESH = -4,         /* element with det J <= 0, node id out of range */
  KS_ERR_BREAKDOWN = -5,    /* PCG breakdown: p^T S p <= 0 or NaN (operator not SPD) */
  KS_ERR_EIG = -6,          /* small eigensolver failed (no positive mass direction) */
  KS_ERR_STATE = -7         /* call order violated (e.g. project before a solve) */
} ks_status;

/* Mesh: a conforming tetrahedral decomposition of the box [-L, L]^3 with
 * Lagrange elements of order 1 (4 nodes) or 2 (10 nodes: v0..v3 then the
 * midpoints of edges 01, 02, 03, 12, 13, 23).  Elements must be positively
 * oriented (det J > 0).  The finite element space is the one of Sec. 2 of
 * the paper (linear elements; quadratic ones accepted as an extension). */
typedef struct {
  int32_t n_nodes, n_elems, order;
  const double *coords_host;       /* [n_nodes][3], Bohr */
  const int32_t *elems_host;       /* [n_elems][4 or 10] node ids */
  const uint8_t *dirichlet_host;   /* [n_nodes], 1 = on the boundary (psi = 0) */
  double L;                        /* half side of the box, for the coarse space */
} ks_mesh_desc;

/* Quadrature rule on the reference tetrahedron: barycentric points and
 * weights summing to 1/6.  Densities and potentials live at these points. */
typedef struct {
  int32_t n_q;                     /* <= 64 */
  const double *bary_host;         /* [n_q][4] */
  const double *w_host;            /* [n_q] */
} ks_quad_desc;

/* Nuclei (Sec. 2): charges Z_k and positions R_k, atomic units. */
typedef struct {
  int32_t n_atoms;
  const double *Z_host;            /* [n_atoms] */
  const double *R_host;            /* [n_atoms][3] */
} ks_atoms_desc;

enum { KS_XC_NONE = 0, KS_XC_X = 1, KS_XC_X_PZ81 = 2 };
enum { KS_HARTREE_OFF = 0, KS_HARTREE_MULTIPOLE = 1, KS_HARTREE_MULTIPOLE_LITERAL = 2 };
enum { KS_PREC_FP64 = 0, KS_PREC_MIXED = 1, KS_PREC_FP64_BLOCK_CG = 2 };

typedef struct {
  double mu;               /* shift of the BVPs; < 0 selects 8 M sum_k Z_k^2 (Sec. 4) */
  int32_t n_H;             /* coarse space: uniform Kuhn P1 mesh with n_H hexes per side */
  int32_t xc_mode;         /* KS_XC_*: LDA of Sec. 3.1 (Slater exchange + Perdew-Zunger) */
  int32_t hartree_mode;    /* KS_HARTREE_*: Poisson with multipole boundary data (eq. bd);
                              LITERAL drops the 1/2 of the quadrupole term */
  int32_t k_max;           /* largest number of orbitals used with this context (<= 64) */
  double tol_solve;        /* BVP relative residual (default 1e-8) */
  double tol_inner;        /* inner SCF: ||rho_out - rho_in||_0 (default 1e-8) */
  double tol_poisson;      /* Hartree Poisson relative residual (default 1e-10) */
  int32_t max_it_solve, max_it_inner, max_it_poisson;
  int32_t anderson_depth;  /* default 5 (Sec. 4) */
  double anderson_beta;    /* default 0.7 (Sec. 4) */
  double mixed_inner_tol;  /* FP32 inner PCG tolerance in the mixed form (default 1e-5) */
  int32_t deterministic;   /* 1: fixed-order reductions (always on in this version) */
} ks_options;

/* Fill *o with the defaults above. */
int ks_options_default(ks_options *o);

/* Replace the options of a live context (the next calls use them): the
 * tolerances, iteration limits, Anderson depth (at most the depth given at
 * ks_create) and beta, and the mixed form's inner tolerance.  mu, n_H,
 * xc_mode, hartree_mode and k_max fix the context's data and must equal the
 * values given at ks_create (KS_ERR_ARG otherwise; the context is then
 * unchanged). */
int ks_set_options(ks_ctx *ctx, const ks_options *o);

/* Per-mesh setup (not part of a step): interior numbering, CSR pattern,
 * element colouring, geometry, stiffness and mass matrices, the external
 * potential at the quadrature points (V_ext = -sum Z_k/|x - R_k|, Sec. 2),
 * A^L = 1/2 K + M[V_ext] (eq. st3), and the coarse interpolation I_H^h by
 * closed-form point location on the uniform coarse mesh (Algorithm 1 on a
 * structured coarse mesh).  Copies every host input; *out receives the
 * context.  Errors: KS_ERR_ARG, KS_ERR_MESH (inverted element or bad id),
 * KS_ERR_NOMEM, KS_ERR_HIP. */
int ks_create(const ks_mesh_desc *mesh, const ks_quad_desc *quad, const ks_atoms_desc *atoms,
              const ks_options *opt, hipStream_t stream, ks_ctx **out);

/* The same with the coarse space S_H on a given P1 tetrahedral mesh T_H that
 * need not be nested in the fine mesh (Sec. 3.2): I_H^h interpolates the
 * coarse P1 functions at the fine nodes by Algorithm 1 (nearest coarse
 * vertex from a bucket grid, then a barycentric walk to the containing
 * element).  coarse->dirichlet_host marks the coarse boundary vertices,
 * which carry no basis function; N_H = the number of the others (N_H + k_max
 * <= 256); opt->n_H is ignored.  Fine nodes outside T_H take the weights of
 * the last element of their walk, projected onto it.  coarse == NULL is
 * ks_create. */
int ks_create_nonnested(const ks_mesh_desc *mesh, const ks_mesh_desc *coarse, const ks_quad_desc *quad,
                        const ks_atoms_desc *atoms, const ks_options *opt, hipStream_t stream, ks_ctx **out);
int ks_destroy(ks_ctx *ctx);
const char *ks_last_error(void);

/* Sizes: out_host[0..10] = N (interior unknowns), n_nodes, n_elems, n_q,
 * N_H (coarse unknowns), nnz of the interior CSR pattern, n_loc, number of
 * element colours, leading dimension of the augmented basis Z, mu, levels
 * of the Hartree solver's multigrid hierarchy (0: Jacobi-PCG). */
int ks_get_sizes(const ks_ctx *ctx, double *out_host);

/* Assemble the Hamiltonian of the density of psi (Sec. 3.1 and 3.3):
 * rho = sum_i occ_i psi_i^2 at the quadrature points, Hartree potential by
 * the Poisson problem with multipole boundary data w_D(rho), LDA potential,
 * V_eff = V_ext + V_H + V_xc, and the BVP operator
 *     S = 1/2 K + M[V_eff] + mu M           (H-tilde of Sec. 3.3)
 * which later calls use.  psi [N][k] may be NULL (then V_eff = V_ext).
 * Optional device outputs (NULL to skip): rho_q, veff_q ([n_elems][n_q]),
 * vh_nodes ([n_nodes], all nodes).  energies_host (NULL to skip) receives
 * { <V_H, rho>/2, <rho, eps_xc>, <V_xc, rho>, <V_ext, rho>, Poisson iterations }. */
int ks_assemble(ks_ctx *ctx, const double *psi, int32_t k, const double *occ_host,
                double *rho_q, double *veff_q, double *vh_nodes, double *energies_host);

/* Copy an assembled operator's CSR arrays out (for inspection):
 * which = 0 S, 1 K (stiffness, interior), 2 M (mass), 3 A^L = 1/2 K + M[V_ext],
 * 4 M[V_nl] of the last inner iteration.  row_ptr [N+1], col [nnz], val [nnz]
 * are device buffers (any may be NULL). */
int ks_export_operator(ks_ctx *ctx, int32_t which, int32_t *row_ptr, int32_t *col, double *val);

typedef struct {
  int32_t iters[64];      /* PCG iterations per column (mixed: FP32 inner iterations summed) */
  int32_t refinements;    /* mixed form: FP64 residual evaluations */
  int32_t converged;      /* 1 if every column met the tolerance */
  double relres[64];      /* final ||b - S x|| / ||b|| per column (true residual, FP64) */
  double seconds;         /* device time of the solve (HIP events) */
} ks_solve_stats;

/* The N boundary value problems of Algorithm 3 (eq. Aux_Linear_Problem):
 *     S psi_hat_i = (lambda_i + mu) M psi_old_i,   i = 1..k,
 * with S from the last ks_assemble, one Jacobi-preconditioned CG recurrence
 * per column sharing every SpMM, started at psi_old, stopped per column at
 * ||b_i - S x_i||_2 <= tol_solve ||b_i||_2.  precision = KS_PREC_MIXED runs
 * FP32 PCG inside FP64 iterative refinement (FP64 residuals);
 * KS_PREC_FP64_BLOCK_CG runs O'Leary's block conjugate gradients in FP64
 * (one Krylov block for all k columns: X += P alpha, R -= S P alpha with
 * alpha = (P^T S P)^-1 (Z^T R), Z = D^-1 R, P = Z + P beta with
 * beta = (Z_old^T R_old)^-1 (Z^T R), the k x k systems by Cholesky on the
 * host), stopped when every column meets the tolerance; KS_ERR_BREAKDOWN
 * when P^T S P or Z^T R loses positive definiteness (the block lost rank).
 * psi_old, psi_hat: device [N][k]; lambda_host [k]; st_host may be NULL.
 * Returns KS_NOT_CONVERGED if max_it_solve was reached. */
int ks_block_solve(ks_ctx *ctx, const double *psi_old, const double *lambda_host, int32_t k,
                   int32_t precision, double *psi_hat, ks_solve_stats *st_host);

/* Generic form S X = B (B, X0, X device [N][k]; X0 may be NULL = zero). */
int ks_block_solve_rhs(ks_ctx *ctx, const double *B, const double *X0, int32_t k,
                       int32_t precision, double tol, double *X, ks_solve_stats *st_host);

/* Reverse mode through the truncated FP64 block solve (the derivative of
 * what the solver returns, not of the exact S^-1 B; the paper has no
 * derivatives).  Runs S X = B from X0 (NULL = zero) by per-column
 * Jacobi-PCG, D = diag S, each column stopped at ||b - S x|| <= tol ||b||
 * or after max_it iterations (tol = 0: exactly max_it), then for
 * L = sum_ij Xbar_ij X_ij sweeps the recurrence backwards:
 *   g_q = dL/dV_q, V the quadrature potential of S = 1/2 K + M[V] + mu M
 *         (dS_ab/dV_q = w_q |J| phi_a phi_b), the preconditioner's
 *         dependence on diag S included; device [n_e][n_q];
 *   Bbar = dL/dB, device [N][k].
 * The forward keeps the per-column scalars of every iteration on the host and
 * the residual and direction blocks every `seg` iterations (0: 8) on the
 * device; the reverse sweep recomputes each segment from its checkpoint
 * (bit-identical kernels and coefficients).  Device memory: about
 * (13 + 2 (seg + 1) + 2 K / seg) blocks of N x k doubles, allocated and freed
 * by the call.  B, X0, Xbar, X: device [N][k] (API order); iters_host [k]
 * (may be NULL) receives the per-column iteration counts.  Requires a prior
 * ks_assemble. */
int ks_block_solve_vjp(ks_ctx *ctx, const double *B, const double *X0, int32_t k, double tol, int32_t max_it,
                       int32_t seg, const double *Xbar, double *X, double *g_q, double *Bbar, int32_t *iters_host);

/* Galerkin projection onto the augmented space (eqs. st1-st7):
 * Z = [I_H^h | psi_tilde] with psi_tilde = psi_hat M-orthogonalised against
 * span(I_H^h) (same span); F = Z^T H Z for H = M (which = 0), A^L (1) or the
 * nonlinear part M[V_H + V_xc] of the last assembly (2).  F is device
 * [m][m], m = N_H + k, row-major.  Also stores Z in the context for
 * ks_scf_step-style use.  FP64 with FP64 MFMA accumulation. */
int ks_augmented_project(ks_ctx *ctx, const double *psi_hat, int32_t k, int32_t which, double *F);

/* Lowest k eigenpairs of the pencil (F_A, F_B) (eq. st1), both device
 * [m][m]: diagonal scaling, canonical orthogonalisation of F_B (directions
 * below 1e-12 of the largest eigenvalue dropped), symmetric Jacobi
 * eigensolve.  U device [m][k]; lambda_host [k]; rank_host may be NULL. */
int ks_small_eig(ks_ctx *ctx, const double *FA, const double *FB, int32_t m, int32_t k,
                 double *U, double *lambda_host, int32_t *rank_host);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * eigensolve as ks_small_eig without a context.  FA, FB device [m][m]
 * row-major (ld m), U device [m][k], lambda_host [k], rank_host may be NULL;
 * work is enqueued on `stream`, which is synchronised twice (the rank of F_B
 * sizes the second stage) before the call returns.  Every work buffer lives
 * in one fixed 19 MiB device array per GPU, held until the process ends:
 * the call itself allocates nothing.  Limits: 1 <= k <= m <= 190
 * (KS_ERR_ARG beyond).  Calls that overlap on one GPU (several host
 * threads, or several streams before the first returns) share that array
 * and race; results are undefined then. */
int ks_small_eig_noalloc(const double *FA, const double *FB, int32_t m, int32_t k, double *U,
                         double *lambda_host, int32_t *rank_host, hipStream_t stream);

/* Initial guess: Ritz pairs of (1/2 K + M[V_ext], M) in span(I_H^h).
 * psi device [N][k], lambda_host [k]. */
int ks_initial_guess(ks_ctx *ctx, int32_t k, double *psi, double *lambda_host);

typedef struct {
  double E_total;        /* sum f lambda - <V_H/2 + V_xc, rho_in> + <rho_in, eps_xc> + E_nn */
  double E_band, E_H, E_xc, E_vxc, E_nn;
  double res_inner;      /* final ||rho_out - rho_in||_0 */
  int32_t inner_iters;   /* nonlinear iterations in the augmented space */
  int32_t poisson_iters; /* PCG iterations of all Hartree solves in the step */
  int32_t rank;          /* numerical rank of F_B */
  int32_t status_solve;
  ks_solve_stats solve;
  double seconds[8];     /* assemble, block solve, project, inner SCF, energies, total */
  double res_outer;      /* ||rho^{l+1} - rho^l||_0: the step's output density against its input */
} ks_step_report;

/* One iteration of Algorithm 3: assemble S from the density of psi, solve
 * the BVPs, project onto the augmented space, solve the small nonlinear
 * Kohn-Sham problem there by the Anderson-mixed inner iteration of Sec. 4
 * (Hartree boundary data w_D frozen at the step's input density), and write
 * the new orbitals and eigenvalues back in place.
 * psi: device [N][k] in/out; lambda_host [k] in/out; occ_host [k];
 * rho_q (device [n_elems][n_q], may be NULL) receives the new density.
 * Returns KS_NOT_CONVERGED when the inner iteration stops at max_it_inner
 * with ||rho_out - rho_in||_0 >= tol_inner (rep_host->res_inner) or the BVP
 * solve at max_it_solve; the outputs are then those of the last inner pass,
 * and its energies use the input density that built that pass's potentials. */
int ks_scf_step(ks_ctx *ctx, double *psi, double *lambda_host, int32_t k, const double *occ_host,
                int32_t precision, double *rho_q, ks_step_report *rep_host);

/* Algorithm 3 to convergence: ks_scf_step repeated (in place on psi,
 * lambda_host) until ||rho^{l+1} - rho^l||_0 < tol_outer (the quadrature L2
 * norm of the density change; Alg. 3's stopping rule) or max_steps steps,
 * then ks_step_energy for E_KS of the last step.  Returns KS_NOT_CONVERGED
 * if max_steps was reached, KS_WARN_DEGENERATE as ks_scf_step; rep_host may
 * be NULL. */
typedef struct {
  int32_t steps, converged;
  int32_t inner_iters, poisson_iters;  /* totals over the steps */
  double res_outer;                    /* of the last step */
  double E_total, E_KS;                /* of the last step; equal at outer convergence */
  double seconds;
} ks_run_report;
int ks_scf_run(ks_ctx *ctx, double *psi, double *lambda_host, int32_t k, const double *occ_host,
               int32_t precision, double tol_outer, int32_t max_steps, double *rho_q, ks_run_report *rep_host);

/* Algorithm 1 (Sec. 3.2) between two meshes, as Algorithm 2 uses it to
 * carry the orbitals to the next mesh: every interior node of this context's
 * mesh is located in the P1 tetrahedral mesh src (nearest vertex from a
 * bucket grid, then a barycentric walk; a node outside src takes the
 * weights of the last element of its walk, projected onto it) and the
 * orbitals, P1 on src and zero on its Dirichlet nodes, are interpolated
 * there.  psi_src: device [N_src][k], rows = src's non-Dirichlet nodes in
 * ascending order (the orbital layout of a context on src); psi: device
 * [N][k] on this context.  The search index (face neighbours, bucket grid)
 * is built on the host; the location runs on the GPU, one thread per node;
 * a few device buffers are allocated for the call.  orthonormalize != 0: the
 * interpolated columns are then made M-orthonormal on this mesh in column
 * order (Cholesky of Psi^T M Psi), as an SCF started from them expects;
 * KS_ERR_EIG if they are linearly dependent.  KS_ERR_ARG for a P2 source or
 * k outside 1..k_max. */
int ks_interpolate(ks_ctx *ctx, const ks_mesh_desc *src, const double *psi_src, int32_t k, int32_t orthonormalize,
                   double *psi);

/* ---- Mesh moving for Algorithm 2 (Sec. 3.2) --------------------------
 * Three mesh-level calls (no context): the Hessian metric of the adaptive
 * function sqrt(rho) (eqs. m1, m2), a metric spring node mover standing in
 * for the remesher (Mshmet/Mmg3d in the paper), and P1 field interpolation
 * between meshes (Algorithm 1).  Meshes are P1 (order 1; KS_ERR_ARG
 * otherwise), given by host arrays as for ks_create; every call copies what
 * it needs to the device, allocates its work buffers and frees them before
 * returning, and is synchronous on `stream`. */
typedef struct {
  double eps;    /* epsilon of eq. m2 (L-infinity interpolation error target) */
  double h_min;  /* shortest edge scale: eigenvalues capped at 1 / h_min^2 */
  double h_max;  /* longest edge scale: eigenvalues raised to 1 / h_max^2 */
} ks_metric_params;

/* Eqs. m1-m2 at every node: u = sqrt(sum_i f_i psi_i^2) (zero on Dirichlet
 * nodes); its gradient recovered as the volume-weighted average of the
 * element gradients of its P1 interpolant around each node (the
 * lumped-mass L2 projection), the same recovery applied to each component
 * of that gradient, H the symmetric part; H = R Lambda R^T (Jacobi
 * rotations), lambda~_i = min(max(C_d |lambda_i| / eps, 1 / h_max^2),
 * 1 / h_min^2), C_d = 9/32, M = R Lambda~ R^T.  psi: device [N][k] over the
 * non-Dirichlet nodes in ascending order (a context's orbital layout on
 * this mesh); occ_host [k]; metric: device [n_nodes][6] = (xx, yy, zz, xy,
 * xz, yz) of M, output. */
int ks_mesh_metric(const ks_mesh_desc *mesh, const double *psi, int32_t k, const double *occ_host,
                   const ks_metric_params *prm, double *metric, hipStream_t stream);

/* Node mover: `sweeps` damped Jacobi sweeps on the spring energy
 * sum over edges (a, b) of (x_b - x_a)^T (M_a + M_b)/2 (x_b - x_a) with the
 * metric carried by the nodes: every non-Dirichlet node moves to
 * (1 - w) x_a + w t_a, t_a the minimiser over x_a with the other nodes
 * fixed; Dirichlet nodes stay.  A sweep that would leave an element with
 * det J <= 0 is redone with w halved (at most 20 times; then KS_ERR_MESH).
 * metric: device [n_nodes][6] as from ks_mesh_metric; 0 < omega < 2;
 * coords_out_host [n_nodes][3] receives the moved nodes; halvings_host
 * (may be NULL) the number of halvings over all sweeps. */
int ks_move_nodes(const ks_mesh_desc *mesh, const double *metric, double omega, int32_t sweeps,
                  double *coords_out_host, int32_t *halvings_host, hipStream_t stream);

/* Algorithm 1 for a nodal field: the P1 interpolant on src of field
 * (device [src n_nodes][m], every node including Dirichlet ones) evaluated
 * at n_pts points (pts_host [n_pts][3]; located on the GPU as in
 * ks_interpolate); out: device [n_pts][m]. */
int ks_interpolate_field(const ks_mesh_desc *src, const double *field, int32_t m, int32_t n_pts,
                         const double *pts_host, double *out, hipStream_t stream);

/* The "direct" method that Sec. 4 compares Algorithm 3 with: the
 * self-consistent field iteration on the whole fine space.  Every pass
 * builds H(rho_in) = 1/2 K + M[V_ext + V_H(rho_in) + V_xc(rho_in)] (Sec. 3.1;
 * the multipole boundary data w_D of eq. bd recomputed from rho_in), takes
 * the lowest k eigenpairs of (H, M) by block LOBPCG (Jacobi preconditioner
 * of 1/2 K + tau M, warm-started from the previous pass, to a relative
 * residual ||H x - lambda M x|| / ||M x|| of max(tol_eig, min(1e-3,
 * 0.1 x the last density residual))), and mixes the density by the Anderson
 * scheme of Sec. 4 (the context's depth and beta), until ||rho_out -
 * rho_in||_0 < tol with the last eigensolve at tol_eig, or max_scf passes.
 * psi: device [N][k] in (the start orbitals) / out; lambda_host [k] in
 * (used for the first preconditioner shift) / out; occ_host [k]; rho_q
 * (device [n_elems][n_q], may be NULL) receives the last output density.
 * The energy is that of Sec. 3.1 on the density that built the final H.
 * Requires k <= min(k_max, 48).  Allocates its LOBPCG work space (about
 * 11 N k_max doubles and one operator) on the first call.  Returns
 * KS_NOT_CONVERGED at max_scf. */
typedef struct {
  int32_t scf_iters, eig_iters, poisson_iters, converged;
  double res;                          /* final ||rho_out - rho_in||_0 */
  double eig_res;                      /* largest relative eigen-residual of the last pass */
  double E_total, E_band, E_H, E_xc, E_vxc, E_nn;
  double seconds;
} ks_direct_report;
int ks_direct_scf(ks_ctx *ctx, double *psi, double *lambda_host, int32_t k, const double *occ_host,
                  double tol, int32_t max_scf, double tol_eig, int32_t max_eig, double *rho_q,
                  ks_direct_report *rep_host);

/* Replace the external potential: either its values at the quadrature
 * points (device [n_elems][n_q]) or new nuclear positions R_host [n_atoms][3]
 * (then V_ext = -sum Z_k/|x - R_k| and E_nn are recomputed).  Recomputes
 * A^L = 1/2 K + M[V_ext] and its coarse block; a following ks_assemble is
 * needed before solves. */
int ks_set_external(ks_ctx *ctx, const double *vext_q, const double *R_host);

/* Kohn-Sham energy (functional form of Sec. 2) of the orbitals produced by
 * the most recent ks_scf_step, with the Hartree boundary data of that step
 * held fixed: out_host[0..5] = {E_KS, kinetic, <V_ext, rho>, E_H^step,
 * <rho, eps_xc>, E_nn}, E_H^step = 1/2 <rho, V_H[rho]> + 1/2 <rho - rho^l, V_bc>
 * (V_bc: harmonic lift of the boundary data).  Two Poisson solves. */
int ks_step_energy(ks_ctx *ctx, double *out_host);

/* Adjoint of the most recent ks_scf_step (its inputs held fixed):
 * g_q = dE * dE_KS/dV_ext at the quadrature points (device [n_elems][n_q])
 * and forces_host = -dE * dE_KS/dR_k ([n_atoms][3], may be NULL).  Uses the
 * stationarity of the converged inner iteration: g_q = dE w_q |J| (rho_q -
 * sum_i Y_i(x_q) psi_hat_i(x_q)) with one adjoint block solve S Y =
 * psi_bar_hat (CG recomputed from zero, nothing stored from the forward
 * solve).  st_host (may be NULL) receives the adjoint solve statistics.
 * KS_ERR_STATE when there is no step, or when its inner iteration stopped at
 * max_it_inner above tol_inner (no stationary point to differentiate). */
int ks_step_backward(ks_ctx *ctx, double dE, double *g_q, double *forces_host,
                     ks_solve_stats *st_host);

/* The same gradient with the BVP part taken by reverse mode through the
 * truncated solve (ks_block_solve_vjp) instead of the implicit adjoint: the
 * step's BVPs are solved again from psi_old by the FP64 per-column PCG
 * (tol_solve, max_it_solve) and the seed psi_bar_hat is swept back through
 * that recurrence (checkpoint segment seg, 0: 8), so g_q is the derivative
 * of the step as truncated rather than of its exact limit; the two agree to
 * about the solve tolerance.  Needs the last ks_scf_step in KS_PREC_FP64
 * (KS_ERR_STATE otherwise); st_host (may be NULL) receives the iteration
 * counts. */
int ks_step_backward_truncated(ks_ctx *ctx, double dE, int32_t seg, double *g_q, double *forces_host,
                               ks_solve_stats *st_host);

/* Mesh-motion (Pulay) terms: the derivative of the most recent ks_scf_step's
 * E_KS with respect to the vertex coordinates of the fine mesh, and nuclear
 * forces for a mesh whose nodes follow the nuclei (the node moves of
 * Algorithm 2, Sec. 3.2, made differentiable).  The step's inputs are held
 * fixed: the nodal coefficients of psi^l, lambda^l, rho^l at the quadrature
 * points, the Hartree boundary data w_B and the matrix of I_H^h (the coarse
 * space moves with the mesh).  Besides the adjoint block solve of
 * ks_step_backward it takes five Poisson solves (V_H of rho^l and of rho
 * with and without w_B, two adjoint loads) and one element pass of the
 * closed-form shape derivatives of the stiffness, mass and potential forms.
 *   dEdX    device [n_nodes][3] (natural node order), dE * dE_KS/dX_n; zero
 *           at P2 edge nodes (the geometry is the vertices'); may be NULL
 *           when motion is given
 *   motion  device [n_nodes][n_atoms] or NULL: node n moves by
 *           motion[n][a] dR_a when nucleus a moves by dR_a; then forces_host
 *           = F (fixed mesh, as ks_step_backward) - sum_n motion[n][a] dEdX_n
 *   g_q     device [n_elems][n_q] or NULL; forces_host [n_atoms][3], needed
 *           with motion
 * KS_ERR_STATE as ks_step_backward, and when V_ext was given as a field
 * (ks_set_external with vext_q: its gradient in x is unknown). */
int ks_step_backward_mesh(ks_ctx *ctx, double dE, const double *motion, double *dEdX, double *g_q,
                          double *forces_host, ks_solve_stats *st_host);

/* ---- Batched form: many independent systems in one persistent launch ----
 * Each system is a context with an assembled operator (ks_assemble); the
 * batch solves S_s X_s = M_s psi_s diag(lambda_s + mu_s) for every s
 * (eq. Aux_Linear_Problem per system) in ONE persistent kernel launch,
 * captured once in a hipGraph and replayed by every ks_batch_block_solve.
 * Workgroups form per-system teams proportional to nnz_s k_s (grid = the
 * resident workgroup count, or grid_req if smaller); the lanes-per-row split
 * of each system comes from its context's autotuned choice (ks_autotune) or
 * a rule by k.  A system's products S_s P_s run through one of its
 * context's halo tilings (row blocks staged in LDS) when that tiling's halo
 * image (largest halo x k_s doubles) fits the LDS the launch can take at its
 * grid; the largest such row block is the default, else row products from
 * the CSR arrays.  Systems must outlive the batch and keep their
 * operators. */
typedef struct ks_batch ks_batch;
typedef struct {
  double seconds;               /* whole launch (HIP events) */
  int32_t n;
  double system_seconds[256];   /* device-clock completion time of each system, from launch start */
  int32_t iters[256];           /* max PCG iterations over the columns */
  double relres[256];           /* max recursive relative residual */
  int32_t status[256];          /* 0 converged, 1 iteration limit */
} ks_batch_stats;
int ks_batch_create(int32_t n, ks_ctx *const *systems, const int32_t *k_host, int32_t grid_req,
                    ks_batch **out);
/* grid_host: workgroups of the launch; team_host/ng_host/tile_host [n] (each
 * may be NULL): team size, lanes per row, and rows per halo-tile block of
 * each system's products (0: row products) */
int ks_batch_info(const ks_batch *b, int32_t *grid_host, int32_t *team_host, int32_t *ng_host,
                  int32_t *tile_host);
/* Sets the layout by hand: ng_host [n] lanes per row (1, 2, 4 or 8, with
 * lanes x k_s <= 64) and tile_host [n] rows per halo-tile block (0: row
 * products; else 32, 64, 85, 128, 170 or 256, a tiling the system's context
 * holds whose halo image fits the launch's LDS); either may be NULL to keep
 * the current choice.  KS_ERR_ARG, with nothing changed, for a value that
 * is not available.  Team sizes and the grid are kept. */
int ks_batch_set_layout(ks_batch *b, const int32_t *ng_host, const int32_t *tile_host);
/* psi_old[s], psi_hat[s]: device [N_s][k_s]; lambda_host[s]: host [k_s].
 * Host arrays of pointers. */
int ks_batch_block_solve(ks_batch *b, const double *const *psi_old,
                         const double *const *lambda_host, double *const *psi_hat,
                         ks_batch_stats *st_host);
/* Autotuner of the batch layout on these inputs (same arguments as the
 * solve; outputs discarded).  For each candidate grid (the resident
 * workgroup count, 3/4, 1/2 and 1/4 of it): lanes per row and product form
 * (row products, or halo tiles of 32, 64, 128 or 256 rows where they fit)
 * per system from one run at each candidate, then `rounds` feedback rounds
 * that resize the teams so that measured completion times equalise.  Keeps the fastest
 * layout (and re-captures the graph for its grid); best_ms (host, may be
 * NULL) receives its launch time. */
int ks_batch_autotune(ks_batch *b, const double *const *psi_old, const double *const *lambda_host,
                      int32_t rounds, double *best_ms);
int ks_batch_destroy(ks_batch *b);

/* Measurement: mean duration (ms, HIP events on the context stream) of
 * `reps` back-to-back launches of one hot-path operation on the current
 * state.  which = 0 SpMM phase q = S p with the p.q reduction (FP64, k
 * columns, the kernel the solver uses), 1 residual update, 2 x/p update;
 * 3..5 the same phases in FP32 (mixed form); 6 the Hartree Poisson SpMM phase
 * (k = 1); 7 potential-matrix assembly M[V] over all colours; 8 density at the
 * quadrature points from the k orbitals of the last ks_assemble; 9 LDA
 * energy density and potential at the quadrature points; 10 projection
 * F = Z^T M[V] Z over the augmented basis of the last step (m = N_H + k) as
 * the inner iteration computes it (coarse blocks from the ELL form of I_H^h,
 * T^T M[V] T on the FP64 matrix cores); 11 that T^T (M[V] T) GEMM alone;
 * 12 the dense projection over all m columns of Z (SpMM + FP64 MFMA GEMM).
 * 7..12 overwrite work buffers (a following ks_step_backward needs a new
 * ks_scf_step).  Requires a prior ks_assemble (10..12: a prior ks_scf_step
 * or ks_augmented_project). */
int ks_time_kernel(ks_ctx *ctx, int32_t which, int32_t k, int32_t reps, double *ms_host);

/* HBM streaming probe: the bandwidth of plain coalesced streams (16-byte
 * vectors, 4 in flight per thread, grid of 16 workgroups per CU) over
 * buffers of `bytes` bytes each, as the practical ceiling next to the
 * nominal 8 TB/s for the memory-bound kernels.  kind 0: read one buffer
 * (per-workgroup sums), 1: copy, 2: triad c = a + s b; nontemporal != 0
 * uses nontemporal loads and stores.  *gbs_host = (streams x bytes x reps) /
 * time, timed with HIP events on `stream` after one warm-up pass.  The
 * buffers are allocated and freed by the call (1 MiB <= bytes <= 64 GiB). */
int ks_stream_probe(int64_t bytes, int32_t kind, int32_t nontemporal, int32_t reps, double *gbs_host,
                    hipStream_t stream);

/* Autotuner of the SpMM phase: on the current operator S (and the Poisson
 * operator K), times the SpMM phase of the block PCG for every kernel
 * candidate -- the row kernel with a row's nonzeros split over NG = 1, 2, 4,
 * 8 lanes, and the LDS-staged halo-tile kernel with row blocks of 32, 64,
 * 85, 128, 170, 256 rows and 256-, 512- or 1024-thread workgroups -- in FP64
 * and FP32 with k columns (Poisson: k = 1), and keeps the fastest for later
 * solves of this context.  report_host (NULL to skip) receives 75 doubles:
 * {NG fp64, NG fp32, NG Poisson, tile rows fp64, fp32, Poisson (0 = row
 * kernel chosen), tile threads fp64, fp32, Poisson, then row-kernel
 * ms[fp64|fp32|Poisson][NG], then tile-kernel ms[fp64|fp32|Poisson][rows]
 * [256|512|1024 threads] (-1: not available for this shape, -2: rejected,
 * and row-kernel entries -2: rejected)}.  Every
 * candidate's q = S p on a fixed p is compared with the first row kernel's;
 * one that differs by more than 1e-12 (FP64) or 1e-5 (FP32) of max|q| is
 * rejected.  Requires a prior ks_assemble. */
int ks_autotune(ks_ctx *ctx, int32_t k, int32_t reps, double *report_host);

/* ks_autotune behind a cache file (a text file at `path`, host string).  Key:
 * the device's architecture name, the element order, floor(log2 N), the
 * rounded nonzeros per row of S, k, and the solver precision (fp64, fp32;
 * poisson with k = 1).  Value: lanes per row, tile rows, tile threads (0 0:
 * row kernel) and the time measured when the entry was written.  If the file
 * holds entries for all three solvers under this key (the last matching
 * line wins, lines that do not parse are skipped), each is checked as
 * ks_autotune checks a candidate (the tiling exists, fits for this k and its
 * q = S p agrees with the row kernel's) and applied: *hit_host = 1, nothing
 * is timed.  Otherwise (missing file included) ks_autotune(ctx, k, reps)
 * runs and its three choices are appended to the file in one write:
 * *hit_host = 0.  hit_host may be NULL.  Errors: those of ks_autotune;
 * KS_ERR_ARG for a NULL or empty path, or when the file cannot be appended to
 * (the tuned choice is applied all the same).  Processes that share a file
 * append whole entries; a file is never rewritten or truncated. */
int ks_autotune_cached(ks_ctx *ctx, int32_t k, int32_t reps, const char *path, int32_t *hit_host);

/* SpMM-phase kernels in use: out_host[0..8] = {NG fp64, NG fp32, NG Poisson
 * (row kernel lanes per row), tile rows fp64, fp32, Poisson (0 = row
 * kernel), tile workgroup threads fp64, fp32, Poisson}.  The tiled kernel is used only where its
 * LDS image fits for the solve's k. */
int ks_spmm_config(const ks_ctx *ctx, int32_t *out_host);

/* Diagnostics: copy n doubles of an internal buffer (by name: "GPP",
 * "FAL_PP", "Z", "Y", "FB", "FAL", "FA", "U", "rho_in", "vh_q", "wB", "mom",
 * "S": the interior operator values in storage order) into the device buffer
 * dst.  "S32" copies the mixed form's FP32 operator copy (nnz floats, packed
 * into the first ceil(nnz / 2) doubles of dst; KS_ERR_STATE when there is
 * none).  For tests and debugging only. */
int ks_debug_buffer(ks_ctx *ctx, const char *name, double *dst, int64_t n);

#ifdef __cplusplus
}
#endif
#endif /* KS_H */
