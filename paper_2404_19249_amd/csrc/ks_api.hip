// Host runtime and C ABI of the KS library: per-mesh setup (interior
// numbering, CSR pattern, element colouring, element->CSR slot map, coarse
// interpolation) and the entry points of one augmented-subspace step
// (Algorithm 3 of the paper), which enqueue the device kernels on the
// context's stream.
#include "../../include/ks.h"
#include "common.h"
#include "kernels.h"

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

using namespace ks;

static thread_local std::string g_err;
static int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}
// the same error channel for entry points defined in other source files
int ks::set_error(int code, const char *msg) { return fail(code, msg); }
#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      return fail(KS_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));        \
  } while (0)

namespace {

// simple parallel-for over [0, n) on the host (setup only)
template <typename F>
void parallel_for(int64_t n, F f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 4096 || nt == 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([=, &f]() {
      for (int64_t i = a; i < b; ++i) f(i);
    });
  }
  for (auto &x : th) x.join();
}

struct DevBuf {
  std::vector<void *> ptrs;
  ~DevBuf() {
    for (void *p : ptrs) (void)hipFree(p);
  }
};

bool debug_on() {
  static int v = -1;
  if (v < 0) {
    const char *e = std::getenv("KS_DEBUG");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v == 1;
}

}  // namespace

struct ks_ctx;
// KS_DEBUG=1: synchronise after a stage, report launch errors and summarise a buffer
static void dbg(ks_ctx *c, const char *what, const double *buf, int64_t n);

struct ks_ctx {
  hipStream_t s = nullptr;
  ks_options opt;
  int order = 1, n_loc = 4, n_nodes = 0, n_e = 0, n_q = 0, N = 0, NB = 0, N_H = 0, n_H = 0;
  int k_max = 0, mp = 0;  // leading dimension of Z
  // halo tiles of the many-column products (projection): row block, column
  // chunk, threads
  int proj_br = 128, proj_kc = 16, proj_tb = 1024;
  double L = 0.0, mu = 0.0;
  int n_atoms = 0;
  std::vector<double> hZ, hR;
  double E_nn = 0.0;
  int64_t nnz = 0, nnzB = 0, nnz_ext = 0;
  int n_colours = 0;
  std::vector<int> colour_off;

  DevBuf mem;
  // mesh / tables
  double *coords = nullptr;
  int32_t *elems = nullptr, *edof = nullptr, *slot = nullptr, *node2int = nullptr,
          *node2bnd = nullptr, *bnodes = nullptr, *elem_perm = nullptr;
  // coarse blocks of the inner iteration's projection (launch_proj_coarse):
  // per CP_ROWS-row block its own / neighbour coarse index lists, partial
  // offsets, and per output the partials that sum into it (cp_ok = 0: the
  // dense projection is used)
  int cp_ok = 0, cp_nblk = 0, cp_ldt = 0, cp_ldo = 0;
  int32_t *cp_uoff = nullptr, *cp_ulist = nullptr, *cp_noff = nullptr, *cp_nlist = nullptr,
          *cp_gpp_ptr = nullptr, *cp_gpt_ptr = nullptr;
  int64_t *cp_ppoff = nullptr, *cp_ptoff = nullptr, *cp_gpp_idx = nullptr, *cp_gpt_idx = nullptr;
  double *cp_pp = nullptr, *cp_pt = nullptr;
  // direct SCF (ks_direct_scf): LOBPCG blocks S = [X | W | P], H S, M S
  // ([N][3 k_d], row-major), two [N][k_d] temporaries, the operator H, the
  // Jacobi preconditioner, Gram matrices and the Ritz coefficients
  int d_k = 0;
  double *dS = nullptr, *dHS = nullptr, *dMS = nullptr, *dT1 = nullptr, *dT2 = nullptr, *dH = nullptr,
         *dDinv = nullptr, *dDM = nullptr, *dGH = nullptr, *dGM = nullptr, *dC = nullptr, *dTheta = nullptr;
  // row form of the potential-matrix assembly: per storage row its incidence
  // records (element, local node, column offsets; IncRec) from r_incptr,
  // each row block's visiting order r_perm, and its LDS size (0: the
  // colour-scatter path is used instead)
  int32_t *r_incptr = nullptr;
  uint8_t *r_inc = nullptr, *r_perm = nullptr;
  size_t r_lds = 0;
  double *load_e = nullptr;  // per-element load values [n_e][n_loc] (row-form load vector)
  double *phib = nullptr;  // basis values b-major [n_loc][n_q] (row-form assembly)
  double *absdet = nullptr, *gl = nullptr, *phi = nullptr, *dphi = nullptr, *pairtab = nullptr,
         *qw = nullptr, *qbary = nullptr, *dZ = nullptr, *dR = nullptr;
  // CSR (interior rows; columns [0,nnz) interior, extension [nnz, nnz_ext) = K_IB part)
  int32_t *rowptr = nullptr, *col = nullptr, *rowptrB = nullptr, *colB = nullptr;
  int32_t *rorder = nullptr;    // active row schedule of the SpMM kernels (nullptr = storage order)
  int32_t *rorder_m = nullptr;  // Morton schedule of the rows
  int32_t *int2nat = nullptr;   // natural (API) index of each stored unknown
  std::vector<int32_t> h_int2nat;
  int ng64 = 0, ng32 = 0, ngP = 0;  // lanes per row in the SpMM phase (0 = default)
  double *K = nullptr, *M = nullptr, *AL = nullptr, *base = nullptr, *S = nullptr,
         *MNL = nullptr, *diagS = nullptr, *diagK = nullptr;
  float *S32 = nullptr, *diagS32 = nullptr;
  bool have_S = false, have_S32 = false;
  // quadrature fields [n_e][n_q]
  double *vext_q = nullptr, *rho_l = nullptr, *rho_in = nullptr, *rho_out = nullptr,
         *vh_q = nullptr, *vxc_q = nullptr, *exc_q = nullptr, *vnl_q = nullptr, *drho = nullptr;
  double *hist_in[5] = {}, *hist_F[5] = {};
  int hist_alloc = 0;  // Anderson history slots allocated at ks_create
  // Hartree
  double *vh_int = nullptr, *vh_nodes = nullptr, *wB = nullptr, *load = nullptr, *rhs = nullptr,
         *mom = nullptr, *mpart = nullptr;
  bool vh_warm = false;
  // coarse
  int32_t *Pidx = nullptr;
  double *Pw = nullptr, *Z = nullptr, *Y = nullptr, *GPP = nullptr, *GPPinv = nullptr,
         *FAL_PP = nullptr;
  // small dense
  double *FB = nullptr, *FAL = nullptr, *FA = nullptr, *Ftail = nullptr, *Ctmp = nullptr,
         *Ttmp = nullptr, *U = nullptr, *theta = nullptr, *eigwork = nullptr, *gwork = nullptr,
         *coef = nullptr, *redpart = nullptr;
  size_t gwork_n = 0;
  int *einfo = nullptr;
  // two-stage eigensolver state: D, V, X (orthogonalised F_B basis), W (warm
  // start eigenvectors), scratch T1, T2; rank r of the current F_B
  double *eRot = nullptr;  // Jacobi rotation log
  double *eD = nullptr, *eV = nullptr, *eX = nullptr, *eW = nullptr, *eT1 = nullptr, *eT2 = nullptr, *eS = nullptr, *eLam = nullptr;
  int e_rank = 0, e_m = 0;
  // state of the most recent ks_scf_step (for its energy and adjoint)
  bool have_step = false, last_nonlinear = false;
  bool last_inner_converged = false;  // the last step's inner iteration met tol_inner
  int last_k = 0;
  std::vector<double> last_theta, last_occ, last_lam_in;  // Ritz values out, occupations, eigenvalues in
  int last_precision = 0;
  double *aux1 = nullptr, *aux2 = nullptr, *Rv = nullptr, *Gv = nullptr, *dMk = nullptr;
  bool vext_atomic = true;  // V_ext is the nuclear potential of (hZ, hR), not a given field
  // per node its (element, local vertex) records 4 e + v (mesh-vertex derivative)
  int32_t *vinc_ptr = nullptr, *vinc_rec = nullptr;
  // block vectors [N][k_max]
  double *Bv = nullptr, *Xv = nullptr, *Wv = nullptr, *PsiHat = nullptr, *PsiNew = nullptr,
         *occ_d = nullptr, *scal = nullptr;
  double *PsiIn = nullptr, *Xs = nullptr;  // API-order inputs in storage order; solve output
  float *X32 = nullptr;
  PCGWork pw64{}, pw32{}, pwP{};
  // halo tilings of the CSR pattern for the LDS-staged SpMM, row blocks of
  // TILE_BR[i] rows; chosen tiling per solver (-1 = row kernel)
  static constexpr int NTILE = 6;
  Multigrid *mg = nullptr;  // V-cycle hierarchy of the Poisson operator (nullptr: Jacobi-PCG)
  int mg_iters_last = 0;
  Tiling til[NTILE];
  int tile64 = -1, tile32 = -1, tileP = -1;
  unsigned int *counters = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  template <typename T>
  int alloc(T **p, size_t count) {
    void *q = nullptr;
    size_t bytes = std::max<size_t>(sizeof(T) * count, 256);
    if (hipMalloc(&q, bytes) != hipSuccess) return fail(KS_ERR_NOMEM, "hipMalloc failed");
    mem.ptrs.push_back(q);
    *p = reinterpret_cast<T *>(q);
    return KS_OK;
  }
  ~ks_ctx() {
    if (mg) mg_destroy(mg);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

static void dbg(ks_ctx *c, const char *what, const double *buf, int64_t n) {
  if (!debug_on()) return;
  hipError_t e1 = hipStreamSynchronize(c->s);
  hipError_t e2 = hipGetLastError();
  double mn = 0, mx = 0, sa = 0;
  int64_t nan = 0;
  if (buf && n > 0) {
    std::vector<double> h(n);
    (void)hipMemcpy(h.data(), buf, sizeof(double) * n, hipMemcpyDeviceToHost);
    mn = h[0];
    mx = h[0];
    for (double v : h) {
      if (std::isnan(v)) { ++nan; continue; }
      mn = std::min(mn, v);
      mx = std::max(mx, v);
      sa += std::fabs(v);
    }
  }
  std::fprintf(stderr, "[ks-debug] %-28s sync=%s last=%s n=%lld min=%.6e max=%.6e sum|.|=%.6e nan=%lld\n",
               what, hipGetErrorString(e1), hipGetErrorString(e2), (long long)n, mn, mx, sa,
               (long long)nan);
}

#define TRY(x)                 \
  do {                         \
    int r_ = (x);              \
    if (r_ < 0) return r_;     \
  } while (0)

extern "C" const char *ks_last_error(void) { return g_err.c_str(); }

extern "C" int ks_options_default(ks_options *o) {
  if (!o) return fail(KS_ERR_ARG, "null options");
  std::memset(o, 0, sizeof(*o));
  o->mu = -1.0;
  o->n_H = 4;
  o->xc_mode = KS_XC_X_PZ81;
  o->hartree_mode = KS_HARTREE_MULTIPOLE;
  o->k_max = 8;
  o->tol_solve = 1e-8;
  o->tol_inner = 1e-8;
  o->tol_poisson = 1e-10;
  o->max_it_solve = 5000;
  o->max_it_inner = 50;
  o->max_it_poisson = 20000;
  o->anderson_depth = 5;
  o->anderson_beta = 0.7;
  o->mixed_inner_tol = 1e-5;
  o->deterministic = 1;
  return KS_OK;
}

extern "C" int ks_set_options(ks_ctx *c, const ks_options *o) {
  if (!c || !o) return fail(KS_ERR_ARG, "null argument");
  const ks_options &p = c->opt;
  if (o->mu != p.mu || o->n_H != p.n_H || o->xc_mode != p.xc_mode || o->hartree_mode != p.hartree_mode ||
      o->k_max != p.k_max)
    return fail(KS_ERR_ARG, "mu, n_H, xc_mode, hartree_mode and k_max are fixed at ks_create");
  if (o->anderson_depth < 1 || o->anderson_depth > c->hist_alloc)
    return fail(KS_ERR_ARG, "anderson_depth must be in 1..(the depth given at ks_create)");
  if (!(o->tol_solve > 0.0) || !(o->tol_inner > 0.0) || !(o->tol_poisson > 0.0) || !(o->mixed_inner_tol > 0.0) ||
      o->max_it_solve < 1 || o->max_it_inner < 1 || o->max_it_poisson < 1)
    return fail(KS_ERR_ARG, "tolerances must be > 0 and iteration limits >= 1");
  c->opt = *o;
  return KS_OK;
}

static int solve_impl(ks_ctx *c, const double *B, double *X, int k, int precision, double tol,
                      ks_solve_stats *st);
static int build_rhs(ks_ctx *c, const double *psi, const double *lambda_host, int k, double *B);
static int vjp_core(ks_ctx *c, const double *B, const double *X0, int k, double tol, int max_it, int seg,
                    const double *xb, double *X, double *g_q, double *Bbar, int32_t *iters_host);

// ------------------------------------------------------------ basis tables
static void basis_tables(int order, int n_q, const double *bary, std::vector<double> &phi,
                         std::vector<double> &dphi) {
  const int nl = order == 1 ? 4 : 10;
  static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  phi.assign((size_t)n_q * nl, 0.0);
  dphi.assign((size_t)n_q * nl * 4, 0.0);
  for (int q = 0; q < n_q; ++q) {
    const double *l = bary + 4 * q;
    if (order == 1) {
      for (int a = 0; a < 4; ++a) {
        phi[q * nl + a] = l[a];
        dphi[(q * nl + a) * 4 + a] = 1.0;
      }
    } else {
      for (int a = 0; a < 4; ++a) {
        phi[q * nl + a] = l[a] * (2.0 * l[a] - 1.0);
        dphi[(q * nl + a) * 4 + a] = 4.0 * l[a] - 1.0;
      }
      for (int e = 0; e < 6; ++e) {
        const int a = E[e][0], b = E[e][1];
        phi[q * nl + 4 + e] = 4.0 * l[a] * l[b];
        dphi[(q * nl + 4 + e) * 4 + a] = 4.0 * l[b];
        dphi[(q * nl + 4 + e) * 4 + b] = 4.0 * l[a];
      }
    }
  }
}

// ---------------------------------------------------------------- helpers
// Y = A X (B null) or Y = B - A X for an operator on the interior pattern
// (S, M, K, ...), X, Y, B row-major [N][k]: the halo tiles of the FP64 block
// solve when they serve k, else the row kernel
static void spmm_op(ks_ctx *c, const double *val, const double *X, int k, double *Y, const double *B) {
  if (c->pw64.til && launch_spmm_tiled(c->N, k, *c->pw64.til, c->pw64.til_tb, c->rowptr, val, X, Y, B, c->s) == 0)
    return;
  launch_spmm(c->N, c->rowptr, c->col, val, X, k, Y, k, k, B, k, B ? 1 : 0, c->rorder, c->s);
}

static int tile_index(int br);
// Y = A X over ncols columns, X and Y with row pitches ldx, ldy (elements):
// halo tiles over column chunks, else the row kernel
static void spmm_cols(ks_ctx *c, const double *val, const double *X, int ldx, double *Y, int ldy, int ncols) {
  // up to the solver's column count: one pass over the FP64 solver's tiling
  // (the operator is read once), where its LDS image fits these columns
  if (ncols <= c->k_max && c->pw64.til &&
      launch_spmm_tiled_cols(c->N, ncols, ldx, ldy, ncols, *c->pw64.til, c->pw64.til_tb, c->rowptr, val, X, Y,
                             nullptr, c->s) == 0)
    return;
  const int ti = tile_index(c->proj_br);
  if (ti >= 0 && c->til[ti].nblk &&
      launch_spmm_tiled_cols(c->N, ncols, ldx, ldy, c->proj_kc, c->til[ti], c->proj_tb, c->rowptr, val, X, Y,
                             nullptr, c->s) == 0)
    return;
  launch_spmm(c->N, c->rowptr, c->col, val, X, ldx, Y, ldy, ncols, nullptr, 0, 0, c->rorder, c->s);
}

static int reduce_small(ks_ctx *c, double *part, int nblk, int nvals, double *out_host) {
  launch_reduce_cols(part, nblk, nvals, c->mom + 64, c->s);
  HIPCHK(hipMemcpyAsync(out_host, c->mom + 64, sizeof(double) * nvals, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  return KS_OK;
}

// out = base + M[V] (eq. st4) over the interior pattern (base null: out =
// M[V]); out32: the FP32 copy of the values as well (nullptr: none).  The
// colour-scatter path, used when the row form does not fit, covers the
// extended pattern.
// Returns true when out32 was written.
static bool assemble_potential_all(ks_ctx *c, const double *Vq, double *out, const double *base = nullptr,
                                   float *out32 = nullptr) {
  if (c->r_lds &&  // one thread per row sums its own slots
      launch_assemble_rows(c->N, c->n_loc, c->n_q, c->rowptr, c->r_incptr, c->r_inc, c->r_perm, c->r_lds,
                           c->absdet, c->phi, c->phib, c->qw, Vq, base, out, out32, c->s) == 0)
    return out32 != nullptr;
  if (base) launch_axpby(c->nnz_ext, 1.0, base, 0.0, out, c->s);
  else launch_fill(c->nnz_ext, 0.0, out, c->s);
  for (int col = 0; col < c->n_colours; ++col) {
    const int a = c->colour_off[col], b = c->colour_off[col + 1];
    launch_assemble_potential(c->elem_perm + a, b - a, c->n_loc, c->n_q, c->slot, c->absdet,
                              c->pairtab, c->qw, Vq, out, c->s);
  }
  return false;
}

// V_H at the quadrature points for density rho with the frozen boundary
// data c->wB (Sec. 3.1): K_II V_I = 4 pi <rho, phi_I> - K_IB w_B.
// tol <= 0: the context's tol_poisson
static int hartree_solve(ks_ctx *c, const double *rho, int *iters, double tol = 0.0) {
  if (!(tol > 0.0)) tol = c->opt.tol_poisson;
  if (!c->r_lds || launch_load_rows(c->N, c->n_e, c->n_loc, c->n_q, c->r_incptr, c->r_inc, c->absdet, c->phi,
                                    c->qw, rho, 4.0 * M_PI, c->load_e, c->load, c->s) != 0) {
    launch_fill(c->N, 0.0, c->load, c->s);
    for (int col = 0; col < c->n_colours; ++col) {
      const int a = c->colour_off[col], b = c->colour_off[col + 1];
      launch_load_vector(c->elem_perm + a, b - a, c->n_loc, c->n_q, c->edof, c->absdet, c->phi,
                         c->qw, rho, 4.0 * M_PI, c->load, c->s);
    }
  }
  // rhs = load - K_IB wB
  launch_spmm(c->N, c->rowptrB, c->colB, c->K + c->nnz, c->wB, 1, c->rhs, 1, 1, c->load, 1, 1, c->rorder, c->s);
  if (!c->vh_warm) launch_fill(c->N, 0.0, c->vh_int, c->s);
  int it[1] = {0}, conv = 0, brk = 0;
  double rr[1];
  if (c->mg) {
    // CG preconditioned by one multigrid V-cycle per iteration
    const int r = mg_pcg(c->mg, c->rhs, c->vh_int, tol, c->opt.max_it_poisson, c->redpart,
                         c->mom + 64, it, rr, c->s);
    if (r == -1) return fail(KS_ERR_HIP, "Poisson MG-PCG failed");
    if (r == -2) return fail(KS_ERR_BREAKDOWN, "Poisson MG-PCG breakdown");
    conv = (r == 0);
  } else {
    int r = pcg_solve<double>(c->N, 1, c->rowptr, c->col, c->K, c->rorder, c->diagK, c->rhs, c->vh_int,
                              tol, c->opt.max_it_poisson, c->pwP, it, rr, &conv, &brk,
                              c->s, c->ngP);
    if (r < 0) return fail(KS_ERR_HIP, "Poisson PCG failed");
    if (brk) return fail(KS_ERR_BREAKDOWN, "Poisson PCG breakdown");
  }
  c->vh_warm = true;
  if (iters) *iters += it[0];
  launch_scatter_nodes(c->n_nodes, c->node2int, c->node2bnd, c->vh_int, c->wB, c->vh_nodes, c->s);
  launch_eval_nodal(c->elems, c->n_loc, c->n_e, c->n_q, c->phi, c->vh_nodes, c->vh_q, c->s);
  return conv ? KS_OK : KS_NOT_CONVERGED;
}

// w_D(rho) at the boundary nodes (eq. bd), stored in c->wB
static int boundary_data(ks_ctx *c, const double *rho) {
  const int nb = moments_blocks(c->n_e);
  double h[16];
  launch_moments(c->coords, c->elems, c->n_loc, c->n_e, c->n_q, c->qbary, c->qw, c->absdet, rho,
                 nullptr, c->mpart, 4, c->s);
  TRY(reduce_small(c, c->mpart, nb, 4, h));
  double mom[16] = {0};
  mom[0] = h[0];
  if (!(h[0] > 0.0)) return fail(KS_ERR_ARG, "density has no charge: cannot place the multipole centre");
  for (int d = 0; d < 3; ++d) mom[1 + d] = h[1 + d] / h[0];
  HIPCHK(hipMemcpyAsync(c->mom, mom, sizeof(double) * 16, hipMemcpyHostToDevice, c->s));
  launch_moments(c->coords, c->elems, c->n_loc, c->n_e, c->n_q, c->qbary, c->qw, c->absdet, rho,
                 c->mom + 1, c->mpart, 9, c->s);
  TRY(reduce_small(c, c->mpart, nb, 9, h));
  for (int j = 0; j < 9; ++j) mom[4 + j] = h[j];
  // mom[7..12] = q_xx q_xy q_xz q_yy q_yz q_zz (h[3..8])
  HIPCHK(hipMemcpyAsync(c->mom, mom, sizeof(double) * 16, hipMemcpyHostToDevice, c->s));
  const double f = c->opt.hartree_mode == KS_HARTREE_MULTIPOLE_LITERAL ? 1.0 : 0.5;
  launch_multipole(c->coords, c->bnodes, c->NB, c->mom, f, c->wB, c->s);
  return KS_OK;
}

static int weighted_dots(ks_ctx *c, int nd, const double *const *a, const double *const *b,
                         double *out) {
  const int64_t npts = (int64_t)c->n_e * c->n_q;
  launch_wdots(npts, c->n_q, c->absdet, c->qw, nd, a, b, c->redpart, c->s);
  return reduce_small(c, c->redpart, wdot_blocks(npts), nd, out);
}

// ------------------------------------------------------------------- create
// row-block sizes of the halo tilings
// (85 and 170 rows fill one pass of 512 / 1024 threads at 6 or 12 lanes per row)
static const int TILE_BR[ks_ctx::NTILE] = {32, 64, 85, 128, 170, 256};
static int tile_index(int br) {
  for (int i = 0; i < ks_ctx::NTILE; ++i)
    if (TILE_BR[i] == br) return i;
  return -1;
}
// tile choice code: NTB * tiling index + workgroup size index (256, 512,
// 1024 threads), -1 = row kernel
constexpr int NTB = 3;
static const int TILE_TB[NTB] = {256, 512, 1024};
static void apply_tiles(ks_ctx *c) {
  auto set = [&](PCGWork &w, int code) {
    const int i = code >= 0 ? code / NTB : -1;
    w.til = (i >= 0 && c->til[i].nblk) ? &c->til[i] : nullptr;
    w.til_tb = TILE_TB[code >= 0 ? code % NTB : 0];
  };
  set(c->pw64, c->tile64);
  set(c->pw32, c->tile32);
  set(c->pwP, c->tileP);
  mg_set_tiling(c->mg, c->pwP.til, c->pwP.til_tb);
}

extern "C" int ks_create(const ks_mesh_desc *mesh, const ks_quad_desc *quad,
                         const ks_atoms_desc *atoms, const ks_options *opt, hipStream_t stream,
                         ks_ctx **out) {
  return ks_create_nonnested(mesh, nullptr, quad, atoms, opt, stream, out);
}

extern "C" int ks_create_nonnested(const ks_mesh_desc *mesh, const ks_mesh_desc *coarse,
                                   const ks_quad_desc *quad, const ks_atoms_desc *atoms, const ks_options *opt,
                                   hipStream_t stream, ks_ctx **out) {
  if (!mesh || !quad || !atoms || !out) return fail(KS_ERR_ARG, "null argument");
  if (coarse && (coarse->order != 1 || coarse->n_nodes < 4 || coarse->n_elems < 1 || !coarse->coords_host ||
                 !coarse->elems_host || !coarse->dirichlet_host))
    return fail(KS_ERR_ARG, "coarse mesh: P1 tetrahedra with coordinates, elements and Dirichlet flags");
  if (!mesh->coords_host || !mesh->elems_host || !mesh->dirichlet_host)
    return fail(KS_ERR_ARG, "mesh arrays missing");
  if (mesh->order != 1 && mesh->order != 2) return fail(KS_ERR_ARG, "order must be 1 or 2");
  if (mesh->n_nodes <= 0 || mesh->n_elems <= 0) return fail(KS_ERR_ARG, "empty mesh");
  if (quad->n_q <= 0 || quad->n_q > MAX_NQ || !quad->bary_host || !quad->w_host)
    return fail(KS_ERR_ARG, "quadrature must have 1..27 points");
  if ((quad->n_q != 8 && quad->n_q != 27))
    return fail(KS_ERR_ARG, "quadrature rules with 8 or 27 points are supported");
  if (atoms->n_atoms < 0 || (atoms->n_atoms > 0 && (!atoms->Z_host || !atoms->R_host)))
    return fail(KS_ERR_ARG, "bad atoms");
  ks_options o;
  if (opt) o = *opt;
  else ks_options_default(&o);
  if (o.k_max < 1 || o.k_max > MAX_K) return fail(KS_ERR_ARG, "k_max must be in 1..64");
  if (o.n_H < 2) return fail(KS_ERR_ARG, "n_H must be >= 2");
  if (o.anderson_depth < 1 || o.anderson_depth > 5) return fail(KS_ERR_ARG, "anderson_depth in 1..5");

  ks_ctx *c = new ks_ctx();
  auto bail = [&](int code) {
    delete c;
    return code;
  };
  c->s = stream;
  c->opt = o;
  c->order = mesh->order;
  c->n_loc = mesh->order == 1 ? 4 : 10;
  c->n_nodes = mesh->n_nodes;
  c->n_e = mesh->n_elems;
  c->n_q = quad->n_q;
  c->L = mesh->L;
  c->n_H = o.n_H;
  c->N_H = (o.n_H - 1) * (o.n_H - 1) * (o.n_H - 1);
  std::vector<int32_t> cint;  // coarse vertex -> coarse unknown (-1 on the coarse boundary)
  if (coarse) {
    cint.assign(coarse->n_nodes, -1);
    int nh = 0;
    for (int v = 0; v < coarse->n_nodes; ++v)
      if (!coarse->dirichlet_host[v]) cint[v] = nh++;
    if (nh < 1) return bail(fail(KS_ERR_MESH, "coarse mesh has no interior vertex"));
    c->n_H = 0;
    c->N_H = nh;
  }
  c->k_max = o.k_max;
  if (c->N_H + c->k_max > 256) return bail(fail(KS_ERR_ARG, "N_H + k_max must be <= 256"));
  c->mp = (c->N_H + c->k_max + 15) / 16 * 16;
  c->n_atoms = atoms->n_atoms;
  c->hZ.assign(atoms->Z_host, atoms->Z_host + atoms->n_atoms);
  c->hR.assign(atoms->R_host, atoms->R_host + 3 * atoms->n_atoms);
  double sz2 = 0.0;
  for (double z : c->hZ) sz2 += z * z;
  c->mu = o.mu >= 0.0 ? o.mu : 8.0 * c->n_atoms * sz2;
  for (int j = 0; j < c->n_atoms; ++j)
    for (int k = 0; k < j; ++k) {
      double dx = c->hR[3 * j] - c->hR[3 * k], dy = c->hR[3 * j + 1] - c->hR[3 * k + 1],
             dz = c->hR[3 * j + 2] - c->hR[3 * k + 2];
      c->E_nn += c->hZ[j] * c->hZ[k] / std::sqrt(dx * dx + dy * dy + dz * dz);
    }

  const int nl = c->n_loc, ne = c->n_e, nn = c->n_nodes;
  const int32_t *el = mesh->elems_host;
  for (int64_t i = 0; i < (int64_t)ne * nl; ++i)
    if (el[i] < 0 || el[i] >= nn) return bail(fail(KS_ERR_MESH, "element node id out of range"));
  // interior / boundary numbering.  The unknowns are stored in Morton
  // (Z-curve) order of their node coordinates, so that consecutive rows are
  // spatial neighbours (compact row blocks, short gather distances); the API
  // numbers them by ascending node id ("natural" index) and every DOF-indexed
  // argument is permuted at the boundary (int2nat).
  std::vector<int32_t> node2int(nn, -1), node2bnd(nn, -1), bnodes, nat_nodes;
  for (int i = 0; i < nn; ++i) {
    if (mesh->dirichlet_host[i]) {
      node2bnd[i] = (int)bnodes.size();
      bnodes.push_back(i);
    } else {
      nat_nodes.push_back(i);
    }
  }
  const int N = (int)nat_nodes.size();
  c->N = N;
  c->NB = (int)bnodes.size();
  if (N == 0) return bail(fail(KS_ERR_MESH, "mesh has no interior node"));
  c->h_int2nat.resize(N);
  for (int r = 0; r < N; ++r) c->h_int2nat[r] = r;
  {
    {
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int r = 0; r < N; ++r)
        for (int d = 0; d < 3; ++d) {
          const double x = mesh->coords_host[3 * (int64_t)nat_nodes[r] + d];
          lo[d] = std::min(lo[d], x);
          hi[d] = std::max(hi[d], x);
        }
      std::vector<uint64_t> key(N);
      parallel_for(N, [&](int64_t r) {
        uint64_t q[3];
        for (int d = 0; d < 3; ++d) {
          const double x = mesh->coords_host[3 * (int64_t)nat_nodes[r] + d];
          const double t = (hi[d] > lo[d]) ? (x - lo[d]) / (hi[d] - lo[d]) : 0.0;
          q[d] = (uint64_t)std::min(1048575.0, std::max(0.0, std::floor(t * 1048576.0)));
        }
        uint64_t k = 0;
        for (int b = 19; b >= 0; --b)
          for (int d = 2; d >= 0; --d) k = (k << 1) | ((q[d] >> b) & 1u);
        key[r] = k;
      });
      std::stable_sort(c->h_int2nat.begin(), c->h_int2nat.end(),
                       [&](int32_t x, int32_t y) { return key[x] < key[y]; });
    }
  }
  for (int r = 0; r < N; ++r) node2int[nat_nodes[c->h_int2nat[r]]] = r;
  std::vector<int32_t> edof((size_t)ne * nl);
  for (int64_t i = 0; i < (int64_t)ne * nl; ++i) edof[i] = node2int[el[i]];
  // node -> element adjacency
  std::vector<int64_t> nadj_off(nn + 1, 0);
  for (int64_t i = 0; i < (int64_t)ne * nl; ++i) nadj_off[el[i] + 1]++;
  for (int i = 0; i < nn; ++i) nadj_off[i + 1] += nadj_off[i];
  std::vector<int32_t> nadj(nadj_off[nn]);
  {
    std::vector<int64_t> pos(nadj_off.begin(), nadj_off.end() - 1);
    for (int e = 0; e < ne; ++e)
      for (int a = 0; a < nl; ++a) nadj[pos[el[(int64_t)e * nl + a]]++] = e;
  }
  // CSR pattern: interior rows; interior columns, then boundary columns (K_IB)
  std::vector<int32_t> rowptr(N + 1, 0), rowptrB(N + 1, 0);
  std::vector<int32_t> interior_nodes(N);
  for (int i = 0; i < nn; ++i)
    if (node2int[i] >= 0) interior_nodes[node2int[i]] = i;
  auto row_cols = [&](int r, std::vector<int32_t> &ci, std::vector<int32_t> &cb) {
    ci.clear();
    cb.clear();
    const int nd = interior_nodes[r];
    for (int64_t p = nadj_off[nd]; p < nadj_off[nd + 1]; ++p) {
      const int e = nadj[p];
      for (int b = 0; b < nl; ++b) {
        const int m = el[(int64_t)e * nl + b];
        if (node2int[m] >= 0) ci.push_back(node2int[m]);
        else cb.push_back(node2bnd[m]);
      }
    }
    std::sort(ci.begin(), ci.end());
    ci.erase(std::unique(ci.begin(), ci.end()), ci.end());
    std::sort(cb.begin(), cb.end());
    cb.erase(std::unique(cb.begin(), cb.end()), cb.end());
  };
  {
    std::vector<int32_t> cntI(N), cntB(N);
    parallel_for(N, [&](int64_t r) {
      thread_local std::vector<int32_t> ci, cb;
      row_cols((int)r, ci, cb);
      cntI[r] = (int32_t)ci.size();
      cntB[r] = (int32_t)cb.size();
    });
    int64_t sI = 0, sB = 0;
    for (int r = 0; r < N; ++r) {
      sI += cntI[r];
      sB += cntB[r];
      if (sI > 2000000000LL) return bail(fail(KS_ERR_ARG, "nnz exceeds int32 range"));
      rowptr[r + 1] = (int32_t)sI;
      rowptrB[r + 1] = (int32_t)sB;
    }
  }
  c->nnz = rowptr[N];
  c->nnzB = rowptrB[N];
  c->nnz_ext = c->nnz + c->nnzB;
  std::vector<int32_t> colI(c->nnz), colB(std::max<int64_t>(1, c->nnzB));
  parallel_for(N, [&](int64_t r) {
    thread_local std::vector<int32_t> ci, cb;
    row_cols((int)r, ci, cb);
    std::copy(ci.begin(), ci.end(), colI.begin() + rowptr[r]);
    std::copy(cb.begin(), cb.end(), colB.begin() + rowptrB[r]);
  });
  // halo tilings (row blocks of consecutive rows in the Morton storage order)
  std::vector<int32_t> t_hptr[ks_ctx::NTILE], t_hcol[ks_ctx::NTILE], t_hself[ks_ctx::NTILE];
  std::vector<uint16_t> t_lcol[ks_ctx::NTILE], t_lbyte[ks_ctx::NTILE];
  std::vector<int32_t> t_pptr[ks_ctx::NTILE];
  // padded index runs: row r's local indices start at prp[r], a multiple of 8
  std::vector<int64_t> prp(N + 1, 0);
  for (int r = 0; r < N; ++r) prp[r + 1] = prp[r] + (rowptr[r + 1] - rowptr[r] + 7) / 8 * 8;
  std::vector<uint32_t> t_rmeta[ks_ctx::NTILE];
  for (int ti = 0; ti < ks_ctx::NTILE; ++ti) {
    const int BR = TILE_BR[ti];
    const int nblk = (N + BR - 1) / BR;
    std::vector<std::vector<int32_t>> halos(nblk);
    t_lcol[ti].assign((size_t)prp[N], 0);
    std::vector<int> ok(nblk, 1);
    parallel_for(nblk, [&](int64_t b) {
      const int r0 = (int)b * BR, r1 = std::min(N, r0 + BR);
      std::vector<int32_t> &h = halos[b];
      h.assign(colI.begin() + rowptr[r0], colI.begin() + rowptr[r1]);
      std::sort(h.begin(), h.end());
      h.erase(std::unique(h.begin(), h.end()), h.end());
      if (h.size() > 65534) {  // local indices and the zero row index fit 16 bits
        ok[b] = 0;
        return;
      }
      for (int r = r0; r < r1; ++r)
        for (int64_t j = rowptr[r]; j < rowptr[r + 1]; ++j)
          t_lcol[ti][prp[r] + (j - rowptr[r])] =
              (uint16_t)(std::lower_bound(h.begin(), h.end(), colI[j]) - h.begin());
    });
    bool all = true;
    for (int b = 0; b < nblk; ++b) all = all && ok[b];
    if (!all) continue;  // halo too large for 16-bit local indices: tiling unused
    t_hptr[ti].assign(nblk + 1, 0);
    int mx = 0;
    for (int b = 0; b < nblk; ++b) {
      t_hptr[ti][b + 1] = t_hptr[ti][b] + (int32_t)halos[b].size();
      mx = std::max(mx, (int)halos[b].size());
    }
    // padding slots of every index run point at halo row mx, which the
    // kernel keeps at zero: the padded nonzeros add exact zeros
    parallel_for(N, [&](int64_t r) {
      for (int64_t q = prp[r] + (rowptr[r + 1] - rowptr[r]); q < prp[r + 1]; ++q) t_lcol[ti][q] = (uint16_t)mx;
    });
    int mnz = 0;
    t_hself[ti].resize(nblk);
    for (int b = 0; b < nblk; ++b) {
      mnz = std::max(mnz, rowptr[std::min(N, (b + 1) * BR)] - rowptr[b * BR]);
      // every row has its diagonal, so the block's rows form one run of the
      // sorted halo; hself = where it starts
      const int r0 = b * BR, nr = std::min(BR, N - r0);
      const int hs = (int)(std::lower_bound(halos[b].begin(), halos[b].end(), r0) - halos[b].begin());
      t_hself[ti][b] = hs;
      for (int rr = 0; rr < nr; ++rr)
        if (hs + rr >= (int)halos[b].size() || halos[b][hs + rr] != r0 + rr) all = false;
    }
    if (!all) {  // a row without its diagonal entry: tiling unused
      c->til[ti] = Tiling();
      continue;
    }
    // the packed row slots need block nonzero offsets below 2^16 and rows
    // of at most 255 nonzeros
    bool fits = mnz < 65536 && prp[N] < ((int64_t)1 << 31);
    for (int r = 0; r < N && fits; ++r) fits = rowptr[r + 1] - rowptr[r] <= 255;
    if (!fits) {
      c->til[ti] = Tiling();
      continue;
    }
    c->til[ti].max_nnz = mnz;
    t_pptr[ti].assign(nblk + 1, 0);
    int mpz = 0;
    for (int b = 0; b <= nblk; ++b) t_pptr[ti][b] = (int32_t)prp[std::min(N, b * BR)];
    for (int b = 0; b < nblk; ++b) mpz = std::max(mpz, t_pptr[ti][b + 1] - t_pptr[ti][b]);
    c->til[ti].max_pnz = mpz;
    // within each block: longest rows first (stable), so that a wavefront's
    // rows have similar nonzero counts; each slot packs the row's offset in
    // the block, its nonzero count and its first nonzero (block-relative)
    t_rmeta[ti].resize((size_t)2 * N);
    parallel_for(nblk, [&](int64_t b) {
      const int r0 = (int)b * BR, nr = std::min(BR, N - r0);
      std::vector<int> o(nr);
      for (int rr = 0; rr < nr; ++rr) o[rr] = rr;
      std::stable_sort(o.begin(), o.end(), [&](int x, int y) {
        return rowptr[r0 + x + 1] - rowptr[r0 + x] > rowptr[r0 + y + 1] - rowptr[r0 + y];
      });
      for (int s = 0; s < nr; ++s) {
        const int rr = o[s];
        const uint32_t rel = (uint32_t)(rowptr[r0 + rr] - rowptr[r0]);
        const uint32_t len = (uint32_t)(rowptr[r0 + rr + 1] - rowptr[r0 + rr]);
        t_rmeta[ti][2 * (size_t)(r0 + s)] = rel | (len << 16) | ((uint32_t)rr << 24);
        t_rmeta[ti][2 * (size_t)(r0 + s) + 1] = (uint32_t)(prp[r0 + rr] - prp[r0]);
      }
    });
    t_hcol[ti].resize(t_hptr[ti][nblk]);
    parallel_for(nblk, [&](int64_t b) {
      std::copy(halos[b].begin(), halos[b].end(), t_hcol[ti].begin() + t_hptr[ti][b]);
    });
    c->til[ti].BR = BR;
    c->til[ti].nblk = nblk;
    c->til[ti].max_halo = mx;
  }
  // element -> value slot map (interior rows only)
  std::vector<int32_t> slot((size_t)ne * nl * nl, -1);
  parallel_for(ne, [&](int64_t e) {
    for (int a = 0; a < nl; ++a) {
      const int ra = edof[e * nl + a];
      if (ra < 0) continue;
      for (int b = 0; b < nl; ++b) {
        const int m = el[e * nl + b];
        int32_t sidx;
        if (node2int[m] >= 0) {
          const int cb = node2int[m];
          const int32_t *p = std::lower_bound(colI.data() + rowptr[ra], colI.data() + rowptr[ra + 1], cb);
          sidx = (int32_t)(p - colI.data());
        } else {
          const int cb = node2bnd[m];
          const int32_t *p =
              std::lower_bound(colB.data() + rowptrB[ra], colB.data() + rowptrB[ra + 1], cb);
          sidx = (int32_t)(c->nnz + (p - colB.data()));
        }
        slot[(e * nl + a) * nl + b] = sidx;
      }
    }
  });
  // row form of the potential assembly (see r_incptr): the incidences of
  // every storage row in ascending element order, and per row block its rows
  // ordered by incidence count (longest first)
  std::vector<int32_t> r_incptr;
  std::vector<uint8_t> r_inc, r_perm;
  size_t r_lds = 0;
  {
    const int RS = nl == 10 ? 16 : 8;  // bytes per record (IncRec)
    int maxlen = 0;
    for (int r = 0; r < N; ++r) maxlen = std::max(maxlen, rowptr[r + 1] - rowptr[r]);
    size_t blk = 0;
    for (int r0 = 0; r0 < N; r0 += ASM_ROWS)
      blk = std::max(blk, (size_t)(rowptr[std::min(N, r0 + ASM_ROWS)] - rowptr[r0]) * sizeof(double));
    if ((nl == 4 || nl == 10) && (c->n_q == 8 || c->n_q == 27) && ne < (1 << 27) && maxlen < 255 && (int64_t)ne * nl < INT32_MAX &&
        blk <= assemble_rows_lds_limit()) {
      r_incptr.assign(N + 1, 0);
      for (int64_t x = 0; x < (int64_t)ne * nl; ++x)
        if (edof[x] >= 0) r_incptr[edof[x] + 1]++;
      for (int r = 0; r < N; ++r) r_incptr[r + 1] += r_incptr[r];
      r_inc.assign((size_t)r_incptr[N] * RS, 0);
      std::vector<int32_t> pos(r_incptr.begin(), r_incptr.end() - 1);
      for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < nl; ++a) {
          const int r = edof[e * nl + a];
          if (r < 0) continue;
          uint8_t *rec = r_inc.data() + (size_t)pos[r]++ * RS;
          const uint32_t ea = (uint32_t)e << 4 | (uint32_t)a;
          std::memcpy(rec, &ea, 4);
          for (int b = 0; b < nl; ++b) {
            const int32_t sl = slot[(e * nl + a) * nl + b];
            rec[4 + b] = (sl >= 0 && sl < c->nnz) ? (uint8_t)(sl - rowptr[r]) : (uint8_t)255;
          }
        }
      r_perm.resize(N);
      parallel_for((N + ASM_ROWS - 1) / ASM_ROWS, [&](int64_t bk) {
        const int r0 = (int)bk * ASM_ROWS, nr = std::min(ASM_ROWS, N - r0);
        std::vector<int> ord(nr);
        for (int t = 0; t < nr; ++t) ord[t] = t;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
          return r_incptr[r0 + x + 1] - r_incptr[r0 + x] > r_incptr[r0 + y + 1] - r_incptr[r0 + y];
        });
        for (int t = 0; t < nr; ++t) r_perm[r0 + t] = (uint8_t)ord[t];
      });
      r_lds = std::max<size_t>(blk, 8);
    }
  }
  // greedy element colouring: no two elements of one colour share a node
  std::vector<int16_t> colour(ne, -1);
  int ncol = 0;
  {
    std::vector<uint8_t> used(1024, 0);
    std::vector<int> touched;
    for (int e = 0; e < ne; ++e) {
      touched.clear();
      for (int a = 0; a < nl; ++a) {
        const int nd = el[(int64_t)e * nl + a];
        for (int64_t p = nadj_off[nd]; p < nadj_off[nd + 1]; ++p) {
          const int f = nadj[p];
          const int cf = colour[f];
          if (cf >= 0 && !used[cf]) {
            used[cf] = 1;
            touched.push_back(cf);
          }
        }
      }
      int cc = 0;
      while (cc < 1024 && used[cc]) ++cc;
      if (cc >= 1024) return bail(fail(KS_ERR_MESH, "element colouring needs more than 1024 colours"));
      colour[e] = (int16_t)cc;
      ncol = std::max(ncol, cc + 1);
      for (int t : touched) used[t] = 0;
    }
  }
  c->n_colours = ncol;
  c->colour_off.assign(ncol + 1, 0);
  for (int e = 0; e < ne; ++e) c->colour_off[colour[e] + 1]++;
  for (int k = 0; k < ncol; ++k) c->colour_off[k + 1] += c->colour_off[k];
  std::vector<int32_t> perm(ne);
  {
    std::vector<int> pos(c->colour_off.begin(), c->colour_off.end() - 1);
    for (int e = 0; e < ne; ++e) perm[pos[colour[e]]++] = e;
  }
  // coarse interpolation (closed-form location in the uniform Kuhn mesh, or
  // Algorithm 1 in a given nonnested coarse mesh)
  std::vector<int32_t> Pidx((size_t)N * 4, -1);
  std::vector<double> Pw((size_t)N * 4, 0.0);
  if (coarse) {
    std::vector<double> pts((size_t)N * 3);
    for (int r = 0; r < N; ++r)
      for (int d = 0; d < 3; ++d) pts[3 * (size_t)r + d] = mesh->coords_host[3 * (int64_t)interior_nodes[r] + d];
    std::vector<int32_t> vid((size_t)N * 4);
    std::vector<double> wv((size_t)N * 4);
    const int rc = nonnested_weights(coarse->n_nodes, coarse->coords_host, coarse->n_elems, coarse->elems_host, N,
                                     pts.data(), vid.data(), wv.data());
    if (rc == -1) return bail(fail(KS_ERR_MESH, "coarse mesh: bad element vertex ids"));
    for (int r = 0; r < N; ++r) {
      int cnt = 0;
      for (int j = 0; j < 4; ++j) {
        const int ci = cint[vid[4 * (size_t)r + j]];
        if (ci < 0 || wv[4 * (size_t)r + j] == 0.0) continue;  // coarse boundary vertex: no basis function
        // an index seen before in this row (an element with a repeated
        // vertex) takes the weight: the row's indices stay distinct
        int dup = -1;
        for (int q = 0; q < cnt; ++q)
          if (Pidx[4 * (size_t)r + q] == ci) dup = q;
        if (dup >= 0) {
          Pw[4 * (size_t)r + dup] += wv[4 * (size_t)r + j];
          continue;
        }
        Pidx[4 * (size_t)r + cnt] = ci;
        Pw[4 * (size_t)r + cnt] = wv[4 * (size_t)r + j];
        ++cnt;
      }
    }
  } else {
    const int nH = c->n_H, ni = nH - 1;
    const double h = 2.0 * c->L / nH;
    parallel_for(N, [&](int64_t r) {
      const double *x = mesh->coords_host + 3 * (int64_t)interior_nodes[r];
      int cell[3];
      double xi[3];
      for (int d = 0; d < 3; ++d) {
        const double t = (x[d] + c->L) / h;
        int ci = (int)std::floor(t);
        ci = std::max(0, std::min(nH - 1, ci));
        cell[d] = ci;
        xi[d] = t - ci;
      }
      int ord[3] = {0, 1, 2};
      // descending xi, ties by axis index
      std::sort(ord, ord + 3, [&](int a, int b) { return xi[a] > xi[b] || (xi[a] == xi[b] && a < b); });
      const double lam[4] = {1.0 - xi[ord[0]], xi[ord[0]] - xi[ord[1]], xi[ord[1]] - xi[ord[2]],
                             xi[ord[2]]};
      int v[3] = {cell[0], cell[1], cell[2]};
      int cnt = 0;
      for (int j = 0; j < 4; ++j) {
        if (j > 0) v[ord[j - 1]] += 1;
        bool inner = true;
        for (int d = 0; d < 3; ++d)
          if (v[d] <= 0 || v[d] >= nH) inner = false;
        if (!inner) continue;
        Pidx[4 * r + cnt] = (v[0] - 1) + ni * ((v[1] - 1) + ni * (v[2] - 1));
        Pw[4 * r + cnt] = lam[j];
        ++cnt;
      }
    });
  }
  // coarse blocks of the projection (launch_proj_coarse): own and neighbour
  // coarse index lists per block of CP_ROWS rows, partial offsets and the
  // gather lists of every output (blocks in ascending order)
  std::vector<int32_t> cp_uoff, cp_ulist, cp_noff, cp_nlist, cp_gpp_ptr, cp_gpt_ptr;
  std::vector<int64_t> cp_ppoff, cp_ptoff, cp_gpp_idx, cp_gpt_idx;
  int cp_ok = 0, cp_ldt = 0, cp_ldo = 0;
  const int cp_nblk = (N + CP_ROWS - 1) / CP_ROWS;
  if (c->N_H <= 256) {
    std::vector<std::vector<int32_t>> own(cp_nblk), nbr(cp_nblk);
    parallel_for(cp_nblk, [&](int64_t b) {
      const int r0 = (int)b * CP_ROWS, r1 = std::min(N, r0 + CP_ROWS);
      for (int r = r0; r < r1; ++r) {
        for (int cc = 0; cc < 4; ++cc)
          if (Pidx[4 * (size_t)r + cc] >= 0) own[b].push_back(Pidx[4 * (size_t)r + cc]);
        for (int jj = rowptr[r]; jj < rowptr[r + 1]; ++jj)
          for (int cc = 0; cc < 4; ++cc)
            if (Pidx[4 * (size_t)colI[jj] + cc] >= 0) nbr[b].push_back(Pidx[4 * (size_t)colI[jj] + cc]);
      }
      for (auto *v : {&own[b], &nbr[b]}) {
        std::sort(v->begin(), v->end());
        v->erase(std::unique(v->begin(), v->end()), v->end());
      }
    });
    cp_ok = 1;
    for (int b = 0; b < cp_nblk; ++b) {
      cp_ldo = std::max(cp_ldo, (int)own[b].size());
      cp_ldt = std::max(cp_ldt, (int)nbr[b].size());
    }
    cp_ldt = std::max(cp_ldt, 1);
    cp_ldo = std::max(cp_ldo, 1);
    if (sizeof(double) * (size_t)CP_ROWS * (cp_ldt + 1 + cp_ldo + c->k_max) > 60 * 1024) cp_ok = 0;
    if (cp_ok) {
      const int nH = c->N_H, km = c->k_max;
      cp_uoff.assign(cp_nblk + 1, 0);
      cp_noff.assign(cp_nblk + 1, 0);
      cp_ppoff.assign(cp_nblk + 1, 0);
      cp_ptoff.assign(cp_nblk + 1, 0);
      for (int b = 0; b < cp_nblk; ++b) {
        cp_uoff[b + 1] = cp_uoff[b] + (int)own[b].size();
        cp_noff[b + 1] = cp_noff[b] + (int)nbr[b].size();
        cp_ppoff[b + 1] = cp_ppoff[b] + (int64_t)own[b].size() * nbr[b].size();
        cp_ptoff[b + 1] = cp_ptoff[b] + (int64_t)own[b].size() * km;
        cp_ulist.insert(cp_ulist.end(), own[b].begin(), own[b].end());
        cp_nlist.insert(cp_nlist.end(), nbr[b].begin(), nbr[b].end());
      }
      // gather lists: (I, J) of the P^T H P block and I of the P^T Y block
      cp_gpp_ptr.assign((size_t)nH * nH + 1, 0);
      cp_gpt_ptr.assign(nH + 1, 0);
      for (int b = 0; b < cp_nblk; ++b)
        for (int I : own[b]) {
          cp_gpt_ptr[I + 1]++;
          for (int J : nbr[b]) cp_gpp_ptr[(size_t)I * nH + J + 1]++;
        }
      for (size_t o = 0; o < (size_t)nH * nH; ++o) cp_gpp_ptr[o + 1] += cp_gpp_ptr[o];
      for (int I = 0; I < nH; ++I) cp_gpt_ptr[I + 1] += cp_gpt_ptr[I];
      cp_gpp_idx.resize(cp_gpp_ptr[(size_t)nH * nH]);
      cp_gpt_idx.resize(cp_gpt_ptr[nH]);
      std::vector<int32_t> fpp(cp_gpp_ptr.begin(), cp_gpp_ptr.end() - 1), fpt(cp_gpt_ptr.begin(), cp_gpt_ptr.end() - 1);
      for (int b = 0; b < cp_nblk; ++b) {
        const int nv = (int)nbr[b].size();
        for (int u = 0; u < (int)own[b].size(); ++u) {
          const int I = own[b][u];
          cp_gpt_idx[fpt[I]++] = cp_ptoff[b] + (int64_t)u * km;
          for (int v = 0; v < nv; ++v) cp_gpp_idx[fpp[(size_t)I * nH + nbr[b][v]]++] = cp_ppoff[b] + (int64_t)u * nv + v;
        }
      }
    }
  }
  // row schedule: interior rows in Morton (Z-curve) order of their
  // coordinates, so the workgroups in flight sweep compact 3D regions.  The
  // unknowns are already stored in that order, so the solvers run in storage
  // order (rorder = nullptr) and this schedule stays unused.
  std::vector<int32_t> rorder(N);
  {
    for (int r = 0; r < N; ++r) rorder[r] = r;
    {
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int r = 0; r < N; ++r)
        for (int d = 0; d < 3; ++d) {
          const double x = mesh->coords_host[3 * (int64_t)interior_nodes[r] + d];
          lo[d] = std::min(lo[d], x);
          hi[d] = std::max(hi[d], x);
        }
      std::vector<uint64_t> key(N);
      parallel_for(N, [&](int64_t r) {
        uint64_t q[3];
        for (int d = 0; d < 3; ++d) {
          const double x = mesh->coords_host[3 * (int64_t)interior_nodes[r] + d];
          const double t = (hi[d] > lo[d]) ? (x - lo[d]) / (hi[d] - lo[d]) : 0.0;
          q[d] = (uint64_t)std::min(1023.0, std::max(0.0, std::floor(t * 1024.0)));
        }
        uint64_t k = 0;
        for (int b = 9; b >= 0; --b)
          for (int d = 2; d >= 0; --d) k = (k << 1) | ((q[d] >> b) & 1u);
        key[r] = k;
      });
      std::stable_sort(rorder.begin(), rorder.end(),
                       [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    }
  }
  // basis tables
  std::vector<double> phi, dphi;
  basis_tables(c->order, c->n_q, quad->bary_host, phi, dphi);
  const int npairs = nl * (nl + 1) / 2;
  std::vector<double> pairtab((size_t)c->n_q * npairs);
  for (int q = 0; q < c->n_q; ++q) {
    int p = 0;
    for (int a = 0; a < nl; ++a)
      for (int b = a; b < nl; ++b, ++p) pairtab[q * npairs + p] = phi[q * nl + a] * phi[q * nl + b];
  }

  // ---------------- device allocations and uploads
  const int64_t nqt = (int64_t)ne * c->n_q;
  const int km = c->k_max;
#define A_(p, n) \
  if (c->alloc(&c->p, (n)) < 0) return bail(KS_ERR_NOMEM)
  A_(coords, (size_t)nn * 3);
  A_(elems, (size_t)ne * nl);
  A_(edof, (size_t)ne * nl);
  A_(slot, (size_t)ne * nl * nl);
  if (r_lds) {
    A_(r_incptr, r_incptr.size());
    A_(r_inc, r_inc.size());
    A_(r_perm, r_perm.size());
    A_(load_e, (size_t)ne * nl);
  }
  A_(node2int, nn);
  A_(node2bnd, nn);
  A_(bnodes, std::max(1, c->NB));
  A_(elem_perm, ne);
  A_(absdet, ne);
  A_(gl, (size_t)ne * 12);
  A_(phi, phi.size());
  A_(dphi, dphi.size());
  A_(pairtab, pairtab.size());
  A_(phib, phi.size());
  A_(qw, c->n_q);
  A_(qbary, 4 * c->n_q);
  A_(dZ, std::max(1, c->n_atoms));
  A_(dR, std::max(3, 3 * c->n_atoms));
  A_(rowptr, N + 1);
  A_(col, c->nnz);
  A_(rowptrB, N + 1);
  A_(rorder_m, N);
  A_(colB, std::max<int64_t>(1, c->nnzB));
  A_(K, c->nnz_ext + 2);  // + 16 bytes: chunked reads of the tiled SpMM
  A_(M, c->nnz_ext);
  A_(AL, c->nnz_ext);
  A_(base, c->nnz_ext);
  A_(S, c->nnz_ext + 2);
  A_(MNL, c->nnz_ext);
  A_(diagS, N);
  A_(diagK, N);
  A_(S32, c->nnz + 8);  // 16-byte chunk reads past the end (tiled SpMM)
  A_(diagS32, N);
  A_(vext_q, nqt);
  A_(rho_l, nqt);
  A_(rho_in, nqt);
  A_(rho_out, nqt);
  A_(drho, nqt);
  A_(vh_q, nqt);
  A_(vxc_q, nqt);
  A_(exc_q, nqt);
  A_(vnl_q, nqt);
  for (int j = 0; j < o.anderson_depth; ++j) {
    A_(hist_in[j], nqt);
    A_(hist_F[j], nqt);
  }
  c->hist_alloc = o.anderson_depth;
  A_(vh_int, N);
  A_(vh_nodes, nn);
  A_(wB, std::max(1, c->NB));
  A_(load, N);
  A_(rhs, N);
  A_(mom, 64 + 256);  // moments, then reduction results (reduce_small: up to 256 values)
  A_(mpart, (size_t)moments_blocks(ne) * 16);
  A_(Pidx, (size_t)N * 4);
  A_(Pw, (size_t)N * 4);
  if (cp_ok) {
    A_(cp_uoff, cp_uoff.size());
    A_(cp_ulist, std::max<size_t>(1, cp_ulist.size()));
    A_(cp_noff, cp_noff.size());
    A_(cp_nlist, std::max<size_t>(1, cp_nlist.size()));
    A_(cp_ppoff, cp_ppoff.size());
    A_(cp_ptoff, cp_ptoff.size());
    A_(cp_gpp_ptr, cp_gpp_ptr.size());
    A_(cp_gpp_idx, std::max<size_t>(1, cp_gpp_idx.size()));
    A_(cp_gpt_ptr, cp_gpt_ptr.size());
    A_(cp_gpt_idx, std::max<size_t>(1, cp_gpt_idx.size()));
    A_(cp_pp, std::max<int64_t>(1, cp_ppoff.back()));
    A_(cp_pt, std::max<int64_t>(1, cp_ptoff.back()));
  }
  A_(Z, (size_t)N * c->mp);
  A_(Y, (size_t)N * c->mp);
  // small dense blocks: the augmented pencil (m <= mp) and the direct SCF's
  // Rayleigh-Ritz pencils (3 k <= 3 k_max)
  const int mm = std::max(c->mp, std::min(256, 3 * c->k_max));
  A_(GPP, (size_t)c->N_H * c->N_H);
  A_(GPPinv, (size_t)c->N_H * c->N_H);
  A_(FAL_PP, (size_t)c->N_H * c->N_H);
  A_(FB, (size_t)mm * mm);
  A_(FAL, (size_t)mm * mm);
  A_(FA, (size_t)mm * mm);
  A_(Ftail, (size_t)mm * mm);
  A_(Ctmp, (size_t)mm * mm);
  A_(Ttmp, (size_t)mm * mm);
  A_(U, (size_t)mm * km);
  A_(theta, mm);
  A_(eigwork, small_eig_work_doubles(mm));
  c->gwork_n = gemm_tn_work_doubles(N, mm, mm);
  A_(gwork, c->gwork_n);
  A_(coef, 64);
  A_(redpart, (size_t)1024 * 32);
  A_(einfo, 8);
  A_(eD, mm);
  A_(eV, (size_t)mm * mm);
  A_(eRot, jacobi_work_doubles(std::min(mm, 190)));
  A_(eX, (size_t)mm * mm);
  A_(eW, (size_t)mm * mm);
  A_(eT1, (size_t)mm * mm);
  A_(eT2, (size_t)mm * mm);
  A_(eS, (size_t)mm * mm);
  A_(eLam, mm);
  A_(aux1, nqt);
  A_(aux2, nqt);
  A_(Rv, (size_t)N * km);
  A_(Gv, (size_t)N * km);
  A_(dMk, (size_t)MAX_K * MAX_K);
  A_(Bv, (size_t)N * km);
  A_(Xv, (size_t)N * km);
  A_(Wv, (size_t)N * km);
  A_(PsiHat, (size_t)N * km);
  A_(PsiIn, (size_t)N * km);
  A_(Xs, (size_t)N * km);
  A_(int2nat, N);
  for (int ti = 0; ti < ks_ctx::NTILE; ++ti)
    if (c->til[ti].nblk) {
      A_(til[ti].halo_ptr, t_hptr[ti].size());
      A_(til[ti].halo_col, t_hcol[ti].size() + 8);  // 16-byte chunk reads past the end
      A_(til[ti].hself, t_hself[ti].size());
      A_(til[ti].lcol, t_lcol[ti].size() + 16);  // 16-byte chunk reads past the end
      // byte-offset runs for FP32 halo rows of k_max columns
      const int rb = km * (int)sizeof(float);
      if ((int64_t)c->til[ti].max_halo * rb < 65536 && rb % 16 == 0) {
        c->til[ti].lb_rowbytes = rb;
        A_(til[ti].lbyte, t_lcol[ti].size() + 16);
      }
      A_(til[ti].pptr, t_pptr[ti].size());
      A_(til[ti].rmeta, t_rmeta[ti].size());
    }
  A_(PsiNew, (size_t)N * km);
  A_(occ_d, 64);
  A_(scal, 128);
  A_(X32, (size_t)N * km);
  A_(counters, 16);
  {
    const int nblk = 2048;
    auto mk = [&](PCGWork &w, size_t elem, int k, int cidx) -> int {
      void *r, *p, *p2, *q, *part, *st;
      if (c->alloc(reinterpret_cast<char **>(&r), elem * N * k) < 0) return -1;
      if (c->alloc(reinterpret_cast<char **>(&p), elem * N * k) < 0) return -1;
      if (c->alloc(reinterpret_cast<char **>(&p2), elem * N * k) < 0) return -1;
      if (c->alloc(reinterpret_cast<char **>(&q), elem * N * k) < 0) return -1;
      if (c->alloc(reinterpret_cast<double **>(&part), (size_t)nblk * 3 * k) < 0) return -1;
      if (c->alloc(reinterpret_cast<char **>(&st), pcg_state_bytes(k)) < 0) return -1;
      w.R = r; w.P = p; w.P2 = p2; w.Q = q; w.part = part; w.state = st;
      w.counter = c->counters + cidx;
      w.nblk_max = nblk;
      return 0;
    };
    if (mk(c->pw64, sizeof(double), km, 0) < 0) return bail(KS_ERR_NOMEM);
    if (mk(c->pw32, sizeof(float), km, 4) < 0) return bail(KS_ERR_NOMEM);
    if (mk(c->pwP, sizeof(double), 1, 8) < 0) return bail(KS_ERR_NOMEM);
  }
#undef A_
  hipStream_t s = c->s;
#define H2D(dst, src, n) \
  if (hipMemcpyAsync(dst, src, sizeof(*(dst)) * (n), hipMemcpyHostToDevice, s) != hipSuccess) \
    return bail(fail(KS_ERR_HIP, "upload failed"))
  H2D(c->coords, mesh->coords_host, (size_t)nn * 3);
  H2D(c->elems, el, (size_t)ne * nl);
  H2D(c->edof, edof.data(), edof.size());
  H2D(c->slot, slot.data(), slot.size());
  if (r_lds) {
    H2D(c->r_incptr, r_incptr.data(), r_incptr.size());
    H2D(c->r_inc, r_inc.data(), r_inc.size());
    H2D(c->r_perm, r_perm.data(), r_perm.size());
    c->r_lds = r_lds;
  }
  H2D(c->node2int, node2int.data(), nn);
  H2D(c->node2bnd, node2bnd.data(), nn);
  if (c->NB) H2D(c->bnodes, bnodes.data(), c->NB);
  H2D(c->elem_perm, perm.data(), ne);
  H2D(c->phi, phi.data(), phi.size());
  H2D(c->dphi, dphi.data(), dphi.size());
  H2D(c->pairtab, pairtab.data(), pairtab.size());
  std::vector<double> phib_h(phi.size());
  for (int q = 0; q < c->n_q; ++q)
    for (int a = 0; a < nl; ++a) phib_h[(size_t)a * c->n_q + q] = phi[(size_t)q * nl + a];
  H2D(c->phib, phib_h.data(), phib_h.size());
  H2D(c->qw, quad->w_host, c->n_q);
  H2D(c->qbary, quad->bary_host, 4 * c->n_q);
  if (c->n_atoms) {
    H2D(c->dZ, c->hZ.data(), c->n_atoms);
    H2D(c->dR, c->hR.data(), 3 * c->n_atoms);
  }
  H2D(c->rowptr, rowptr.data(), N + 1);
  H2D(c->col, colI.data(), c->nnz);
  H2D(c->rowptrB, rowptrB.data(), N + 1);
  H2D(c->rorder_m, rorder.data(), N);
  H2D(c->int2nat, c->h_int2nat.data(), N);
  for (int ti = 0; ti < ks_ctx::NTILE; ++ti)
    if (c->til[ti].nblk) {
      H2D(c->til[ti].halo_ptr, t_hptr[ti].data(), t_hptr[ti].size());
      if (!t_hcol[ti].empty()) H2D(c->til[ti].halo_col, t_hcol[ti].data(), t_hcol[ti].size());
      H2D(c->til[ti].hself, t_hself[ti].data(), t_hself[ti].size());
      if (!t_lcol[ti].empty()) H2D(c->til[ti].lcol, t_lcol[ti].data(), t_lcol[ti].size());
      if (c->til[ti].lbyte && !t_lcol[ti].empty()) {
        const int rb = c->til[ti].lb_rowbytes;
        t_lbyte[ti].resize(t_lcol[ti].size());
        parallel_for((int64_t)t_lcol[ti].size(), [&](int64_t q) { t_lbyte[ti][q] = (uint16_t)(t_lcol[ti][q] * rb); });
        H2D(c->til[ti].lbyte, t_lbyte[ti].data(), t_lbyte[ti].size());
      }
      H2D(c->til[ti].pptr, t_pptr[ti].data(), t_pptr[ti].size());
      H2D(c->til[ti].rmeta, t_rmeta[ti].data(), t_rmeta[ti].size());
    }
  {
    c->rorder = nullptr;
    c->ng64 = c->ng32 = c->ngP = 0;
    // SpMM phase kernel before any autotuning: halo tiles of 85 rows with
    // 1024 threads (FP64), 85 rows with 512 threads (FP32), 128 rows with 256
    // threads (Poisson, one column)
    auto tile_of = [&](int rows, int tb) {
      const int i = tile_index(rows);
      return i >= 0 ? NTB * i + (tb == 1024 ? 2 : (tb == 512 ? 1 : 0)) : -1;
    };
    c->tile64 = tile_of(85, 1024);
    c->tile32 = tile_of(85, 512);
    c->tileP = tile_of(128, 256);
    apply_tiles(c);
  }
  H2D(c->colB, colB.data(), colB.size());
  H2D(c->Pidx, Pidx.data(), Pidx.size());
  H2D(c->Pw, Pw.data(), Pw.size());
  if (cp_ok) {
    H2D(c->cp_uoff, cp_uoff.data(), cp_uoff.size());
    if (!cp_ulist.empty()) H2D(c->cp_ulist, cp_ulist.data(), cp_ulist.size());
    H2D(c->cp_noff, cp_noff.data(), cp_noff.size());
    if (!cp_nlist.empty()) H2D(c->cp_nlist, cp_nlist.data(), cp_nlist.size());
    H2D(c->cp_ppoff, cp_ppoff.data(), cp_ppoff.size());
    H2D(c->cp_ptoff, cp_ptoff.data(), cp_ptoff.size());
    H2D(c->cp_gpp_ptr, cp_gpp_ptr.data(), cp_gpp_ptr.size());
    if (!cp_gpp_idx.empty()) H2D(c->cp_gpp_idx, cp_gpp_idx.data(), cp_gpp_idx.size());
    H2D(c->cp_gpt_ptr, cp_gpt_ptr.data(), cp_gpt_ptr.size());
    if (!cp_gpt_idx.empty()) H2D(c->cp_gpt_idx, cp_gpt_idx.data(), cp_gpt_idx.size());
    c->cp_ok = 1;
    c->cp_nblk = cp_nblk;
    c->cp_ldt = cp_ldt;
    c->cp_ldo = cp_ldo;
  }
#undef H2D
  if (hipMemsetAsync(c->counters, 0, 16 * sizeof(unsigned int), s) != hipSuccess)
    return bail(fail(KS_ERR_HIP, "memset failed"));
  if (hipMemsetAsync(c->einfo, 0, 8 * sizeof(int), s) != hipSuccess)
    return bail(fail(KS_ERR_HIP, "memset failed"));
  // ---------------- a1: geometry, K, M, V_ext, M[V_ext]
  launch_geometry(c->coords, c->elems, nl, ne, c->absdet, c->gl, c->einfo, s);
  int bad = 0;
  if (hipMemcpyAsync(&bad, c->einfo, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bail(fail(KS_ERR_HIP, "geometry kernel failed"));
  if (bad) return bail(fail(KS_ERR_MESH, "mesh has " + std::to_string(bad) + " element(s) with det J <= 0"));
  launch_fill(c->nnz_ext, 0.0, c->K, s);
  launch_fill(c->nnz_ext, 0.0, c->M, s);
  for (int k = 0; k < ncol; ++k) {
    const int a = c->colour_off[k], b = c->colour_off[k + 1];
    launch_assemble_KM(c->elem_perm + a, b - a, nl, c->n_q, c->slot, c->absdet, c->gl, c->phi,
                       c->dphi, c->qw, c->K, c->M, s);
  }
  launch_vext(c->coords, c->elems, nl, ne, c->n_q, c->qbary, c->n_atoms, c->dZ, c->dR, c->vext_q, s);
  dbg(c, "K", c->K, c->nnz_ext);
  dbg(c, "M", c->M, c->nnz_ext);
  dbg(c, "vext_q", c->vext_q, (int64_t)ne * c->n_q);
  assemble_potential_all(c, c->vext_q, c->AL);
  launch_axpby(c->nnz_ext, 0.5, c->K, 1.0, c->AL, s);                  // A^L = K/2 + M[V_ext]
  launch_combine3(c->nnz_ext, 1.0, c->AL, c->mu, c->M, 0.0, nullptr, c->base, s);  // + mu M
  launch_extract_diag(N, c->rowptr, c->col, c->K, c->diagK, s);
  // ---------------- coarse blocks: dense P in Z, G_PP = P^T M P, P^T A^L P
  launch_fill((int64_t)N * c->mp, 0.0, c->Z, s);
  launch_dense_P(N, c->Pidx, c->Pw, c->N_H, c->Z, c->mp, s);
  dbg(c, "AL", c->AL, c->nnz_ext);
  dbg(c, "Z(P dense)", c->Z, (int64_t)N * c->mp);
  spmm_cols(c, c->M, c->Z, c->mp, c->Y, c->mp, c->N_H);
  dbg(c, "Y = M P", c->Y, (int64_t)N * c->mp);
  launch_gemm_tn(N, c->N_H, c->N_H, c->Z, c->mp, c->Y, c->mp, c->GPP, c->N_H, c->gwork, c->gwork_n, s);
  dbg(c, "G_PP", c->GPP, (int64_t)c->N_H * c->N_H);
  spmm_cols(c, c->AL, c->Z, c->mp, c->Y, c->mp, c->N_H);
  launch_gemm_tn(N, c->N_H, c->N_H, c->Z, c->mp, c->Y, c->mp, c->FAL_PP, c->N_H, c->gwork, c->gwork_n,
                 s);
  {
    // G_PP^{-1} on the host (N_H <= 255): Gauss-Jordan with partial pivoting
    const int n = c->N_H;
    std::vector<double> G((size_t)n * n), I((size_t)n * n, 0.0);
    if (hipMemcpyAsync(G.data(), c->GPP, sizeof(double) * n * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return bail(fail(KS_ERR_HIP, "coarse mass matrix download failed"));
    for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
    for (int p = 0; p < n; ++p) {
      int piv = p;
      for (int r = p + 1; r < n; ++r)
        if (std::fabs(G[(size_t)r * n + p]) > std::fabs(G[(size_t)piv * n + p])) piv = r;
      if (!(std::fabs(G[(size_t)piv * n + p]) > 0.0)) {
        if (debug_on()) break;
        return bail(fail(KS_ERR_MESH, "coarse space is rank deficient on this mesh (mesh too coarse for n_H)"));
      }
      if (piv != p)
        for (int j = 0; j < n; ++j) {
          std::swap(G[(size_t)p * n + j], G[(size_t)piv * n + j]);
          std::swap(I[(size_t)p * n + j], I[(size_t)piv * n + j]);
        }
      const double d = 1.0 / G[(size_t)p * n + p];
      for (int j = 0; j < n; ++j) {
        G[(size_t)p * n + j] *= d;
        I[(size_t)p * n + j] *= d;
      }
      for (int r = 0; r < n; ++r) {
        if (r == p) continue;
        const double f = G[(size_t)r * n + p];
        if (f == 0.0) continue;
        for (int j = 0; j < n; ++j) {
          G[(size_t)r * n + j] -= f * G[(size_t)p * n + j];
          I[(size_t)r * n + j] -= f * I[(size_t)p * n + j];
        }
      }
    }
    if (hipMemcpyAsync(c->GPPinv, I.data(), sizeof(double) * n * n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return bail(fail(KS_ERR_HIP, "upload failed"));
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess)
    return bail(fail(KS_ERR_HIP, "event creation failed"));
  // multigrid hierarchy for the Hartree Poisson solves
  {
    if (c->opt.hartree_mode != KS_HARTREE_OFF) {
      std::vector<double> Kh(c->nnz), X((size_t)N * 3);
      if (hipMemcpyAsync(Kh.data(), c->K, sizeof(double) * c->nnz, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return bail(fail(KS_ERR_HIP, "download failed"));
      for (int r = 0; r < N; ++r)
        for (int d = 0; d < 3; ++d) X[3 * (size_t)r + d] = mesh->coords_host[3 * (int64_t)interior_nodes[r] + d];
      // P2: the first coarse level is P1 on the mesh's own vertices (nested:
      // vertices inject, edge midpoints average their two ends, boundary
      // vertices drop out), then uniform lattices of half the fine cells per
      // side and coarser; P1: uniform lattices from half the fine cells
      const int side = (int)std::lround(std::cbrt((double)nn));
      const int nfine = std::max(1, (side - 1) / c->order);
      const int n1 = nfine / 2;
      MGFirst first;
      if (c->order == 2) {
        std::vector<int32_t> vidx(nn, -1), e0(nn, -1), e1(nn, -1);
        static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
        std::vector<char> isv(nn, 0);
        for (int64_t e = 0; e < ne; ++e) {
          for (int a = 0; a < 4; ++a) isv[el[e * nl + a]] = 1;
          for (int t = 0; t < 6; ++t) {
            const int m = el[e * nl + 4 + t];
            e0[m] = el[e * nl + E[t][0]];
            e1[m] = el[e * nl + E[t][1]];
          }
        }
        for (int r = 0; r < N; ++r)  // coarse unknowns in the fine storage order
          if (isv[interior_nodes[r]]) vidx[interior_nodes[r]] = first.nc++;
        first.Pi.assign((size_t)N * 4, -1);
        first.Pw.assign((size_t)N * 4, 0.0);
        first.X.resize((size_t)first.nc * 3);
        bool ok = first.nc > 0;
        for (int r = 0; r < N && ok; ++r) {
          const int nd = interior_nodes[r];
          if (vidx[nd] >= 0) {
            first.Pi[4 * (size_t)r] = vidx[nd];
            first.Pw[4 * (size_t)r] = 1.0;
            for (int d = 0; d < 3; ++d) first.X[3 * (size_t)vidx[nd] + d] = mesh->coords_host[3 * (int64_t)nd + d];
          } else if (e0[nd] >= 0) {
            int t = 0;
            for (const int v : {e0[nd], e1[nd]})
              if (vidx[v] >= 0) {
                first.Pi[4 * (size_t)r + t] = vidx[v];
                first.Pw[4 * (size_t)r + t++] = 0.5;
              }
          } else {
            ok = false;  // a node that is neither vertex nor edge midpoint
          }
        }
        if (!ok) first = MGFirst();
      }
      c->mg = mg_build(N, c->rowptr, c->col, c->K, c->pwP.til, c->pwP.til_tb, rowptr, colI, Kh, X, c->L,
                       c->order == 2 && first.nc > 0 ? n1 : (c->order == 2 ? nfine : n1), s,
                       first.nc > 0 ? &first : nullptr);
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(KS_ERR_HIP, "setup failed"));
  *out = c;
  return KS_OK;
}

extern "C" int ks_debug_buffer(ks_ctx *c, const char *name, double *dst, int64_t n) {
  if (!c || !name || !dst) return fail(KS_ERR_ARG, "null argument");
  struct { const char *n; const double *p; int64_t size; } tab[] = {
      {"GPP", c->GPP, (int64_t)c->N_H * c->N_H}, {"FAL_PP", c->FAL_PP, (int64_t)c->N_H * c->N_H},
      {"Z", c->Z, (int64_t)c->N * c->mp}, {"Y", c->Y, (int64_t)c->N * c->mp},
      {"FB", c->FB, (int64_t)c->mp * c->mp}, {"FAL", c->FAL, (int64_t)c->mp * c->mp},
      {"FA", c->FA, (int64_t)c->mp * c->mp}, {"U", c->U, (int64_t)c->mp * c->k_max},
      {"rho_in", c->rho_in, (int64_t)c->n_e * c->n_q}, {"vh_q", c->vh_q, (int64_t)c->n_e * c->n_q},
      {"wB", c->wB, (int64_t)c->NB}, {"mom", c->mom, 16}, {"S", c->S, (int64_t)c->nnz},
      // LOBPCG blocks of the direct SCF ([N][3 k] storage order; Gram matrices m x m)
      {"dS", c->dS, c->d_k ? (int64_t)c->N * 3 * c->d_k : 0}, {"dHS", c->dHS, c->d_k ? (int64_t)c->N * 3 * c->d_k : 0},
      {"dMS", c->dMS, c->d_k ? (int64_t)c->N * 3 * c->d_k : 0}, {"dGM", c->dGM, (int64_t)9 * c->d_k * c->d_k},
      {"dGH", c->dGH, (int64_t)9 * c->d_k * c->d_k}};
  // "S32": the FP32 operator copy, nnz floats packed into ceil(nnz / 2) doubles
  if (std::strcmp(name, "S32") == 0) {
    if (!c->have_S32) return fail(KS_ERR_STATE, "no FP32 operator copy");
    if (n < ((int64_t)c->nnz + 1) / 2) return fail(KS_ERR_ARG, "buffer smaller than requested");
    HIPCHK(hipMemcpyAsync(dst, c->S32, sizeof(float) * c->nnz, hipMemcpyDeviceToDevice, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    return KS_OK;
  }
  for (auto &t : tab)
    if (std::strcmp(t.n, name) == 0) {
      if (n > t.size || !t.p) return fail(KS_ERR_ARG, "buffer smaller than requested");
      const bool rows = (t.p == c->Z || t.p == c->Y) && n == t.size;
      if (rows) launch_rows_to_api(c->N, c->mp, t.p, dst, c->int2nat, c->s);  // API row order
      else HIPCHK(hipMemcpyAsync(dst, t.p, sizeof(double) * n, hipMemcpyDeviceToDevice, c->s));
      HIPCHK(hipStreamSynchronize(c->s));
      return KS_OK;
    }
  return fail(KS_ERR_ARG, std::string("unknown buffer ") + name);
}

// fp32 operator copy on demand
static void ensure_s32(ks_ctx *c) {
  if (!c->have_S32) {
    launch_to_float(c->nnz, c->S, c->S32, c->s);
    launch_to_float(c->N, c->diagS, c->diagS32, c->s);
    c->have_S32 = true;
  }
}

static int time_phase(ks_ctx *c, int which, int k, int reps, int ng, float *ms) {
  if (which >= 0 && which <= 2)
    return pcg_time_phase<double>(c->N, k, which, c->rowptr, c->col, c->S, c->rorder, c->diagS,
                                  c->Xv, c->pw64, reps, ms, c->s, ng);
  if (which >= 3 && which <= 5) {
    ensure_s32(c);
    return pcg_time_phase<float>(c->N, k, which - 3, c->rowptr, c->col, c->S32, c->rorder,
                                 c->diagS32, c->X32, c->pw32, reps, ms, c->s, ng);
  }
  return pcg_time_phase<double>(c->N, 1, 0, c->rowptr, c->col, c->K, c->rorder, c->diagK, c->vh_int,
                                c->pwP, reps, ms, c->s, ng);
}

extern "C" int ks_spmm_config(const ks_ctx *c, int32_t *out_host) {  // 9 values
  if (!c || !out_host) return fail(KS_ERR_ARG, "null argument");
  out_host[0] = c->ng64;
  out_host[1] = c->ng32;
  out_host[2] = c->ngP;
  const PCGWork *ws[3] = {&c->pw64, &c->pw32, &c->pwP};
  for (int w = 0; w < 3; ++w) out_host[3 + w] = ws[w]->til ? ws[w]->til->BR : 0;
  for (int w = 0; w < 3; ++w) out_host[6 + w] = ws[w]->til ? ws[w]->til_tb : 0;
  return KS_OK;
}

static void project_full(ks_ctx *c, const double *H, int m, double *F);
static void project_nl(ks_ctx *c, const double *H, int k, double *F);

// mean duration of `reps` back-to-back runs of one of the other hot-path
// operations (see ks_time_kernel), on the context's current state
static int time_op(ks_ctx *c, int which, int k, int reps, float *ms) {
  hipStream_t s = c->s;
  const int64_t nqt = (int64_t)c->n_e * c->n_q;
  const int m = c->N_H + k;
  auto op = [&]() {
    switch (which) {
      case 7:  // potential matrix M[V_nl] over all colours (a4)
        assemble_potential_all(c, c->vnl_q, c->MNL);
        break;
      case 8:  // density at the quadrature points (a2)
        launch_density(c->edof, c->n_loc, c->n_e, c->n_q, c->phi, c->PsiIn, k, k, c->occ_d, c->aux1, s);
        break;
      case 9:  // LDA energy density and potential (a2)
        launch_xc(nqt, c->rho_l, c->opt.xc_mode == KS_XC_NONE ? KS_XC_X_PZ81 : c->opt.xc_mode, c->aux1, c->aux2, s);
        break;
      case 10:  // projection F = Z^T (M[V_nl] Z) as the inner iteration runs it (a6/a7)
        project_nl(c, c->MNL, k, c->Ctmp);
        break;
      case 11:  // its tall-skinny GEMM T^T (H T) alone (FP64 MFMA)
        launch_gemm_tn_sym(c->N, k, c->Z + c->N_H, c->mp, c->Wv, k, c->Ttmp, k, c->gwork, s);
        break;
      default:  // 12: the dense projection over all m columns of Z (SpMM + MFMA GEMM)
        project_full(c, c->MNL, m, c->Ctmp);
        break;
    }
  };
  op();  // warm
  HIPCHK(hipEventRecord(c->ev0, s));
  for (int r = 0; r < reps; ++r) op();
  HIPCHK(hipEventRecord(c->ev1, s));
  HIPCHK(hipEventSynchronize(c->ev1));
  float t = 0.f;
  HIPCHK(hipEventElapsedTime(&t, c->ev0, c->ev1));
  *ms = t / reps;
  c->have_step = false;  // MNL / work buffers were overwritten
  return KS_OK;
}

extern "C" int ks_time_kernel(ks_ctx *c, int32_t which, int32_t k, int32_t reps, double *ms_host) {
  if (!c || !ms_host) return fail(KS_ERR_ARG, "null argument");
  if (reps < 1 || k < 1 || k > c->k_max) return fail(KS_ERR_ARG, "bad k or reps");
  if (!c->have_S) return fail(KS_ERR_STATE, "no operator assembled");
  if (which < 0 || which > 12) return fail(KS_ERR_ARG, "which must be 0..12");
  if (which >= 7) {
    float ms = 0.f;
    TRY(time_op(c, which, k, reps, &ms));
    *ms_host = ms;
    return KS_OK;
  }
  const int ng = (which <= 2) ? c->ng64 : (which <= 5 ? c->ng32 : c->ngP);
  float ms = 0.f;
  if (time_phase(c, which, k, reps, ng, &ms) < 0) return fail(KS_ERR_HIP, "timing launch failed");
  *ms_host = ms;
  return KS_OK;
}

// Autotuner: times the SpMM phase of the block PCG (FP64, FP32) and of the
// Poisson solve on the current operator for every kernel candidate -- the
// row kernel with NG = 1, 2, 4, 8 lanes per row and the LDS-staged halo
// kernel with row blocks of 32, 64, 128, 256 rows -- and keeps the fastest
// for this context.
extern "C" int ks_autotune(ks_ctx *c, int32_t k, int32_t reps, double *report_host) {
  if (!c) return fail(KS_ERR_ARG, "null context");
  if (k < 1 || k > c->k_max || reps < 1) return fail(KS_ERR_ARG, "bad k or reps");
  if (!c->have_S) return fail(KS_ERR_STATE, "no operator assembled");
  const int ngs[4] = {1, 2, 4, 8};
  double t_row[3][4], t_til[3][NTB * ks_ctx::NTILE];
  int best_ng[3] = {1, 1, 8}, best_tile[3] = {-1, -1, -1};
  PCGWork *ws[3] = {&c->pw64, &c->pw32, &c->pwP};
  c->rorder = nullptr;
  for (int w = 0; w < 3; ++w) {
    const int which = w == 0 ? 0 : (w == 1 ? 3 : 6);
    const int kk = w == 2 ? 1 : k;
    double bt = 1e300;
    const Tiling *keep = ws[w]->til;
    const int keep_db = ws[w]->til_tb;
    ws[w]->til = nullptr;
    // every candidate's q = S p on a fixed p is compared with the first row
    // kernel's; one that differs by more than rounding is never chosen
    const bool f32 = w == 1;
    if (which >= 3) ensure_s32(c);
    const double dev_tol = f32 ? 1e-5 : 1e-12;
    void *ref = nullptr;
    if (hipMalloc(&ref, (f32 ? sizeof(float) : sizeof(double)) * (size_t)c->N * kk) != hipSuccess)
      return fail(KS_ERR_NOMEM, "autotune: hipMalloc failed");
    auto check = [&](int mode, double *dev) {
      return f32 ? pcg_phase_check<float>(*ws[w], c->N, kk, mode, ref, dev, c->s)
                 : pcg_phase_check<double>(*ws[w], c->N, kk, mode, ref, dev, c->s);
    };
    auto restore = [&]() {
      ws[w]->til = keep;
      ws[w]->til_tb = keep_db;
      (void)hipFree(ref);
    };
    double dev = 0.0;
    if (check(0, &dev) < 0) {
      restore();
      return fail(KS_ERR_HIP, "autotune check failed");
    }
    for (int i = 0; i < 4; ++i) {
      float ms = 0.f;
      if (time_phase(c, which, kk, reps, ngs[i], &ms) < 0 || check(i == 0 ? 1 : 2, &dev) < 0) {
        restore();
        return fail(KS_ERR_HIP, "autotune timing failed");
      }
      if (i > 0 && !(dev <= dev_tol)) {
        t_row[w][i] = -2.0;  // wrong result: never chosen
        continue;
      }
      t_row[w][i] = ms;
      if (ms < bt) {
        bt = ms;
        best_ng[w] = ngs[i];
        best_tile[w] = -1;
      }
    }
    for (int code = 0; code < NTB * ks_ctx::NTILE; ++code) {
      const int i = code / NTB;
      t_til[w][code] = -1.0;
      if (!c->til[i].nblk) continue;
      ws[w]->til = &c->til[i];
      ws[w]->til_tb = TILE_TB[code % NTB];
      float ms = 0.f;
      const int r = time_phase(c, which, kk, reps, 0, &ms);
      if (r == -3) continue;  // does not fit in LDS for this shape
      if (r < 0 || check(2, &dev) < 0) {
        restore();
        return fail(KS_ERR_HIP, "autotune timing failed");
      }
      if (!(dev <= dev_tol)) {
        t_til[w][code] = -2.0;  // wrong result: never chosen
        continue;
      }
      t_til[w][code] = ms;
      if (ms < bt) {
        bt = ms;
        best_tile[w] = code;
      }
    }
    restore();
    // keep the configuration in use unless another is more than 3% faster:
    // closer timings are within the run-to-run noise
    const int cur = w == 0 ? c->tile64 : (w == 1 ? c->tile32 : c->tileP);
    if (cur >= 0 && t_til[w][cur] > 0.0 && t_til[w][cur] <= 1.03 * bt) best_tile[w] = cur;
  }
  c->ng64 = best_ng[0];
  c->ng32 = best_ng[1];
  c->ngP = best_ng[2];
  c->tile64 = best_tile[0];
  c->tile32 = best_tile[1];
  c->tileP = best_tile[2];
  apply_tiles(c);
  if (report_host) {
    for (int w = 0; w < 3; ++w) {
      report_host[w] = best_ng[w];
      report_host[3 + w] = best_tile[w] >= 0 ? TILE_BR[best_tile[w] / NTB] : 0;
      report_host[6 + w] = best_tile[w] >= 0 ? TILE_TB[best_tile[w] % NTB] : 0;
      for (int i = 0; i < 4; ++i) report_host[9 + w * 4 + i] = t_row[w][i];
      for (int i = 0; i < NTB * ks_ctx::NTILE; ++i) report_host[21 + w * NTB * ks_ctx::NTILE + i] = t_til[w][i];
    }
  }
  return KS_OK;
}

// ------------------------------------------------------- autotune cache
// One text line per tuned solver: arch order log2N nnz/row k precision ng
// tile_rows tile_threads ms.  The key is everything before ng; the last
// matching line wins; lines that do not parse are skipped.
namespace {
struct TuneKey {
  std::string arch;
  int order = 0, log2n = 0, nnz_row = 0, k = 0;
};
const char *const TUNE_PREC[3] = {"fp64", "fp32", "poisson"};

bool tune_key(const ks_ctx *c, int k, TuneKey *key) {
  int dev = 0;
  if (hipStreamGetDevice(c->s, &dev) != hipSuccess) return false;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return false;
  key->arch.clear();
  for (const char *q = p.gcnArchName; *q && key->arch.size() < 200; ++q)
    key->arch.push_back((*q == ' ' || *q == '\t') ? '_' : *q);
  if (key->arch.empty()) key->arch = "unknown";
  key->order = c->order;
  key->log2n = 0;
  while ((2LL << key->log2n) <= (long long)c->N) ++key->log2n;
  key->nnz_row = (int)((c->nnz + c->N / 2) / std::max(c->N, 1));
  key->k = k;
  return true;
}

struct TuneEntry {
  bool found = false;
  int ng = 0, rows = 0, threads = 0;
};

// last entry of each precision for this key (k = 1 for the Poisson solver)
void tune_lookup(const char *path, const TuneKey &key, TuneEntry e[3]) {
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char line[512], arch[256], prec[32];
  while (std::fgets(line, sizeof line, f)) {
    int order, log2n, nnz_row, k, ng, rows, threads;
    double ms;
    if (line[0] == '#') continue;
    if (std::sscanf(line, "%255s %d %d %d %d %31s %d %d %d %lf", arch, &order, &log2n, &nnz_row, &k,
                    prec, &ng, &rows, &threads, &ms) != 10)
      continue;
    if (key.arch != arch || order != key.order || log2n != key.log2n || nnz_row != key.nnz_row) continue;
    for (int w = 0; w < 3; ++w)
      if (!std::strcmp(prec, TUNE_PREC[w]) && k == (w == 2 ? 1 : key.k)) e[w] = {true, ng, rows, threads};
  }
  std::fclose(f);
}
}  // namespace

// Is (ng, code) usable for solver w with kk columns: the tiling exists and
// fits, and q = S p on a fixed p agrees with the one-lane row kernel's (the
// tolerances of ks_autotune).
static int check_choice(ks_ctx *c, int w, int kk, int ng, int code, bool *ok) {
  PCGWork *ws[3] = {&c->pw64, &c->pw32, &c->pwP};
  PCGWork &pw = *ws[w];
  const int which = w == 0 ? 0 : (w == 1 ? 3 : 6);
  const bool f32 = w == 1;
  *ok = false;
  if (code >= 0 && !c->til[code / NTB].nblk) return KS_OK;
  if (f32) ensure_s32(c);
  void *ref = nullptr;
  if (hipMalloc(&ref, (f32 ? sizeof(float) : sizeof(double)) * (size_t)c->N * kk) != hipSuccess)
    return fail(KS_ERR_NOMEM, "autotune cache: hipMalloc failed");
  const Tiling *keep = pw.til;
  const int keep_tb = pw.til_tb;
  auto check = [&](int mode, double *dev) {
    return f32 ? pcg_phase_check<float>(pw, c->N, kk, mode, ref, dev, c->s)
               : pcg_phase_check<double>(pw, c->N, kk, mode, ref, dev, c->s);
  };
  double dev = 0.0;
  float ms = 0.f;
  int r = check(0, &dev);
  pw.til = nullptr;
  if (r == 0) r = time_phase(c, which, kk, 1, 1, &ms);
  if (r == 0) r = check(1, &dev);
  if (r == 0) {
    pw.til = code >= 0 ? &c->til[code / NTB] : nullptr;
    pw.til_tb = TILE_TB[code >= 0 ? code % NTB : 0];
    r = time_phase(c, which, kk, 1, ng, &ms);
    if (r == 0) {
      r = check(2, &dev);
      *ok = r == 0 && dev <= (f32 ? 1e-5 : 1e-12);
    } else if (r == -3) {
      r = 0;  // does not fit in LDS for this shape
    }
  }
  pw.til = keep;
  pw.til_tb = keep_tb;
  (void)hipFree(ref);
  return r < 0 ? fail(KS_ERR_HIP, "autotune cache: check launch failed") : KS_OK;
}

extern "C" int ks_autotune_cached(ks_ctx *c, int32_t k, int32_t reps, const char *path, int32_t *hit_host) {
  if (!c || !path || !*path) return fail(KS_ERR_ARG, "null context or cache path");
  if (k < 1 || k > c->k_max || reps < 1) return fail(KS_ERR_ARG, "bad k or reps");
  if (!c->have_S) return fail(KS_ERR_STATE, "no operator assembled");
  if (hit_host) *hit_host = 0;
  TuneKey key;
  if (!tune_key(c, k, &key)) return fail(KS_ERR_HIP, "autotune cache: device query failed");
  TuneEntry e[3];
  tune_lookup(path, key, e);
  bool hit = e[0].found && e[1].found && e[2].found;
  int ng[3] = {1, 1, 1}, code[3] = {-1, -1, -1};
  for (int w = 0; hit && w < 3; ++w) {
    const int ti = e[w].rows ? tile_index(e[w].rows) : -1;
    const int tb = e[w].threads == 256 ? 0 : (e[w].threads == 512 ? 1 : (e[w].threads == 1024 ? 2 : -1));
    const bool ng_ok = e[w].ng == 1 || e[w].ng == 2 || e[w].ng == 4 || e[w].ng == 8;
    if (!ng_ok || (e[w].rows && (ti < 0 || tb < 0))) {
      hit = false;
      break;
    }
    ng[w] = e[w].ng;
    code[w] = e[w].rows ? NTB * ti + tb : -1;
    bool ok = false;
    TRY(check_choice(c, w, w == 2 ? 1 : k, ng[w], code[w], &ok));
    hit = ok;
  }
  if (hit) {
    c->rorder = nullptr;
    c->ng64 = ng[0];
    c->ng32 = ng[1];
    c->ngP = ng[2];
    c->tile64 = code[0];
    c->tile32 = code[1];
    c->tileP = code[2];
    apply_tiles(c);
    if (hit_host) *hit_host = 1;
    return KS_OK;
  }
  std::vector<double> rep(21 + 3 * NTB * ks_ctx::NTILE);
  TRY(ks_autotune(c, k, reps, rep.data()));
  std::string text;
  for (int w = 0; w < 3; ++w) {
    const int g = (int)rep[w], rows = (int)rep[3 + w], tb = (int)rep[6 + w];
    int gi = 0;
    while (gi < 3 && (1 << gi) != g) ++gi;
    const double ms = rows ? rep[21 + w * NTB * ks_ctx::NTILE + NTB * tile_index(rows) +
                                 (tb == 256 ? 0 : (tb == 512 ? 1 : 2))]
                           : rep[9 + w * 4 + gi];
    char line[512];
    std::snprintf(line, sizeof line, "%s %d %d %d %d %s %d %d %d %.6g\n", key.arch.c_str(), key.order,
                  key.log2n, key.nnz_row, w == 2 ? 1 : k, TUNE_PREC[w], g, rows, tb, ms);
    text += line;
  }
  // one append of all three lines, so that concurrent writers do not
  // interleave within an entry
  FILE *f = std::fopen(path, "a");
  const bool wrote = f && std::fwrite(text.data(), 1, text.size(), f) == text.size();
  const bool closed = f && std::fclose(f) == 0;
  if (!wrote || !closed) return fail(KS_ERR_ARG, "autotune cache: cannot append to the cache file");
  return KS_OK;
}

// ---------------------------------------------------- external potential
// Recompute everything that depends on V_ext: A^L, A^L + mu M and P^T A^L P.
static int refresh_external(ks_ctx *c) {
  hipStream_t s = c->s;
  assemble_potential_all(c, c->vext_q, c->AL);
  launch_axpby(c->nnz_ext, 0.5, c->K, 1.0, c->AL, s);
  launch_combine3(c->nnz_ext, 1.0, c->AL, c->mu, c->M, 0.0, nullptr, c->base, s);
  spmm_cols(c, c->AL, c->Z, c->mp, c->Y, c->mp, c->N_H);
  launch_gemm_tn(c->N, c->N_H, c->N_H, c->Z, c->mp, c->Y, c->mp, c->FAL_PP, c->N_H, c->gwork,
                 c->gwork_n, s);
  c->have_S = c->have_S32 = c->have_step = false;
  HIPCHK(hipStreamSynchronize(s));
  return KS_OK;
}

extern "C" int ks_set_external(ks_ctx *c, const double *vext_q, const double *R_host) {
  if (!c) return fail(KS_ERR_ARG, "null context");
  if (vext_q && R_host) return fail(KS_ERR_ARG, "give either vext_q or R_host");
  if (R_host) {
    if (c->n_atoms == 0) return fail(KS_ERR_ARG, "no nuclei to move");
    c->hR.assign(R_host, R_host + 3 * c->n_atoms);
    HIPCHK(hipMemcpyAsync(c->dR, c->hR.data(), sizeof(double) * 3 * c->n_atoms, hipMemcpyHostToDevice, c->s));
    c->E_nn = 0.0;
    for (int j = 0; j < c->n_atoms; ++j)
      for (int k = 0; k < j; ++k) {
        double dx = c->hR[3 * j] - c->hR[3 * k], dy = c->hR[3 * j + 1] - c->hR[3 * k + 1],
               dz = c->hR[3 * j + 2] - c->hR[3 * k + 2];
        c->E_nn += c->hZ[j] * c->hZ[k] / std::sqrt(dx * dx + dy * dy + dz * dz);
      }
    launch_vext(c->coords, c->elems, c->n_loc, c->n_e, c->n_q, c->qbary, c->n_atoms, c->dZ, c->dR,
                c->vext_q, c->s);
    c->vext_atomic = true;
  } else if (vext_q) {
    HIPCHK(hipMemcpyAsync(c->vext_q, vext_q, sizeof(double) * c->n_e * c->n_q, hipMemcpyDeviceToDevice, c->s));
    c->vext_atomic = false;
  } else {
    return fail(KS_ERR_ARG, "nothing to set");
  }
  return refresh_external(c);
}

// ------------------------------------------------------ step energy E_KS
extern "C" int ks_step_energy(ks_ctx *c, double *out) {
  if (!c || !out) return fail(KS_ERR_ARG, "null argument");
  if (!c->have_step) return fail(KS_ERR_STATE, "no ks_scf_step result to evaluate");
  hipStream_t s = c->s;
  const int k = c->last_k, N = c->N;
  const int64_t nqt = (int64_t)c->n_e * c->n_q;
  // kinetic: 1/2 sum_i f_i psi_i^T K psi_i
  spmm_op(c, c->K, c->PsiNew, k, c->Wv, nullptr);
  std::vector<double> kd(k);
  const int nb = launch_coldots(N, k, c->PsiNew, c->Wv, c->redpart, s);
  TRY(reduce_small(c, c->redpart, nb, k, kd.data()));
  double kin = 0.0;
  for (int j = 0; j < k; ++j) kin += 0.5 * c->last_occ[j] * kd[j];
  double eh = 0.0, exc = 0.0, ext = 0.0;
  {
    const double *a[1] = {c->vext_q};
    const double *b[1] = {c->rho_out};
    TRY(weighted_dots(c, 1, a, b, &ext));
  }
  if (c->opt.hartree_mode != KS_HARTREE_OFF) {
    // E_H^step = 1/2 <rho, V_H[rho]> + 1/2 <rho - rho^l, V_bc>, w_D frozen
    int it = 0;
    if (hartree_solve(c, c->rho_out, &it) < 0) return KS_ERR_BREAKDOWN;
    HIPCHK(hipMemcpyAsync(c->aux1, c->vh_q, sizeof(double) * nqt, hipMemcpyDeviceToDevice, s));
    launch_fill(nqt, 0.0, c->aux2, s);
    if (hartree_solve(c, c->aux2, &it) < 0) return KS_ERR_BREAKDOWN;  // V_bc
    launch_combine3(nqt, 1.0, c->rho_out, -1.0, c->rho_l, 0.0, nullptr, c->aux2, s);
    const double *a[2] = {c->aux1, c->vh_q};
    const double *b[2] = {c->rho_out, c->aux2};
    double e2[2];
    TRY(weighted_dots(c, 2, a, b, e2));
    eh = 0.5 * e2[0] + 0.5 * e2[1];
    c->vh_warm = false;
  }
  if (c->opt.xc_mode != KS_XC_NONE) {
    launch_xc(nqt, c->rho_out, c->opt.xc_mode, c->aux2, c->aux1, s);
    const double *a[1] = {c->aux2};
    const double *b[1] = {c->rho_out};
    TRY(weighted_dots(c, 1, a, b, &exc));
  }
  out[1] = kin;
  out[2] = ext;
  out[3] = eh;
  out[4] = exc;
  out[5] = c->E_nn;
  out[0] = kin + ext + eh + exc + c->E_nn;
  return KS_OK;
}

// --------------------------------------------------------------- adjoint
// mesh-vertex derivative of the step (ks_step_backward_mesh): the output
// dE/dX and optionally the node motion that follows the nuclei
struct MeshReq {
  const double *motion = nullptr;  // device [n_nodes][n_atoms] or null
  double *dEdX = nullptr;          // device [n_nodes][3]
};

// per node the records 4 e + v of the elements that have it as vertex v,
// in element order (built once per context)
static int vertex_incidence(ks_ctx *c) {
  if (c->vinc_ptr) return KS_OK;
  const int ne = c->n_e, nl = c->n_loc, nn = c->n_nodes;
  std::vector<int32_t> el((size_t)ne * nl);
  HIPCHK(hipMemcpyAsync(el.data(), c->elems, sizeof(int32_t) * el.size(), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  std::vector<int32_t> ptr((size_t)nn + 1, 0);
  for (int e = 0; e < ne; ++e)
    for (int v = 0; v < 4; ++v) ptr[(size_t)el[(size_t)e * nl + v] + 1]++;
  for (int n = 0; n < nn; ++n) ptr[n + 1] += ptr[n];
  std::vector<int32_t> rec((size_t)std::max(ptr[nn], 1)), pos(ptr.begin(), ptr.end() - 1);
  for (int e = 0; e < ne; ++e)
    for (int v = 0; v < 4; ++v) rec[pos[el[(size_t)e * nl + v]]++] = 4 * e + v;
  int32_t *dp = nullptr, *dr = nullptr;
  TRY(c->alloc(&dp, ptr.size()));
  TRY(c->alloc(&dr, rec.size()));
  HIPCHK(hipMemcpyAsync(dp, ptr.data(), sizeof(int32_t) * ptr.size(), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemcpyAsync(dr, rec.data(), sizeof(int32_t) * rec.size(), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  c->vinc_ptr = dp;
  c->vinc_rec = dr;
  return KS_OK;
}

// dE/dX at every node (device [n_nodes][3], scaled by dE) for the step just
// differentiated: Y solves the adjoint BVPs, PC = P G^-1 P^T psi_bar_tilde.
// Terms (inputs, boundary data and the matrix of I_H^h held fixed):
//   stiffness pairs  (psi, psi) f/2, (Y, psi_hat) -1/2, (V_0, V_0) -1/(8 pi),
//                    (W, V_bc) -1, (W2, V_H^l) +1;
//   mass pairs       (psi, psi) -f theta, (Y, psi_hat) -mu, (PC, psi_tilde) -1,
//                    (Y, psi^l) lambda^l + mu;
//   fixed field      F = rho eps - gam V_xc^l + rho V_0 + (rho - rho^l/2) V_bc
//                        - gam V_H^l - 4 pi rho^l W2,   gam = sum_i Y_i psi_hat_i;
//   moving V_ext     with weight rho - gam;
// V_0 = V_H[rho_out] with zero boundary values, V_bc the lift of w_B,
// V_H^l = V_H[rho^l] with w_B, K_II W = <rho - rho^l/2, phi>, K_II W2 = <gam, phi>.
static int mesh_gradient(ks_ctx *c, double dE, const double *PC, const double *Y, double *dEdX) {
  hipStream_t s = c->s;
  const int k = c->last_k, nH = c->N_H, nn = c->n_nodes;
  const int64_t nqt = (int64_t)c->n_e * c->n_q;
  TRY(vertex_incidence(c));
  DevBuf tmp;
  auto get = [&](int64_t n) -> double * {
    void *q = nullptr;
    if (hipMalloc(&q, sizeof(double) * std::max<int64_t>(n, 1)) != hipSuccess) return nullptr;
    tmp.ptrs.push_back(q);
    return static_cast<double *>(q);
  };
  double *gam = get(nqt), *eps = get(nqt), *vxl = get(nqt), *scr = get(nqt), *F = get(nqt), *G = get(nqt),
         *per = get((int64_t)c->n_e * 12), *coef = get(8 * (int64_t)k);
  if (!gam || !eps || !vxl || !scr || !F || !G || !per || !coef) return fail(KS_ERR_NOMEM, "hipMalloc failed");
  launch_pair_q(c->edof, c->n_loc, c->n_e, c->n_q, c->phi, Y, k, c->PsiHat, k, k, gam, s);
  launch_xc(nqt, c->rho_out, c->opt.xc_mode, eps, scr, s);
  launch_xc(nqt, c->rho_l, c->opt.xc_mode, scr, vxl, s);
  MeshGradPairs pr;
  double *V0q = nullptr, *Vbcq = nullptr, *VHlq = nullptr, *W2q = nullptr;
  if (c->opt.hartree_mode != KS_HARTREE_OFF) {
    double *V0 = get(nn), *Vbc = get(nn), *VHl = get(nn), *W = get(nn), *W2 = get(nn), *wBs = get(c->NB);
    V0q = get(nqt);
    Vbcq = get(nqt);
    VHlq = get(nqt);
    W2q = get(nqt);
    if (!V0 || !Vbc || !VHl || !W || !W2 || !wBs || !V0q || !Vbcq || !VHlq || !W2q)
      return fail(KS_ERR_NOMEM, "hipMalloc failed");
    const int64_t nb = std::max(1, c->NB);
    HIPCHK(hipMemcpyAsync(wBs, c->wB, sizeof(double) * nb, hipMemcpyDeviceToDevice, s));
    struct RestoreWB {  // the step's boundary data are back in place on every exit
      ks_ctx *c;
      const double *src;
      int64_t n;
      ~RestoreWB() {
        (void)hipMemcpyAsync(c->wB, src, sizeof(double) * n, hipMemcpyDeviceToDevice, c->s);
        c->vh_warm = false;
      }
    } restore{c, wBs, nb};
    auto solve = [&](const double *f, double *nodal, double *atq) -> int {
      c->vh_warm = false;
      int it = 0;
      const int r = hartree_solve(c, f, &it);
      if (r < 0) return r;
      HIPCHK(hipMemcpyAsync(nodal, c->vh_nodes, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
      if (atq) HIPCHK(hipMemcpyAsync(atq, c->vh_q, sizeof(double) * nqt, hipMemcpyDeviceToDevice, s));
      return KS_OK;
    };
    const double f4pi = 1.0 / (4.0 * M_PI);
    TRY(solve(c->rho_l, VHl, VHlq));
    launch_fill(nqt, 0.0, scr, s);
    TRY(solve(scr, Vbc, Vbcq));
    launch_fill(nb, 0.0, c->wB, s);
    TRY(solve(c->rho_out, V0, V0q));
    launch_combine3(nqt, f4pi, c->rho_out, -0.5 * f4pi, c->rho_l, 0.0, nullptr, scr, s);
    TRY(solve(scr, W, nullptr));
    launch_combine3(nqt, f4pi, gam, 0.0, nullptr, 0.0, nullptr, scr, s);
    TRY(solve(scr, W2, W2q));
    pr.n_nodal = 3;
    pr.nu[0] = V0, pr.nv[0] = V0, pr.nw[0] = -1.0 / (8.0 * M_PI);
    pr.nu[1] = W, pr.nv[1] = Vbc, pr.nw[1] = -1.0;
    pr.nu[2] = W2, pr.nv[2] = VHl, pr.nw[2] = 1.0;
  }
  launch_pulay_fields(nqt, c->rho_out, c->rho_l, eps, vxl, gam, V0q, Vbcq, VHlq, W2q, F, G, s);
  std::vector<double> cf((size_t)8 * k);
  for (int i = 0; i < k; ++i) {
    const double f = c->last_occ[i];
    cf[(0 * k + i) * 2] = 0.5 * f, cf[(0 * k + i) * 2 + 1] = -f * c->last_theta[i];
    cf[(1 * k + i) * 2] = -0.5, cf[(1 * k + i) * 2 + 1] = -c->mu;
    cf[(2 * k + i) * 2] = 0.0, cf[(2 * k + i) * 2 + 1] = -1.0;
    cf[(3 * k + i) * 2] = 0.0, cf[(3 * k + i) * 2 + 1] = c->last_lam_in[i] + c->mu;
  }
  HIPCHK(hipMemcpyAsync(coef, cf.data(), sizeof(double) * cf.size(), hipMemcpyHostToDevice, s));
  pr.n = 4;
  pr.u[0] = c->PsiNew, pr.v[0] = c->PsiNew, pr.ldu[0] = k, pr.ldv[0] = k;
  pr.u[1] = Y, pr.v[1] = c->PsiHat, pr.ldu[1] = k, pr.ldv[1] = k;
  pr.u[2] = PC, pr.v[2] = c->Z + nH, pr.ldu[2] = k, pr.ldv[2] = c->mp;
  pr.u[3] = Y, pr.v[3] = c->PsiIn, pr.ldu[3] = k, pr.ldv[3] = k;
  if (!launch_mesh_grad(c->coords, c->elems, c->edof, c->n_loc, c->n_e, c->n_q, c->phi, c->dphi, c->qw, c->qbary,
                        pr, coef, k, F, G, c->n_atoms, c->dZ, c->dR, dE, per, s))
    return fail(KS_ERR_ARG, "no mesh-derivative kernel for this element order and quadrature");
  launch_vertex_gather(nn, c->vinc_ptr, c->vinc_rec, per, dEdX, s);
  HIPCHK(hipStreamSynchronize(s));  // before the temporaries are freed
  return KS_OK;
}

// truncated: the BVP part by reverse mode through the truncated FP64 PCG
// (vjp_core, checkpoint segment seg) instead of the implicit adjoint solve
static int step_backward_impl(ks_ctx *c, double dE, double *g_q, double *forces_host, ks_solve_stats *st,
                              bool truncated, int seg, const MeshReq *mesh = nullptr) {
  if (!c || !g_q) return fail(KS_ERR_ARG, "null argument");
  if (!c->have_step) return fail(KS_ERR_STATE, "no ks_scf_step result to differentiate");
  // the adjoint uses the stationarity of the converged inner iteration; an
  // inner iteration stopped at its limit has no such point
  if (!c->last_inner_converged)
    return fail(KS_ERR_STATE, "the last ks_scf_step's inner iteration did not reach tol_inner; "
                              "its gradient is not defined");
  hipStream_t s = c->s;
  const int k = c->last_k, N = c->N, nH = c->N_H, m = nH + k;
  // R = A Psi - M Psi Theta with A the Hamiltonian of the final inner iteration
  spmm_op(c, c->AL, c->PsiNew, k, c->Wv, nullptr);
  if (c->last_nonlinear)
    spmm_op(c, c->MNL, c->PsiNew, k, c->Bv, nullptr);
  spmm_op(c, c->M, c->PsiNew, k, c->Xv, nullptr);
  HIPCHK(hipMemcpyAsync(c->scal, c->last_theta.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
  launch_residual_cols(N, k, c->Wv, c->last_nonlinear ? c->Bv : nullptr, c->Xv, c->scal, c->Rv, s);
  // psi_bar_tilde = R (2 F U_tail^T)
  std::vector<double> U((size_t)m * k), Mk((size_t)k * k);
  HIPCHK(hipMemcpyAsync(U.data(), c->U, sizeof(double) * m * k, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int l = 0; l < k; ++l)
    for (int j = 0; j < k; ++j) Mk[(size_t)l * k + j] = 2.0 * c->last_occ[l] * U[(size_t)(nH + j) * k + l];
  HIPCHK(hipMemcpyAsync(c->dMk, Mk.data(), sizeof(double) * k * k, hipMemcpyHostToDevice, s));
  launch_right_mult(N, k, c->Rv, c->dMk, c->Gv, s);
  // psi_bar_hat = psi_bar_tilde - M P G^{-1} P^T psi_bar_tilde
  launch_gemm_tn(N, nH, k, c->Z, c->mp, c->Gv, k, c->Ctmp, k, c->gwork, c->gwork_n, s);
  launch_small_gemm(nH, k, nH, c->GPPinv, nH, c->Ctmp, k, c->Ttmp, k, 0.0, s);
  launch_ellP_times(N, c->Pidx, c->Pw, c->Ttmp, k, k, 1.0, nullptr, 0, c->Wv, k, s);
  spmm_op(c, c->M, c->Wv, k, c->Xv, nullptr);
  launch_combine3((int64_t)N * k, 1.0, c->Gv, -1.0, c->Xv, 0.0, nullptr, c->Rv, s);
  int r = KS_OK;
  if (!truncated) {
    // P G^-1 P^T psi_bar_tilde (in Wv, which the solve overwrites) for the mesh terms
    DevBuf pcb;
    double *PC = nullptr;
    if (mesh) {
      void *q = nullptr;
      if (hipMalloc(&q, sizeof(double) * N * k) != hipSuccess) return fail(KS_ERR_NOMEM, "hipMalloc failed");
      pcb.ptrs.push_back(q);
      PC = static_cast<double *>(q);
      HIPCHK(hipMemcpyAsync(PC, c->Wv, sizeof(double) * N * k, hipMemcpyDeviceToDevice, s));
    }
    // adjoint boundary value problems S Y = psi_bar_hat (from zero, FP64)
    HIPCHK(hipMemsetAsync(c->Gv, 0, sizeof(double) * N * k, s));
    const double tol = std::min(c->opt.tol_solve, 1e-10);
    r = solve_impl(c, c->Rv, c->Gv, k, KS_PREC_FP64, tol, st);
    if (r < 0) return r;
    // g_q = dE * w |J| (rho - sum Y psi_hat)
    launch_grad_q(c->edof, c->n_loc, c->n_e, c->n_q, c->phi, c->qw, c->absdet, c->Gv, c->PsiHat, k,
                  c->rho_out, dE, g_q, s);
    if (mesh) TRY(mesh_gradient(c, dE, PC, c->Gv, mesh->dEdX));
  } else {
    // the step's BVPs again: S psi_hat = (lambda + mu) M psi_old from psi_old,
    // differentiated through the truncated recurrence with psi_bar_hat as seed
    const int64_t nq = (int64_t)c->n_e * c->n_q;
    double *gb = nullptr;
    if (hipMalloc(&gb, sizeof(double) * nq) != hipSuccess) return fail(KS_ERR_NOMEM, "hipMalloc failed");
    struct Free {
      double *p;
      ~Free() { (void)hipFree(p); }
    } guard{gb};
    if (k > MAX_K) return fail(KS_ERR_ARG, "k too large for the truncated reverse mode");
    TRY(build_rhs(c, c->PsiIn, c->last_lam_in.data(), k, c->Xv));
    int32_t its[MAX_K] = {0};
    TRY(vjp_core(c, c->Xv, c->PsiIn, k, c->opt.tol_solve, c->opt.max_it_solve, seg, c->Rv, c->Wv, gb, nullptr,
                 its));
    if (st) {
      std::memset(st, 0, sizeof(*st));
      for (int j = 0; j < k && j < 64; ++j) st->iters[j] = its[j];
      st->converged = 1;
    }
    // g_q = dE * w |J| rho + dE * dL/dV (L = psi_bar_hat . psi_hat)
    launch_grad_q(c->edof, c->n_loc, c->n_e, c->n_q, c->phi, c->qw, c->absdet, nullptr, nullptr, 0, c->rho_out, dE,
                  g_q, s);
    launch_axpby(nq, dE, gb, 1.0, g_q, s);
  }
  if (forces_host) {
    const int nb = force_blocks(c->n_e);
    for (int a0 = 0; a0 < c->n_atoms; a0 += 8) {
      const int na = std::min(8, c->n_atoms - a0);
      launch_force_partials(c->coords, c->elems, c->n_loc, c->n_e, c->n_q, c->qbary, g_q, a0, na,
                            c->dZ, c->dR, c->redpart, s);
      double f[24];
      TRY(reduce_small(c, c->redpart, nb, 24, f));
      for (int a = 0; a < na; ++a)
        for (int d = 0; d < 3; ++d) forces_host[3 * (a0 + a) + d] = -f[3 * a + d];
    }
    // - dE_nn / dR_a, scaled by the seed
    for (int a = 0; a < c->n_atoms; ++a)
      for (int b = 0; b < c->n_atoms; ++b) {
        if (a == b) continue;
        double d[3], r2 = 0.0;
        for (int t = 0; t < 3; ++t) {
          d[t] = c->hR[3 * a + t] - c->hR[3 * b + t];
          r2 += d[t] * d[t];
        }
        const double r3 = r2 * std::sqrt(r2);
        for (int t = 0; t < 3; ++t) forces_host[3 * a + t] += dE * c->hZ[a] * c->hZ[b] * d[t] / r3;
      }
    // nodes that follow the nuclei: F_a -= sum_v motion[v][a] dE/dX_v
    if (mesh && mesh->motion) {
      const int nb = motion_blocks(c->n_nodes);
      for (int a0 = 0; a0 < c->n_atoms; a0 += 8) {
        const int na = std::min(8, c->n_atoms - a0);
        launch_motion_partials(c->n_nodes, mesh->motion, c->n_atoms, a0, na, mesh->dEdX, c->redpart, s);
        double f[24];
        TRY(reduce_small(c, c->redpart, nb, 24, f));
        for (int a = 0; a < na; ++a)
          for (int d = 0; d < 3; ++d) forces_host[3 * (a0 + a) + d] -= f[3 * a + d];
      }
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  return r;
}

extern "C" int ks_step_backward(ks_ctx *c, double dE, double *g_q, double *forces_host, ks_solve_stats *st) {
  return step_backward_impl(c, dE, g_q, forces_host, st, false, 0);
}

extern "C" int ks_step_backward_truncated(ks_ctx *c, double dE, int32_t seg, double *g_q, double *forces_host,
                                          ks_solve_stats *st) {
  if (c && c->have_step && c->last_precision != KS_PREC_FP64)
    return fail(KS_ERR_STATE, "the truncated reverse mode needs the last ks_scf_step in KS_PREC_FP64");
  return step_backward_impl(c, dE, g_q, forces_host, st, true, seg);
}

extern "C" int ks_step_backward_mesh(ks_ctx *c, double dE, const double *motion, double *dEdX, double *g_q,
                                     double *forces_host, ks_solve_stats *st) {
  if (!c || (!dEdX && !motion)) return fail(KS_ERR_ARG, "null argument: give dEdX, motion or both");
  if (motion && !forces_host) return fail(KS_ERR_ARG, "motion given without forces_host");
  if (!c->vext_atomic)
    return fail(KS_ERR_STATE, "V_ext was set as a field; the mesh derivative needs the nuclear potential");
  DevBuf tmp;
  auto get = [&](int64_t n) -> double * {
    void *q = nullptr;
    if (hipMalloc(&q, sizeof(double) * std::max<int64_t>(n, 1)) != hipSuccess) return nullptr;
    tmp.ptrs.push_back(q);
    return static_cast<double *>(q);
  };
  MeshReq m;
  m.motion = motion;
  m.dEdX = dEdX ? dEdX : get(3 * (int64_t)c->n_nodes);
  if (!g_q) g_q = get((int64_t)c->n_e * c->n_q);
  if (!m.dEdX || !g_q) return fail(KS_ERR_NOMEM, "hipMalloc failed");
  return step_backward_impl(c, dE, g_q, forces_host, st, false, 0, &m);
}

// ---------------------------------------------------------------- batches
struct ks_batch {
  int n = 0, grid = 0, grid_max = 0;
  hipStream_t s = nullptr;
  std::vector<ks_ctx *> sys;
  std::vector<int> k, team, team0, ng;
  // per system the halo tiling its products use (index into the context's
  // tilings, -1: row products) when it fits the launch's LDS
  std::vector<int> tile;
  size_t lds = 0;              // dynamic LDS of the launch (keeps `grid` resident)
  std::vector<double> weight;  // relative cost per system, drives the team split
  DevBuf mem;
  void *table = nullptr;
  int *wg_sys = nullptr, *iters = nullptr, *status = nullptr;
  double *relres = nullptr, *part = nullptr;
  unsigned int *bar = nullptr;
  unsigned long long *t_done = nullptr, *t0 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~ks_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
  }
  template <typename T>
  int alloc(T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(sizeof(T) * count, 256)) != hipSuccess)
      return fail(KS_ERR_NOMEM, "hipMalloc failed");
    mem.ptrs.push_back(q);
    *p = reinterpret_cast<T *>(q);
    return KS_OK;
  }
};

// largest NG (lanes per row) allowed for k columns: k*NG lanes fit a wave
static int batch_ng_cap(int k, int ng) {
  while (ng > 1 && ng * k > 64) ng >>= 1;
  return ng;
}

// the tiling system i uses under the current LDS budget (nullptr: row
// products): tile ti when it exists and its halo image fits
static const Tiling *batch_tiling(const ks_batch *b, int i, int ti) {
  if (ti < 0 || ti >= ks_ctx::NTILE) return nullptr;
  const Tiling &t = b->sys[i]->til[ti];
  if (!t.nblk || (size_t)t.max_halo * b->k[i] * sizeof(double) > b->lds) return nullptr;
  return &t;
}
// the launch's LDS budget for the current grid; every system's default
// tiling: the largest row block whose halo image fits
static int batch_set_grid(ks_batch *b, int grid, bool reset_tiles) {
  b->grid = grid;
  const int64_t lds = batch_lds_budget(grid);
  if (lds < 0) return fail(KS_ERR_HIP, "batch: occupancy query failed");
  b->lds = (size_t)lds;
  if (reset_tiles)
    for (int i = 0; i < b->n; ++i) {
      b->tile[i] = -1;
      for (int ti = ks_ctx::NTILE - 1; ti >= 0 && b->tile[i] < 0; --ti)
        if (batch_tiling(b, i, ti)) b->tile[i] = ti;
    }
  return KS_OK;
}

// Teams proportional to the weights (largest remainders), at least one
// workgroup each, summing to the grid; table and workgroup map uploaded.
static int batch_layout(ks_batch *b) {
  const int n = b->n;
  double total = 0.0;
  for (double w : b->weight) total += w;
  const int left = b->grid - n;
  std::vector<std::pair<double, int>> rem(n);
  int used = 0;
  for (int i = 0; i < n; ++i) {
    const double share = (double)left * b->weight[i] / total;
    const int extra = (int)std::floor(share);
    b->team[i] = 1 + extra;
    used += b->team[i];
    rem[i] = {share - extra, i};
  }
  std::sort(rem.begin(), rem.end(), [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
    return x.first > y.first || (x.first == y.first && x.second < y.second);
  });
  for (int j = 0; used < b->grid; j = (j + 1) % n, ++used) b->team[rem[j].second]++;
  std::vector<int> wg(b->grid);
  for (int i = 0, o = 0; i < n; ++i) {
    b->team0[i] = o;
    for (int t = 0; t < b->team[i]; ++t) wg[o++] = i;
  }
  std::vector<char> tab(batch_sys_bytes() * n);
  for (int i = 0; i < n; ++i) {
    ks_ctx *c = b->sys[i];
    pack_batch_sys(tab.data() + batch_sys_bytes() * i, c->rowptr, c->col, c->S, c->diagS, c->Bv, c->Xv,
                   (double *)c->pw64.R, (double *)c->pw64.P, (double *)c->pw64.Q, b->part,
                   b->bar + 2 * i, c->N, b->k[i], b->ng[i], b->team0[i], b->team[i],
                   c->opt.max_it_solve, c->opt.tol_solve, b->iters + (size_t)i * MAX_K,
                   b->relres + (size_t)i * MAX_K, b->t_done + i, b->status + i,
                   batch_tiling(b, i, b->tile[i]));
  }
  // the launch reads these at its start: upload synchronously
  HIPCHK(hipMemcpyAsync(b->table, tab.data(), tab.size(), hipMemcpyHostToDevice, b->s));
  HIPCHK(hipMemcpyAsync(b->wg_sys, wg.data(), sizeof(int) * b->grid, hipMemcpyHostToDevice, b->s));
  HIPCHK(hipStreamSynchronize(b->s));
  return KS_OK;
}

// (re)capture the launch for the current grid; every solve replays it (the
// table it reads is rewritten in place when the layout is retuned)
static int batch_capture(ks_batch *b) {
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  hipStream_t s = b->s;
  HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  launch_batch_reset(b->table, b->n, b->t0, s);
  launch_batch_pcg(b->grid, b->table, b->wg_sys, b->lds, s);
  HIPCHK(hipStreamEndCapture(s, &b->graph));
  HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return KS_OK;
}

extern "C" int ks_batch_create(int32_t n, ks_ctx *const *systems, const int32_t *k_host,
                               int32_t grid_req, ks_batch **out) {
  if (n < 1 || n > 256 || !systems || !k_host || !out)
    return fail(KS_ERR_ARG, "batch needs 1..256 systems and non-null arrays");
  ks_batch *b = new ks_batch();
  auto bail = [&](int code) {
    delete b;
    return code;
  };
  b->n = n;
  // a stream of the batch's own (default priority): capture needs a
  // non-null stream, and the contexts' streams may be the null stream
  if (hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(KS_ERR_HIP, "stream creation failed"));
  for (int i = 0; i < n; ++i) {
    ks_ctx *c = systems[i];
    if (!c) return bail(fail(KS_ERR_ARG, "null system"));
    if (k_host[i] < 1 || k_host[i] > c->k_max) return bail(fail(KS_ERR_ARG, "k out of range"));
    if (std::find(b->sys.begin(), b->sys.end(), c) != b->sys.end())
      return bail(fail(KS_ERR_ARG, "a context appears twice in the batch"));
    b->sys.push_back(c);
    b->k.push_back(k_host[i]);
    // initial cost model: matrix entries times columns, plus rows
    b->weight.push_back((double)c->nnz * k_host[i] + 8.0 * c->N);
    // lanes per row: the system's autotuned choice, else a rule by k
    const int ng = c->ng64 > 0 ? c->ng64 : (k_host[i] == 1 ? 8 : (k_host[i] <= 4 ? 4 : (k_host[i] <= 12 ? 2 : 1)));
    b->ng.push_back(batch_ng_cap(k_host[i], ng));
  }
  const int resident = batch_resident_grid();
  if (resident <= 0) return bail(fail(KS_ERR_HIP, "occupancy query failed"));
  const int grid = grid_req > 0 ? std::min<int>(grid_req, resident) : resident;
  if (grid < n) return bail(fail(KS_ERR_ARG, "more systems than resident workgroups"));
  b->grid_max = grid;
  b->tile.assign(n, -1);
  if (batch_set_grid(b, grid, true) < 0) return bail(KS_ERR_HIP);
  b->team.assign(n, 1);
  b->team0.assign(n, 0);
  if (b->alloc(reinterpret_cast<char **>(&b->table), batch_sys_bytes() * n) < 0 ||
      b->alloc(&b->wg_sys, b->grid) < 0 || b->alloc(&b->iters, (size_t)n * MAX_K) < 0 ||
      b->alloc(&b->status, n) < 0 || b->alloc(&b->relres, (size_t)n * MAX_K) < 0 ||
      b->alloc(&b->part, (size_t)b->grid * batch_part_stride()) < 0 || b->alloc(&b->bar, (size_t)2 * n) < 0 ||
      b->alloc(&b->t_done, n) < 0 || b->alloc(&b->t0, 1) < 0)
    return bail(KS_ERR_NOMEM);
  if (hipMemsetAsync(b->bar, 0, sizeof(unsigned) * 2 * n, b->s) != hipSuccess)
    return bail(fail(KS_ERR_HIP, "batch clear failed"));
  {
    int r = batch_layout(b);
    if (r >= 0) r = batch_capture(b);
    if (r < 0) return bail(r);
  }
  if (hipEventCreate(&b->e0) != hipSuccess || hipEventCreate(&b->e1) != hipSuccess)
    return bail(fail(KS_ERR_HIP, "event creation failed"));
  *out = b;
  return KS_OK;
}

extern "C" int ks_batch_info(const ks_batch *b, int32_t *grid_host, int32_t *team_host,
                             int32_t *ng_host, int32_t *tile_host) {
  if (!b) return fail(KS_ERR_ARG, "null batch");
  if (grid_host) *grid_host = b->grid;
  for (int i = 0; i < b->n; ++i) {
    if (team_host) team_host[i] = b->team[i];
    if (ng_host) ng_host[i] = b->ng[i];
    if (tile_host) {
      const Tiling *t = batch_tiling(b, i, b->tile[i]);
      tile_host[i] = t ? t->BR : 0;
    }
  }
  return KS_OK;
}

extern "C" int ks_batch_set_layout(ks_batch *b, const int32_t *ng_host, const int32_t *tile_host) {
  if (!b) return fail(KS_ERR_ARG, "null batch");
  std::vector<int> ng = b->ng, tile = b->tile;
  for (int i = 0; i < b->n; ++i) {
    if (ng_host) {
      const int g = ng_host[i];
      if ((g != 1 && g != 2 && g != 4 && g != 8) || g * b->k[i] > 64)
        return fail(KS_ERR_ARG, "lanes per row must be 1, 2, 4 or 8 with lanes x k <= 64");
      ng[i] = g;
    }
    if (tile_host) {
      const int rows = tile_host[i];
      const int ti = rows ? tile_index(rows) : -1;
      if (rows && !batch_tiling(b, i, ti))
        return fail(KS_ERR_ARG, "system " + std::to_string(i) + " has no halo tiling of that row block fitting the launch's LDS");
      tile[i] = ti;
    }
  }
  b->ng = ng;
  b->tile = tile;
  return batch_layout(b);
}

// right-hand sides B_s = M_s psi_s diag(lambda_s + mu_s), X_s = psi_s
static int batch_prepare(ks_batch *b, const double *const *psi_old, const double *const *lambda_host) {
  for (int i = 0; i < b->n; ++i) {
    ks_ctx *c = b->sys[i];
    hipStream_t s = c->s;
    if (!c->have_S) return fail(KS_ERR_STATE, "system " + std::to_string(i) + " has no assembled operator");
    const int k = b->k[i];
    launch_rows_to_storage(c->N, k, psi_old[i], c->PsiIn, c->int2nat, s);
    spmm_op(c, c->M, c->PsiIn, k, c->Bv, nullptr);
    std::vector<double> sc(k);
    for (int j = 0; j < k; ++j) sc[j] = lambda_host[i][j] + c->mu;
    HIPCHK(hipMemcpyAsync(c->scal, sc.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    launch_scale_cols(c->N, k, c->Bv, c->scal, s);
    HIPCHK(hipMemcpyAsync(c->Xv, c->PsiIn, sizeof(double) * c->N * k, hipMemcpyDeviceToDevice, s));
    // the batch stream must see each system's right-hand side
    HIPCHK(hipStreamSynchronize(s));
  }
  return KS_OK;
}

// one replay of the captured launch; per-system results into st
static int batch_run(ks_batch *b, ks_batch_stats *st) {
  hipStream_t s = b->s;
  HIPCHK(hipEventRecord(b->e0, s));
  HIPCHK(hipGraphLaunch(b->exec, s));
  HIPCHK(hipEventRecord(b->e1, s));
  std::vector<int> it((size_t)b->n * MAX_K), status(b->n);
  std::vector<double> rr((size_t)b->n * MAX_K);
  std::vector<unsigned long long> td(b->n);
  unsigned long long t0 = 0;
  HIPCHK(hipMemcpyAsync(it.data(), b->iters, sizeof(int) * it.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(rr.data(), b->relres, sizeof(double) * rr.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(status.data(), b->status, sizeof(int) * b->n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(td.data(), b->t_done, sizeof(unsigned long long) * b->n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&t0, b->t0, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, b->e0, b->e1));
  int clk_khz = 100000;  // wall_clock64 runs at a constant rate (100 MHz unless reported)
  (void)hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, 0);
  int ret = KS_OK;
  for (int i = 0; i < b->n; ++i) {
    if (status[i] == -2)
      return fail(KS_ERR_HIP, "batched solve: barrier wait limit hit (system " + std::to_string(i) + ")");
    if (status[i] == -1) return fail(KS_ERR_BREAKDOWN, "batched solve: PCG breakdown in system " + std::to_string(i));
    if (status[i] == 1) ret = KS_NOT_CONVERGED;
  }
  std::memset(st, 0, sizeof(*st));
  st->seconds = ms * 1e-3;
  st->n = b->n;
  for (int i = 0; i < b->n; ++i) {
    st->system_seconds[i] = (double)(td[i] - t0) / ((double)clk_khz * 1e3);
    int mx = 0;
    double rmax = 0.0;
    for (int j = 0; j < b->k[i]; ++j) {
      mx = std::max(mx, it[(size_t)i * MAX_K + j]);
      rmax = std::max(rmax, rr[(size_t)i * MAX_K + j]);
    }
    st->iters[i] = mx;
    st->relres[i] = rmax;
    st->status[i] = status[i];
  }
  return ret;
}

extern "C" int ks_batch_block_solve(ks_batch *b, const double *const *psi_old,
                                    const double *const *lambda_host, double *const *psi_hat,
                                    ks_batch_stats *st) {
  if (!b || !psi_old || !lambda_host || !psi_hat) return fail(KS_ERR_ARG, "null argument");
  TRY(batch_prepare(b, psi_old, lambda_host));
  ks_batch_stats loc;
  const int ret = batch_run(b, &loc);
  if (ret < 0) return ret;
  for (int i = 0; i < b->n; ++i) {
    ks_ctx *c = b->sys[i];
    launch_rows_to_api(c->N, b->k[i], c->Xv, psi_hat[i], c->int2nat, b->s);
  }
  HIPCHK(hipStreamSynchronize(b->s));
  if (st) *st = loc;
  return ret;
}

// Autotuner of the batch layout on the given inputs.  For each candidate
// grid (the resident workgroup count and fractions of it): (1) lanes per
// row, per system, from one run at each candidate; (2) team sizes by
// feedback: the weight of a system becomes its measured time times its
// team, so the next split equalises completion times.  Keeps the fastest
// layout seen.
extern "C" int ks_batch_autotune(ks_batch *b, const double *const *psi_old,
                                 const double *const *lambda_host, int32_t rounds, double *best_ms) {
  if (!b || !psi_old || !lambda_host) return fail(KS_ERR_ARG, "null argument");
  ks_batch_stats st;
  const int n = b->n;
  const std::vector<double> w0 = b->weight;
  double best = 1e300;
  int best_grid = b->grid;
  std::vector<int> best_ng = b->ng, best_tile = b->tile;
  std::vector<double> best_w = b->weight;
  auto run = [&]() -> int {
    TRY(batch_layout(b));
    TRY(batch_prepare(b, psi_old, lambda_host));
    const int r = batch_run(b, &st);
    return r < 0 ? r : KS_OK;
  };
  for (int frac : {4, 3, 2, 1}) {
    const int g = b->grid_max * frac / 4;
    if (g < n) continue;
    TRY(batch_set_grid(b, g, false));
    TRY(batch_capture(b));
    b->weight = w0;
    std::vector<double> t_best(n, 1e300);
    std::vector<int> ng_best(b->ng), tile_best(b->tile);
    // every system on the row products, then on each tiling that fits it
    // (row blocks of 32, 64, 128 and 256 rows), at every lanes-per-row split
    for (int ti : {-1, 0, 1, 3, 5})
      for (int ng : {1, 2, 4, 8}) {
        bool any = false;
        for (int i = 0; i < n; ++i) {
          b->ng[i] = batch_ng_cap(b->k[i], ng);
          b->tile[i] = batch_tiling(b, i, ti) ? ti : -1;
          any = any || b->tile[i] >= 0;
        }
        if (ti >= 0 && !any) continue;
        TRY(run());
        for (int i = 0; i < n; ++i)
          if ((ti < 0 || b->tile[i] >= 0) && st.system_seconds[i] < t_best[i]) {
            t_best[i] = st.system_seconds[i];
            ng_best[i] = b->ng[i];
            tile_best[i] = b->tile[i];
          }
      }
    b->ng = ng_best;
    b->tile = tile_best;
    for (int r = 0; r < std::max(1, (int)rounds); ++r) {
      TRY(run());
      if (st.seconds < best) {
        best = st.seconds;
        best_grid = g;
        best_ng = b->ng;
        best_tile = b->tile;
        best_w = b->weight;
      }
      for (int i = 0; i < n; ++i) b->weight[i] = std::max(st.system_seconds[i], 1e-7) * b->team[i];
    }
  }
  TRY(batch_set_grid(b, best_grid, false));
  b->ng = best_ng;
  b->tile = best_tile;
  b->weight = best_w;
  TRY(batch_layout(b));
  TRY(batch_capture(b));
  if (best_ms) *best_ms = best * 1e3;
  return KS_OK;
}

extern "C" int ks_batch_destroy(ks_batch *b) {
  if (b) {
    (void)hipStreamSynchronize(b->s);
    delete b;
  }
  return KS_OK;
}

extern "C" int ks_destroy(ks_ctx *c) {
  if (!c) return KS_OK;
  (void)hipStreamSynchronize(c->s);
  delete c;
  return KS_OK;
}

extern "C" int ks_get_sizes(const ks_ctx *c, double *o) {
  if (!c || !o) return fail(KS_ERR_ARG, "null argument");
  o[0] = c->N;
  o[1] = c->n_nodes;
  o[2] = c->n_e;
  o[3] = c->n_q;
  o[4] = c->N_H;
  o[5] = (double)c->nnz;
  o[6] = c->n_loc;
  o[7] = c->n_colours;
  o[8] = c->mp;
  o[9] = c->mu;
  o[10] = mg_levels(c->mg);
  return KS_OK;
}

// --------------------------------------------------------------- assemble
// rho_l, w_B, V_H, V_xc of the density of psi; S = base + M[V_H + V_xc].
// want_s32: also the FP32 copy of S (the step solves in the mixed form)
static int assemble_impl(ks_ctx *c, const double *psi, int k, const double *occ_host, int *p_iters,
                         bool want_s32 = false) {
  hipStream_t s = c->s;
  const int64_t nqt = (int64_t)c->n_e * c->n_q;
  const bool nonlinear = psi && (c->opt.hartree_mode != KS_HARTREE_OFF || c->opt.xc_mode != KS_XC_NONE);
  if (psi) {
    HIPCHK(hipMemcpyAsync(c->occ_d, occ_host, sizeof(double) * k, hipMemcpyHostToDevice, s));
    launch_density(c->edof, c->n_loc, c->n_e, c->n_q, c->phi, psi, k, k, c->occ_d, c->rho_l, s);
  } else {
    launch_fill(nqt, 0.0, c->rho_l, s);
  }
  launch_fill(nqt, 0.0, c->vh_q, s);
  if (psi && c->opt.hartree_mode != KS_HARTREE_OFF) {
    TRY(boundary_data(c, c->rho_l));
    int r = hartree_solve(c, c->rho_l, p_iters);
    if (r < 0) return r;
  } else {
    launch_fill(std::max(1, c->NB), 0.0, c->wB, s);
    launch_fill(c->n_nodes, 0.0, c->vh_nodes, s);
  }
  launch_xc(nqt, c->rho_l, psi ? c->opt.xc_mode : KS_XC_NONE, c->exc_q, c->vxc_q, s);
  launch_add(nqt, c->vh_q, c->vxc_q, c->vnl_q, s);
  // the mixed form's FP32 copy of S comes out of the same pass
  const bool mixed = want_s32;
  c->have_S32 = false;
  if (nonlinear) {  // S = A^L + mu M + M[V_nl]
    c->have_S32 = assemble_potential_all(c, c->vnl_q, c->S, c->base, mixed ? c->S32 : nullptr);
  } else {
    launch_axpby(c->nnz_ext, 1.0, c->base, 0.0, c->S, s);
  }
  launch_extract_diag(c->N, c->rowptr, c->col, c->S, c->diagS, s);
  if (c->have_S32) launch_to_float(c->N, c->diagS, c->diagS32, s);
  c->have_S = true;
  c->have_step = false;
  return KS_OK;
}

extern "C" int ks_assemble(ks_ctx *c, const double *psi, int32_t k, const double *occ_host,
                           double *rho_q, double *veff_q, double *vh_nodes, double *energies_host) {
  if (!c) return fail(KS_ERR_ARG, "null context");
  if (psi && (k < 1 || k > c->k_max || !occ_host)) return fail(KS_ERR_ARG, "k must be in 1..k_max with occupations");
  int piters = 0;
  if (psi) launch_rows_to_storage(c->N, k, psi, c->PsiIn, c->int2nat, c->s);
  TRY(assemble_impl(c, psi ? c->PsiIn : nullptr, k, occ_host, &piters));
  const int64_t nqt = (int64_t)c->n_e * c->n_q;
  if (rho_q) HIPCHK(hipMemcpyAsync(rho_q, c->rho_l, sizeof(double) * nqt, hipMemcpyDeviceToDevice, c->s));
  if (veff_q) launch_combine3(nqt, 1.0, c->vext_q, 1.0, c->vh_q, 1.0, c->vxc_q, veff_q, c->s);
  if (vh_nodes) HIPCHK(hipMemcpyAsync(vh_nodes, c->vh_nodes, sizeof(double) * c->n_nodes, hipMemcpyDeviceToDevice, c->s));
  if (energies_host) {
    const double *a[4] = {c->vh_q, c->exc_q, c->vxc_q, c->vext_q};
    const double *b[4] = {c->rho_l, c->rho_l, c->rho_l, c->rho_l};
    double e[4];
    TRY(weighted_dots(c, 4, a, b, e));
    energies_host[0] = 0.5 * e[0];
    energies_host[1] = e[1];
    energies_host[2] = e[2];
    energies_host[3] = e[3];
    energies_host[4] = piters;
  }
  HIPCHK(hipStreamSynchronize(c->s));
  return KS_OK;
}

extern "C" int ks_export_operator(ks_ctx *c, int32_t which, int32_t *row_ptr, int32_t *colp,
                                  double *val) {
  if (!c) return fail(KS_ERR_ARG, "null context");
  const double *src = nullptr;
  switch (which) {
    case 0: src = c->S; if (!c->have_S) return fail(KS_ERR_STATE, "S not assembled"); break;
    case 1: src = c->K; break;
    case 2: src = c->M; break;
    case 3: src = c->AL; break;
    case 4: src = c->MNL; break;
    default: return fail(KS_ERR_ARG, "which must be 0..4");
  }
  // stored rows/columns are in storage order: rebuild the CSR in the API's
  // natural numbering on the host (inspection only, not a hot path)
  const int N = c->N;
  std::vector<int32_t> rp(N + 1), cl(c->nnz), nrp(N + 1, 0), ncl(c->nnz);
  std::vector<double> vl(c->nnz), nvl(c->nnz);
  HIPCHK(hipMemcpyAsync(rp.data(), c->rowptr, sizeof(int32_t) * (N + 1), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipMemcpyAsync(cl.data(), c->col, sizeof(int32_t) * c->nnz, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipMemcpyAsync(vl.data(), src, sizeof(double) * c->nnz, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  const std::vector<int32_t> &i2n = c->h_int2nat;
  std::vector<int32_t> n2i(N);
  for (int r = 0; r < N; ++r) n2i[i2n[r]] = r;
  for (int i = 0; i < N; ++i) nrp[i + 1] = nrp[i] + (rp[n2i[i] + 1] - rp[n2i[i]]);
  parallel_for(N, [&](int64_t i) {
    const int r = n2i[i];
    std::vector<std::pair<int32_t, double>> e;
    e.reserve(rp[r + 1] - rp[r]);
    for (int j = rp[r]; j < rp[r + 1]; ++j) e.push_back({i2n[cl[j]], vl[j]});
    std::sort(e.begin(), e.end(), [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
      return x.first < y.first;
    });
    for (size_t t = 0; t < e.size(); ++t) {
      ncl[nrp[i] + t] = e[t].first;
      nvl[nrp[i] + t] = e[t].second;
    }
  });
  if (row_ptr) HIPCHK(hipMemcpyAsync(row_ptr, nrp.data(), sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice, c->s));
  if (colp) HIPCHK(hipMemcpyAsync(colp, ncl.data(), sizeof(int32_t) * c->nnz, hipMemcpyHostToDevice, c->s));
  if (val) HIPCHK(hipMemcpyAsync(val, nvl.data(), sizeof(double) * c->nnz, hipMemcpyHostToDevice, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  return KS_OK;
}

// ------------------------------------------------------------ block solve
static int true_residual(ks_ctx *c, const double *B, const double *X, int k, double *relres,
                         bool *ok) {
  spmm_op(c, c->S, X, k, c->Wv, B);
  std::vector<double> rn(k), bn(k);
  int nb = launch_colnorms(c->N, k, c->Wv, c->redpart, c->s);
  TRY(reduce_small(c, c->redpart, nb, k, rn.data()));
  nb = launch_colnorms(c->N, k, B, c->redpart, c->s);
  TRY(reduce_small(c, c->redpart, nb, k, bn.data()));
  *ok = true;
  for (int j = 0; j < k; ++j) {
    relres[j] = bn[j] > 0 ? std::sqrt(rn[j] / bn[j]) : std::sqrt(rn[j]);
    if (!(relres[j] <= c->opt.tol_solve * 1.0000001) && bn[j] > 0) *ok = false;
  }
  return KS_OK;
}

// S X = B from X (in/out), FP64 or FP32-in-FP64-refinement
// Cholesky solve of the k x k SPD system G Y = H (row-major, host); false
// if G is not positive definite
static bool chol_solve(int k, std::vector<double> G, const std::vector<double> &H, std::vector<double> &Y) {
  for (int j = 0; j < k; ++j) {
    double d = G[(size_t)j * k + j];
    for (int p = 0; p < j; ++p) d -= G[(size_t)j * k + p] * G[(size_t)j * k + p];
    if (!(d > 0.0)) return false;
    const double l = std::sqrt(d);
    G[(size_t)j * k + j] = l;
    for (int i = j + 1; i < k; ++i) {
      double t = G[(size_t)i * k + j];
      for (int p = 0; p < j; ++p) t -= G[(size_t)i * k + p] * G[(size_t)j * k + p];
      G[(size_t)i * k + j] = t / l;
    }
  }
  Y = H;
  for (int c = 0; c < k; ++c) {
    for (int i = 0; i < k; ++i) {  // L y = h
      double t = Y[(size_t)i * k + c];
      for (int p = 0; p < i; ++p) t -= G[(size_t)i * k + p] * Y[(size_t)p * k + c];
      Y[(size_t)i * k + c] = t / G[(size_t)i * k + i];
    }
    for (int i = k - 1; i >= 0; --i) {  // L^T y = y
      double t = Y[(size_t)i * k + c];
      for (int p = i + 1; p < k; ++p) t -= G[(size_t)p * k + i] * Y[(size_t)p * k + c];
      Y[(size_t)i * k + c] = t / G[(size_t)i * k + i];
    }
  }
  return true;
}

// O'Leary's block preconditioned CG in FP64 for S X = B (Jacobi
// preconditioner); X holds the start on entry.  Work blocks: the FP64 PCG
// buffers (R, P, P2 = Z, Q) and c->Wv.
static int block_cg(ks_ctx *c, const double *B, double *X, int k, double tol, ks_solve_stats *st) {
  const int N = c->N;
  hipStream_t s = c->s;
  double *R = static_cast<double *>(c->pw64.R), *P = static_cast<double *>(c->pw64.P);
  double *Z = static_cast<double *>(c->pw64.P2), *Q = static_cast<double *>(c->pw64.Q), *T = c->Wv;
  const size_t kk = (size_t)k * k;
  double *dG = nullptr;
  if (hipMalloc(&dG, sizeof(double) * 2 * kk) != hipSuccess) return fail(KS_ERR_NOMEM, "hipMalloc failed");
  struct Free {
    double *p;
    ~Free() { (void)hipFree(p); }
  } guard{dG};
  std::vector<double> bn(k), rn(k), g1(kk), g2(kk), g3(kk), co(kk);
  auto gram = [&](const double *A, const double *Bm, std::vector<double> &h) -> int {
    launch_gemm_tn_sym(N, k, A, k, Bm, k, dG, k, c->gwork, s);
    HIPCHK(hipMemcpyAsync(h.data(), dG, sizeof(double) * kk, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return KS_OK;
  };
  auto colnorms = [&](const double *A, std::vector<double> &out) -> int {
    const int nb = launch_colnorms(N, k, A, c->redpart, s);
    TRY(reduce_small(c, c->redpart, nb, k, out.data()));
    for (auto &v : out) v = std::sqrt(v);
    return KS_OK;
  };
  // Out = A C (C k x k on the host)
  auto times = [&](const double *A, const std::vector<double> &C, double *Out) -> int {
    HIPCHK(hipMemcpyAsync(dG + kk, C.data(), sizeof(double) * kk, hipMemcpyHostToDevice, s));
    if (launch_tsmm(N, k, A, k, dG + kk, k, Out, k, s) < 0) return fail(KS_ERR_ARG, "k too large for block CG");
    return KS_OK;
  };
  TRY(colnorms(B, bn));
  spmm_op(c, c->S, X, k, R, B);  // R = B - S X
  launch_row_div(N, k, R, c->diagS, Z, s);
  launch_axpby((int64_t)N * k, 1.0, Z, 0.0, P, s);
  TRY(gram(Z, R, g2));
  TRY(colnorms(R, rn));
  auto done = [&]() {
    for (int j = 0; j < k; ++j)
      if (rn[j] > tol * bn[j]) return false;
    return true;
  };
  int it = 0;
  bool conv = done();
  for (it = 0; !conv && it < c->opt.max_it_solve;) {
    ++it;
    spmm_op(c, c->S, P, k, Q, nullptr);
    TRY(gram(P, Q, g1));
    if (!chol_solve(k, g1, g2, co)) return fail(KS_ERR_BREAKDOWN, "block CG: P^T S P is not positive definite");
    TRY(times(P, co, T));
    launch_axpby((int64_t)N * k, 1.0, T, 1.0, X, s);
    TRY(times(Q, co, T));
    launch_axpby((int64_t)N * k, -1.0, T, 1.0, R, s);
    TRY(colnorms(R, rn));
    conv = done();
    if (conv) break;
    launch_row_div(N, k, R, c->diagS, Z, s);
    TRY(gram(Z, R, g3));
    if (!chol_solve(k, g2, g3, co)) return fail(KS_ERR_BREAKDOWN, "block CG: Z^T R is not positive definite");
    TRY(times(P, co, T));
    launch_combine3((int64_t)N * k, 1.0, Z, 1.0, T, 0.0, nullptr, P, s);
    g2 = g3;
  }
  for (int j = 0; j < k && j < 64; ++j) st->iters[j] = it;
  st->converged = conv ? 1 : 0;  // the caller recomputes the true residuals
  return KS_OK;
}

static int solve_impl(ks_ctx *c, const double *B, double *X, int k, int precision, double tol,
                      ks_solve_stats *st) {
  hipStream_t s = c->s;
  if (!c->have_S) return fail(KS_ERR_STATE, "no operator assembled: call ks_assemble first");
  ks_solve_stats loc;
  std::memset(&loc, 0, sizeof(loc));
  HIPCHK(hipEventRecord(c->ev0, s));
  int conv = 0, brk = 0;
  if (precision == KS_PREC_FP64_BLOCK_CG) {
    TRY(block_cg(c, B, X, k, tol, &loc));
    conv = loc.converged;
    loc.refinements = 0;
  } else if (precision == KS_PREC_FP64) {
    int r = pcg_solve<double>(c->N, k, c->rowptr, c->col, c->S, c->rorder, c->diagS, B, X, tol,
                              c->opt.max_it_solve, c->pw64, loc.iters, loc.relres, &conv, &brk, s,
                              c->ng64);
    if (r < 0) return fail(KS_ERR_HIP, "PCG launch failed");
    if (brk) return fail(KS_ERR_BREAKDOWN, "PCG breakdown: p^T S p <= 0 (S not positive definite; increase mu)");
    loc.refinements = 0;
  } else {
    // FP32 operator copy (once per assembly)
    if (!c->have_S32) {
      launch_to_float(c->nnz, c->S, c->S32, s);
      launch_to_float(c->N, c->diagS, c->diagS32, s);
      c->have_S32 = true;
    }
    const int max_ref = 20;
    std::vector<double> rn(k), bn(k), sc(k);
    int nb = launch_colnorms(c->N, k, B, c->redpart, s);
    TRY(reduce_small(c, c->redpart, nb, k, bn.data()));
    int total_it[MAX_K] = {0};
    conv = 0;
    for (int ref = 0; ref < max_ref; ++ref) {
      // FP64 residual and its column norms (one pass through the halo
      // tiles when they serve k; the FP64 PCG workspace holds the partials)
      double *npart = reinterpret_cast<double *>(c->pw64.part);
      nb = c->pw64.til ? launch_residual_tiled_norms(c->N, k, *c->pw64.til, c->pw64.til_tb, c->rowptr, c->S, X,
                                                     c->Wv, B, npart, s)
                       : -1;
      if (nb < 0) {
        spmm_op(c, c->S, X, k, c->Wv, B);
        npart = c->redpart;
        nb = launch_colnorms(c->N, k, c->Wv, npart, s);
      }
      TRY(reduce_small(c, npart, nb, k, rn.data()));
      loc.refinements = ref + 1;
      bool all = true;
      // inexact refinement: column j's FP32 solve stops once its residual
      // is below half of what the outer tolerance still asks of it (never
      // tighter than the inner tolerance): factor max(1, tol/(2 inner rel))
      sc.resize(2 * k);
      for (int j = 0; j < k; ++j) {
        const double rel = bn[j] > 0 ? std::sqrt(rn[j] / bn[j]) : 0.0;
        if (rel > tol) all = false;
        sc[j] = rn[j] > 0 ? 1.0 / std::sqrt(rn[j]) : 0.0;
        sc[k + j] = rel > 0 ? std::max(1.0, 0.5 * tol / (rel * c->opt.mixed_inner_tol)) : 1.0;
      }
      if (all) {
        conv = 1;
        break;
      }
      // FP32 PCG from zero on the scaled residual: one pass writes its
      // right-hand side (the start residual), first direction, X = 0 and
      // start partials
      HIPCHK(hipMemcpyAsync(c->scal, sc.data(), sizeof(double) * 2 * k, hipMemcpyHostToDevice, s));
      if (launch_refine_prep(c->N, k, c->Wv, c->scal, c->diagS32, c->X32, c->pw32, s) < 0)
        return fail(KS_ERR_ARG, "FP32 correction start: unsupported k");
      int it[MAX_K] = {0};
      double rr[MAX_K];
      int c32 = 0;
      int r = pcg_solve<float>(c->N, k, c->rowptr, c->col, c->S32, c->rorder, c->diagS32, nullptr, c->X32,
                               c->opt.mixed_inner_tol, c->opt.max_it_solve, c->pw32, it, rr, &c32,
                               &brk, s, c->ng32, 2);
      if (r < 0) return fail(KS_ERR_HIP, "FP32 PCG launch failed");
      if (brk) return fail(KS_ERR_BREAKDOWN, "FP32 PCG breakdown");
      for (int j = 0; j < k; ++j) total_it[j] += it[j];
      // X += ||r|| d
      for (int j = 0; j < k; ++j) sc[j] = std::sqrt(rn[j]);
      HIPCHK(hipMemcpyAsync(c->scal, sc.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
      launch_refine_update(c->N, k, c->X32, c->scal, X, s);
    }
    for (int j = 0; j < k; ++j) loc.iters[j] = total_it[j];
  }
  HIPCHK(hipEventRecord(c->ev1, s));
  bool ok = true;
  TRY(true_residual(c, B, X, k, loc.relres, &ok));
  float ms = 0.f;
  HIPCHK(hipEventSynchronize(c->ev1));
  HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  loc.seconds = ms * 1e-3;
  loc.converged = conv ? 1 : 0;
  if (st) *st = loc;
  return conv ? KS_OK : KS_NOT_CONVERGED;
}

extern "C" int ks_block_solve_rhs(ks_ctx *c, const double *B, const double *X0, int32_t k,
                                  int32_t precision, double tol, double *X, ks_solve_stats *st) {
  if (!c || !B || !X) return fail(KS_ERR_ARG, "null argument");
  if (k < 1 || k > c->k_max) return fail(KS_ERR_ARG, "k must be in 1..k_max");
  if (precision != KS_PREC_FP64 && precision != KS_PREC_MIXED && precision != KS_PREC_FP64_BLOCK_CG)
    return fail(KS_ERR_ARG, "bad precision");
  launch_rows_to_storage(c->N, k, B, c->Bv, c->int2nat, c->s);
  if (X0) launch_rows_to_storage(c->N, k, X0, c->Xs, c->int2nat, c->s);
  else HIPCHK(hipMemsetAsync(c->Xs, 0, sizeof(double) * c->N * k, c->s));
  const int r = solve_impl(c, c->Bv, c->Xs, k, precision, tol > 0 ? tol : c->opt.tol_solve, st);
  if (r < 0) return r;
  launch_rows_to_api(c->N, k, c->Xs, X, c->int2nat, c->s);
  HIPCHK(hipStreamSynchronize(c->s));
  return r;
}

// B = M psi diag(lambda + mu)
static int build_rhs(ks_ctx *c, const double *psi, const double *lambda_host, int k, double *B) {
  spmm_op(c, c->M, psi, k, B, nullptr);
  double sc[MAX_K];
  for (int j = 0; j < k; ++j) sc[j] = lambda_host[j] + c->mu;
  HIPCHK(hipMemcpyAsync(c->scal, sc, sizeof(double) * k, hipMemcpyHostToDevice, c->s));
  launch_scale_cols(c->N, k, B, c->scal, c->s);
  return KS_OK;
}

// Reverse mode through the truncated FP64 per-column Jacobi-PCG (see
// ks_block_solve_vjp in ks.h).  The forward keeps the per-column scalars of
// every iteration on the host and (R, P) every `seg` iterations on the
// device; the reverse sweep recomputes each segment's iterates from its
// checkpoint with the same kernels and coefficients (bit-identical) and
// runs the adjoint recurrence backwards through it.
// storage-order core of ks_block_solve_vjp: B, X0, xb in; X, g_q, Bbar out
static int vjp_core(ks_ctx *c, const double *B, const double *X0, int k, double tol, int max_it, int seg,
                    const double *xb, double *X, double *g_q, double *Bbar, int32_t *iters_host) {
  if (seg <= 0) seg = 8;
  hipStream_t s = c->s;
  const int N = c->N;
  const size_t nk = (size_t)N * k;
  // device work: B, X0, X, R, P, Z, Q, xbar, Rbar, Pbar, Zbar, Qbar, T, dbar, coefficients,
  // checkpoints (grown as needed) and one segment of (R, P)
  std::vector<void *> bufs;
  auto dalloc = [&](size_t n) -> double * {
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(double) * std::max<size_t>(n, 1)) != hipSuccess) return nullptr;
    bufs.push_back(p);
    return static_cast<double *>(p);
  };
  struct Release {
    std::vector<void *> &b;
    ~Release() {
      for (void *p : b) (void)hipFree(p);
    }
  } release{bufs};
  double *R = dalloc(nk), *P = dalloc(nk), *Z = dalloc(nk);
  double *Q = dalloc(nk), *Rb = dalloc(nk), *Pb = dalloc(nk), *Zb = dalloc(nk), *Qb = dalloc(nk);
  double *T = dalloc(nk), *dbar = dalloc(N), *coef = dalloc((size_t)16 * k);
  double *segR = dalloc(nk * (seg + 1)), *segP = dalloc(nk * (seg + 1));
  if (!R || !P || !Z || !Q || !Rb || !Pb || !Zb || !Qb || !T || !dbar || !coef || !segR || !segP)
    return fail(KS_ERR_NOMEM, "ks_block_solve_vjp: hipMalloc failed");
  std::vector<double *> ckR, ckP;
  const double *d = c->diagS;
  // host-side coefficient slots: slot i of coef holds k values
  std::vector<std::vector<double>> hc(16, std::vector<double>(k));
  auto put = [&](int slot, const std::vector<double> &v) -> const double * {
    hc[slot] = v;
    (void)hipMemcpyAsync(coef + (size_t)slot * k, hc[slot].data(), sizeof(double) * k, hipMemcpyHostToDevice, s);
    return coef + (size_t)slot * k;
  };
  auto dots = [&](const double *A, const double *Bm, std::vector<double> &out) -> int {
    const int nb = launch_coldots(N, k, A, Bm, c->redpart, s);
    out.assign(k, 0.0);
    return reduce_small(c, c->redpart, nb, k, out.data());
  };
  auto norms = [&](const double *A, std::vector<double> &out) -> int {
    const int nb = launch_colnorms(N, k, A, c->redpart, s);
    out.assign(k, 0.0);
    TRY(reduce_small(c, c->redpart, nb, k, out.data()));
    for (auto &v : out) v = std::sqrt(v);
    return KS_OK;
  };
  const std::vector<double> ones(k, 1.0), zeros(k, 0.0);
  // forward: r_0 = b - S x_0, z_0 = D^-1 r_0, p_0 = z_0, rho_0 = r_0.z_0
  launch_axpby((int64_t)nk, 1.0, X0, 0.0, X, s);
  spmm_op(c, c->S, X, k, R, B);
  launch_row_div(N, k, R, d, Z, s);
  launch_axpby((int64_t)nk, 1.0, Z, 0.0, P, s);
  std::vector<double> rho, bn, rn;
  TRY(dots(R, Z, rho));
  TRY(norms(B, bn));
  TRY(norms(R, rn));
  std::vector<char> active(k);
  for (int j = 0; j < k; ++j) active[j] = rn[j] > tol * bn[j];
  struct Step {
    std::vector<char> act;
    std::vector<double> alpha, beta, rho, sig;
  };
  std::vector<Step> steps;
  auto checkpoint = [&]() -> int {
    double *r = dalloc(nk), *p = dalloc(nk);
    if (!r || !p) return fail(KS_ERR_NOMEM, "ks_block_solve_vjp: hipMalloc failed");
    launch_axpby((int64_t)nk, 1.0, R, 0.0, r, s);
    launch_axpby((int64_t)nk, 1.0, P, 0.0, p, s);
    ckR.push_back(r);
    ckP.push_back(p);
    return KS_OK;
  };
  TRY(checkpoint());
  // one forward iteration from (Rc, Pc) into (Rn, Pn) with the step's coefficients
  auto advance = [&](const Step &st, const double *Rc, const double *Pc, double *Rn, double *Pn, bool keep_z) {
    spmm_op(c, c->S, Pc, k, Q, nullptr);
    if (Rn != Rc) launch_axpby((int64_t)nk, 1.0, Rc, 0.0, Rn, s);
    std::vector<double> ma(k), pa(k), pb(k);
    for (int j = 0; j < k; ++j) {
      ma[j] = -st.alpha[j];
      pa[j] = st.act[j] ? 1.0 : 0.0;
      pb[j] = st.act[j] ? st.beta[j] : 1.0;
    }
    launch_col_axpby(N, k, put(0, ma), Q, put(1, ones), Rn, s);
    launch_row_div(N, k, Rn, d, Z, s);
    if (Pn != Pc) launch_axpby((int64_t)nk, 1.0, Pc, 0.0, Pn, s);
    launch_col_axpby(N, k, put(2, pa), Z, put(3, pb), Pn, s);
    (void)keep_z;
    (void)hipStreamSynchronize(s);  // the host coefficient slots are reused by the next call
  };
  for (int it = 0; it < max_it; ++it) {
    bool any = false;
    for (int j = 0; j < k; ++j) any = any || active[j];
    if (!any) break;
    Step st;
    st.act = active;
    st.rho = rho;
    spmm_op(c, c->S, P, k, Q, nullptr);
    TRY(dots(P, Q, st.sig));
    st.alpha.assign(k, 0.0);
    for (int j = 0; j < k; ++j)
      if (active[j]) st.alpha[j] = rho[j] / st.sig[j];
    launch_col_axpby(N, k, put(4, st.alpha), P, put(5, ones), X, s);
    // R, Z, P as advance() recomputes them (Q already holds S P)
    std::vector<double> ma(k);
    for (int j = 0; j < k; ++j) ma[j] = -st.alpha[j];
    launch_col_axpby(N, k, put(0, ma), Q, put(1, ones), R, s);
    launch_row_div(N, k, R, d, Z, s);
    std::vector<double> rho_n;
    TRY(dots(R, Z, rho_n));
    st.beta.assign(k, 0.0);
    std::vector<double> pa(k), pb(k);
    for (int j = 0; j < k; ++j) {
      if (active[j]) st.beta[j] = rho_n[j] / rho[j];
      pa[j] = active[j] ? 1.0 : 0.0;
      pb[j] = active[j] ? st.beta[j] : 1.0;
    }
    launch_col_axpby(N, k, put(2, pa), Z, put(3, pb), P, s);
    for (int j = 0; j < k; ++j)
      if (active[j]) rho[j] = rho_n[j];
    steps.push_back(st);
    if ((int)steps.size() % seg == 0) TRY(checkpoint());
    TRY(norms(R, rn));
    for (int j = 0; j < k; ++j) active[j] = active[j] && rn[j] > tol * bn[j];
  }
  const int K = (int)steps.size();
  if (iters_host)
    for (int j = 0; j < k; ++j) {
      int n = 0;
      for (const Step &st : steps) n += st.act[j] ? 1 : 0;
      iters_host[j] = n;
    }
  // reverse sweep
  launch_fill((int64_t)nk, 0.0, Rb, s);
  launch_fill((int64_t)nk, 0.0, Pb, s);
  launch_fill(N, 0.0, dbar, s);
  launch_fill((int64_t)c->n_e * c->n_q, 0.0, g_q, s);
  std::vector<double> rhobar(k, 0.0);
  const int nseg = (K + seg - 1) / seg;
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int j0 = sg * seg, j1 = std::min(K, j0 + seg);
    // recompute the segment's iterates from its checkpoint
    launch_axpby((int64_t)nk, 1.0, ckR[sg], 0.0, segR, s);
    launch_axpby((int64_t)nk, 1.0, ckP[sg], 0.0, segP, s);
    for (int j = j0; j < j1; ++j)
      advance(steps[j], segR + nk * (j - j0), segP + nk * (j - j0), segR + nk * (j + 1 - j0),
              segP + nk * (j + 1 - j0), false);
    for (int j = j1 - 1; j >= j0; --j) {
      const Step &st = steps[j];
      const double *p = segP + nk * (j - j0), *r1 = segR + nk * (j + 1 - j0);
      spmm_op(c, c->S, p, k, Q, nullptr);
      launch_row_div(N, k, r1, d, Z, s);  // z_{j+1}
      std::vector<double> a(k), betabar, alphabar, t1, t2;
      for (int i = 0; i < k; ++i) a[i] = st.act[i] ? 1.0 : 0.0;
      // p_{j+1} = z_{j+1} + beta p_j
      launch_col_axpby(N, k, put(0, a), Pb, put(1, zeros), Zb, s);
      TRY(dots(Pb, p, betabar));
      std::vector<double> pbs(k);
      for (int i = 0; i < k; ++i) {
        betabar[i] *= a[i];
        pbs[i] = st.act[i] ? st.beta[i] : 1.0;
      }
      launch_col_axpby(N, k, nullptr, nullptr, put(2, pbs), Pb, s);
      // beta = rho_{j+1} / rho_j; rho_{j+1} = r_{j+1}.z_{j+1}
      std::vector<double> rho1b(k), rhojb(k);
      for (int i = 0; i < k; ++i) {
        rho1b[i] = st.act[i] ? rhobar[i] + betabar[i] / st.rho[i] : 0.0;
        rhojb[i] = st.act[i] ? -betabar[i] * st.beta[i] / st.rho[i] : 0.0;
      }
      launch_col_axpby(N, k, put(3, rho1b), Z, put(4, ones), Rb, s);
      launch_col_axpby(N, k, put(5, rho1b), r1, put(6, ones), Zb, s);
      // z_{j+1} = D^-1 r_{j+1}
      launch_zbar_back(N, k, Zb, Z, d, Rb, dbar, s);
      // r_{j+1} = r_j - alpha q; x_{j+1} = x_j + alpha p
      TRY(dots(Rb, Q, t1));
      TRY(dots(xb, p, t2));
      alphabar.assign(k, 0.0);
      std::vector<double> malpha(k);
      for (int i = 0; i < k; ++i) {
        alphabar[i] = st.act[i] ? -t1[i] + t2[i] : 0.0;
        malpha[i] = -st.alpha[i];
      }
      launch_col_axpby(N, k, put(7, malpha), Rb, put(8, zeros), Qb, s);
      launch_col_axpby(N, k, put(9, st.alpha), xb, put(10, ones), Pb, s);
      // alpha = rho_j / sigma_j; sigma = p.q
      std::vector<double> sigb(k);
      for (int i = 0; i < k; ++i) {
        rhojb[i] += st.act[i] ? alphabar[i] / st.sig[i] : 0.0;
        sigb[i] = st.act[i] ? -alphabar[i] * st.alpha[i] / st.sig[i] : 0.0;
      }
      launch_col_axpby(N, k, put(11, sigb), Q, put(12, ones), Pb, s);
      launch_col_axpby(N, k, put(13, sigb), p, put(14, ones), Qb, s);
      // q = S p: pbar += S qbar, Sbar += qbar p^T -> g
      spmm_op(c, c->S, Qb, k, T, nullptr);
      launch_axpby((int64_t)nk, 1.0, T, 1.0, Pb, s);
      launch_pair_accum(c->edof, c->n_loc, c->n_e, c->n_q, c->phi, c->qw, c->absdet, Qb, p, k, 1.0, g_q, s);
      for (int i = 0; i < k; ++i)
        if (st.act[i]) rhobar[i] = rhojb[i];
      HIPCHK(hipStreamSynchronize(s));  // the coefficient slots are reused next step
    }
  }
  // start: rho_0 = r_0.z_0, p_0 = z_0, z_0 = D^-1 r_0, r_0 = b - S x_0
  const double *r0 = ckR[0];
  launch_row_div(N, k, r0, d, Z, s);
  launch_col_axpby(N, k, put(0, rhobar), Z, put(1, ones), Rb, s);
  launch_axpby((int64_t)nk, 1.0, Pb, 0.0, Zb, s);
  launch_col_axpby(N, k, put(2, rhobar), r0, put(3, ones), Zb, s);
  launch_zbar_back(N, k, Zb, Z, d, Rb, dbar, s);
  if (Bbar) launch_axpby((int64_t)nk, 1.0, Rb, 0.0, Bbar, s);
  launch_pair_accum(c->edof, c->n_loc, c->n_e, c->n_q, c->phi, c->qw, c->absdet, Rb, X0, k, -1.0, g_q, s);
  launch_pair_accum(c->edof, c->n_loc, c->n_e, c->n_q, c->phi, c->qw, c->absdet, nullptr, dbar, 1, 1.0, g_q, s);
  HIPCHK(hipStreamSynchronize(s));
  return KS_OK;
}

extern "C" int ks_block_solve_vjp(ks_ctx *c, const double *B_api, const double *X0_api, int32_t k, double tol,
                                  int32_t max_it, int32_t seg, const double *Xbar_api, double *X_api, double *g_q,
                                  double *Bbar_api, int32_t *iters_host) {
  if (!c || !B_api || !Xbar_api || !X_api || !g_q || !Bbar_api) return fail(KS_ERR_ARG, "null argument");
  if (k < 1 || k > c->k_max) return fail(KS_ERR_ARG, "k must be in 1..k_max");
  if (!(tol >= 0.0) || max_it < 1) return fail(KS_ERR_ARG, "need tol >= 0 and max_it >= 1");
  if (!c->have_S) return fail(KS_ERR_STATE, "no operator assembled: call ks_assemble first");
  hipStream_t s = c->s;
  const int N = c->N;
  const size_t nk = (size_t)N * k;
  double *buf = nullptr;
  if (hipMalloc(&buf, sizeof(double) * 5 * nk) != hipSuccess) return fail(KS_ERR_NOMEM, "hipMalloc failed");
  struct Free {
    double *p;
    ~Free() { (void)hipFree(p); }
  } guard{buf};
  double *B = buf, *X0 = buf + nk, *xb = buf + 2 * nk, *X = buf + 3 * nk, *Bb = buf + 4 * nk;
  launch_rows_to_storage(N, k, B_api, B, c->int2nat, s);
  if (X0_api) launch_rows_to_storage(N, k, X0_api, X0, c->int2nat, s);
  else launch_fill((int64_t)nk, 0.0, X0, s);
  launch_rows_to_storage(N, k, Xbar_api, xb, c->int2nat, s);
  TRY(vjp_core(c, B, X0, k, tol, max_it, seg, xb, X, g_q, Bb, iters_host));
  launch_rows_to_api(N, k, X, X_api, c->int2nat, s);
  launch_rows_to_api(N, k, Bb, Bbar_api, c->int2nat, s);
  HIPCHK(hipStreamSynchronize(s));
  return KS_OK;
}

extern "C" int ks_block_solve(ks_ctx *c, const double *psi_old, const double *lambda_host, int32_t k,
                              int32_t precision, double *psi_hat, ks_solve_stats *st) {
  if (!c || !psi_old || !lambda_host || !psi_hat) return fail(KS_ERR_ARG, "null argument");
  if (k < 1 || k > c->k_max) return fail(KS_ERR_ARG, "k must be in 1..k_max");
  if (precision != KS_PREC_FP64 && precision != KS_PREC_MIXED && precision != KS_PREC_FP64_BLOCK_CG)
    return fail(KS_ERR_ARG, "bad precision");
  launch_rows_to_storage(c->N, k, psi_old, c->PsiIn, c->int2nat, c->s);
  TRY(build_rhs(c, c->PsiIn, lambda_host, k, c->Bv));
  HIPCHK(hipMemcpyAsync(c->Xs, c->PsiIn, sizeof(double) * c->N * k, hipMemcpyDeviceToDevice, c->s));
  const int r = solve_impl(c, c->Bv, c->Xs, k, precision, c->opt.tol_solve, st);
  if (r < 0) return r;
  launch_rows_to_api(c->N, k, c->Xs, psi_hat, c->int2nat, c->s);
  HIPCHK(hipStreamSynchronize(c->s));
  return r;
}

// -------------------------------------------------------- augmented basis
// Z[:, N_H : N_H + k] = psi_hat - P G^{-1} P^T M psi_hat ; zero padding after.
static int build_tail(ks_ctx *c, const double *psi_hat, int k) {
  hipStream_t s = c->s;
  const int N = c->N, nH = c->N_H;
  spmm_op(c, c->M, psi_hat, k, c->Wv, nullptr);
  launch_gemm_tn(N, nH, k, c->Z, c->mp, c->Wv, k, c->Ctmp, k, c->gwork, c->gwork_n, s);
  launch_small_gemm(nH, k, nH, c->GPPinv, nH, c->Ctmp, k, c->Ttmp, k, 0.0, s);
  launch_ellP_times(N, c->Pidx, c->Pw, c->Ttmp, k, k, -1.0, psi_hat, k, c->Z + nH, c->mp, s);
  if (nH + k < c->mp) launch_zero_cols(N, nH + k, c->mp, c->Z, c->mp, s);
  return KS_OK;
}

// F (m x m, ld m) = Z^T H Z with the P-P block taken from PP if given
static void project_full(ks_ctx *c, const double *H, int m, double *F) {
  // columns m.. of Z are zero: an even count keeps two-column vector lanes
  spmm_cols(c, H, c->Z, c->mp, c->Y, c->mp, std::min(c->mp, (m + 1) & ~1));
  launch_gemm_tn_sym(c->N, m, c->Z, c->mp, c->Y, c->mp, F, m, c->gwork, c->s);
}
// F (m x m, ld m) = Z^T H Z for the inner iteration's H = M[V_nl]: the
// blocks P^T H P and P^T H T from the ELL form of P (launch_proj_coarse),
// T^T H T on the FP64 matrix cores; the dense product over all of Z where
// the coarse blocks do not fit
static void project_nl(ks_ctx *c, const double *H, int k, double *F) {
  const int m = c->N_H + k, nH = c->N_H;
  if (c->cp_ok) {
    spmm_cols(c, H, c->Z + nH, c->mp, c->Wv, k, k);  // Y = H T
    launch_gemm_tn_sym(c->N, k, c->Z + nH, c->mp, c->Wv, k, c->Ttmp, k, c->gwork, c->s);
    if (launch_proj_coarse(c->N, nH, k, c->k_max, c->cp_nblk, c->cp_ldt, c->cp_ldo, c->rowptr, c->col, H, c->Pidx,
                           c->Pw, c->Wv, c->cp_uoff, c->cp_ulist, c->cp_noff, c->cp_nlist, c->cp_ppoff, c->cp_ptoff,
                           c->cp_pp, c->cp_pt, c->cp_gpp_ptr, c->cp_gpp_idx, c->cp_gpt_ptr, c->cp_gpt_idx, F, m,
                           c->s) == 0) {
      launch_copy_cols(k, k, c->Ttmp, k, F + (size_t)nH * m, m, nH, c->s);  // T^T H T
      return;
    }
  }
  project_full(c, H, m, F);
}
// F from the fixed P-P block and the tail columns Z^T (H psi_tilde)
static void project_tail(ks_ctx *c, const double *H, const double *PP, int k, double *F) {
  const int m = c->N_H + k;
  spmm_cols(c, H, c->Z + c->N_H, c->mp, c->Wv, k, k);
  launch_gemm_tn(c->N, m, k, c->Z, c->mp, c->Wv, k, c->Ftail, k, c->gwork, c->gwork_n, c->s);
  launch_fill_pencil(m, c->N_H, PP, c->Ftail, F, c->s);
}

extern "C" int ks_augmented_project(ks_ctx *c, const double *psi_hat, int32_t k, int32_t which,
                                    double *F) {
  if (!c || !psi_hat || !F) return fail(KS_ERR_ARG, "null argument");
  if (k < 1 || k > c->k_max) return fail(KS_ERR_ARG, "k must be in 1..k_max");
  const double *H = nullptr;
  if (which == 0) H = c->M;
  else if (which == 1) H = c->AL;
  else if (which == 2) {
    if (!c->have_S) return fail(KS_ERR_STATE, "no assembly");
    assemble_potential_all(c, c->vnl_q, c->MNL);
    H = c->MNL;
  } else
    return fail(KS_ERR_ARG, "which must be 0, 1 or 2");
  c->have_step = false;
  launch_rows_to_storage(c->N, k, psi_hat, c->PsiIn, c->int2nat, c->s);
  TRY(build_tail(c, c->PsiIn, k));
  project_full(c, H, c->N_H + k, F);
  HIPCHK(hipStreamSynchronize(c->s));
  return KS_OK;
}

// ---------------------------------------------------------------- eigen
// Orthogonalise the pencil's F_B (once per augmented space); rank in c->e_rank.
static int orth_impl(ks_ctx *c, const double *FB, int m) {
  if (!packed_eig_supported(m)) {
    c->e_m = 0;
    return KS_OK;  // the one-stage fallback handles it per call
  }
  HIPCHK(hipMemsetAsync(c->einfo, 0, 8 * sizeof(int), c->s));
  if (launch_orth(m, FB, m, c->eD, c->eV, c->eX, c->eRot, c->einfo, c->s) < 0)
    return fail(KS_ERR_HIP, "cannot enable the LDS size of the eigensolver");
  int info[8];
  HIPCHK(hipMemcpyAsync(info, c->einfo, sizeof(int) * 8, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  if (info[2]) return fail(KS_ERR_EIG, "F_B has a non-positive diagonal entry");
  c->e_rank = info[0];
  c->e_m = m;
  return KS_OK;
}

// Lowest k eigenpairs of (FA, FB) (FB orthogonalised by orth_impl); warm:
// start from the eigenvectors of the previous call on the same F_B.
static int eig_impl(ks_ctx *c, const double *FA, const double *FB, int m, int k, double *U,
                    std::vector<double> &theta_all, int *rank, bool warm = false) {
  if (!packed_eig_supported(m)) {
    HIPCHK(hipMemsetAsync(c->einfo, 0, 8 * sizeof(int), c->s));
    launch_small_eig(m, k, FA, m, FB, m, c->eigwork, c->theta, U, c->einfo, c->s);
    int info[8];
    theta_all.resize(m);
    HIPCHK(hipMemcpyAsync(info, c->einfo, sizeof(int) * 8, hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipMemcpyAsync(theta_all.data(), c->theta, sizeof(double) * m, hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    if (info[2]) return fail(KS_ERR_EIG, "F_B has a non-positive diagonal entry");
    if (info[0] < k) return fail(KS_ERR_EIG, "augmented space has rank " + std::to_string(info[0]) + " < k");
    theta_all.resize(info[0]);
    if (rank) *rank = info[0];
    return KS_OK;
  }
  if (c->e_m != m) TRY(orth_impl(c, FB, m));
  const int r = c->e_rank;
  if (r < k) return fail(KS_ERR_EIG, "augmented space has rank " + std::to_string(r) + " < k");
  if (launch_reduced_eig_split(m, k, r, FA, m, c->eD, c->eX, c->eW, warm ? 1 : 0, c->eS, c->eT1, c->eT2,
                               c->eRot, c->eLam, c->theta, U, c->einfo + 4, c->s) < 0)
    return fail(KS_ERR_HIP, "cannot enable the LDS size of the eigensolver");
  theta_all.resize(r);
  HIPCHK(hipMemcpyAsync(theta_all.data(), c->theta, sizeof(double) * r, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  if (rank) *rank = r;
  return KS_OK;
}

extern "C" int ks_small_eig(ks_ctx *c, const double *FA, const double *FB, int32_t m, int32_t k,
                            double *U, double *lambda_host, int32_t *rank_host) {
  if (!c || !FA || !FB || !U || !lambda_host) return fail(KS_ERR_ARG, "null argument");
  if (m < 1 || m > 256 || k < 1 || k > m || m > c->mp) return fail(KS_ERR_ARG, "bad sizes");
  std::vector<double> th;
  int rank = 0;
  c->have_step = false;
  TRY(orth_impl(c, FB, m));
  TRY(eig_impl(c, FA, FB, m, k, U, th, &rank));
  for (int j = 0; j < k; ++j) lambda_host[j] = th[j];
  if (rank_host) *rank_host = rank;
  return KS_OK;
}

extern "C" int ks_initial_guess(ks_ctx *c, int32_t k, double *psi, double *lambda_host) {
  if (!c || !psi || !lambda_host) return fail(KS_ERR_ARG, "null argument");
  if (k < 1 || k > c->k_max || k > c->N_H) return fail(KS_ERR_ARG, "bad k");
  std::vector<double> th;
  int rank = 0;
  c->have_step = false;
  TRY(orth_impl(c, c->GPP, c->N_H));
  TRY(eig_impl(c, c->FAL_PP, c->GPP, c->N_H, k, c->U, th, &rank));
  launch_ellP_times(c->N, c->Pidx, c->Pw, c->U, k, k, 1.0, nullptr, 0, c->Xs, k, c->s);
  launch_rows_to_api(c->N, k, c->Xs, psi, c->int2nat, c->s);
  for (int j = 0; j < k; ++j) lambda_host[j] = th[j];
  HIPCHK(hipStreamSynchronize(c->s));
  return KS_OK;
}

// ---------------------------------------------------------------- SCF step
static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Anderson mixing (Sec. 4): coefficients from the normal equations of
// min ||F~||, new input = rho~_in + beta F~.
static int solve_small_spd(int n, std::vector<double> A, std::vector<double> b, std::vector<double> &x) {
  x.assign(n, 0.0);
  for (int p = 0; p < n; ++p) {
    int piv = p;
    for (int r = p + 1; r < n; ++r)
      if (std::fabs(A[r * n + p]) > std::fabs(A[piv * n + p])) piv = r;
    if (!(std::fabs(A[piv * n + p]) > 0.0)) return -1;
    if (piv != p) {
      for (int j = 0; j < n; ++j) std::swap(A[p * n + j], A[piv * n + j]);
      std::swap(b[p], b[piv]);
    }
    for (int r = p + 1; r < n; ++r) {
      const double f = A[r * n + p] / A[p * n + p];
      for (int j = p; j < n; ++j) A[r * n + j] -= f * A[p * n + j];
      b[r] -= f * b[p];
    }
  }
  for (int p = n - 1; p >= 0; --p) {
    double t = b[p];
    for (int j = p + 1; j < n; ++j) t -= A[p * n + j] * x[j];
    x[p] = t / A[p * n + p];
  }
  return 0;
}

// Anderson mixing of the density (Sec. 4, eqs. mix2-mix6), shared by the
// inner iteration of a step and the direct SCF.  A ring of (rho_in, F =
// rho_out - rho_in) pairs lives in the context's history slots.
struct AndersonRing {
  int nhist = 0, head = 0;
  int nh = 0, jidx[4] = {0, 0, 0, 0};
  double g[21] = {};
};
// Record the pass (rho_in, rho_out) and return ||rho_out - rho_in||_0 in *res.
static int anderson_record(ks_ctx *c, AndersonRing &a, const double *rho_out, const double *rho_in, double *res) {
  hipStream_t s = c->s;
  const int64_t nqt = (int64_t)c->n_e * c->n_q;
  const int depth = c->opt.anderson_depth;
  double *Fm = c->hist_F[a.head], *Im = c->hist_in[a.head];
  launch_combine3(nqt, 1.0, rho_out, -1.0, rho_in, 0.0, nullptr, Fm, s);
  HIPCHK(hipMemcpyAsync(Im, rho_in, sizeof(double) * nqt, hipMemcpyDeviceToDevice, s));
  a.nh = std::min(a.nhist, depth - 1);  // previous iterates used
  const double *Fj[4];
  for (int j = 0; j < a.nh; ++j) {
    // oldest first: j = 0 is the oldest kept
    a.jidx[j] = (a.head - a.nh + j + depth) % depth;
    Fj[j] = c->hist_F[a.jidx[j]];
  }
  int nb = launch_anderson_gram(nqt, c->n_q, c->absdet, c->qw, Fm, a.nh, Fj, c->redpart, s);
  TRY(reduce_small(c, c->redpart, nb, 21, a.g));
  *res = std::sqrt(std::max(a.g[0], 0.0));
  return KS_OK;
}
// The next input density from the ring (after anderson_record) into rho_in.
static int anderson_mix_next(ks_ctx *c, AndersonRing &a, double *rho_in) {
  hipStream_t s = c->s;
  const int64_t nqt = (int64_t)c->n_e * c->n_q;
  const int depth = c->opt.anderson_depth;
  const int nh = a.nh;
  std::vector<double> alpha;
  if (nh > 0) {
    std::vector<double> G(nh * nh), b(nh);
    double tr = 0.0;
    for (int j = 0; j < nh; ++j) {
      b[j] = a.g[1 + j];
      for (int l = 0; l < nh; ++l) G[j * nh + l] = a.g[5 + 4 * j + l];
      tr += G[j * nh + j];
    }
    for (int j = 0; j < nh; ++j) G[j * nh + j] += 1e-12 * std::max(tr, 1e-300);
    if (solve_small_spd(nh, G, b, alpha) < 0) alpha.assign(nh, 0.0);
  }
  // new rho_in = sum coef * {in_j, F_j}
  const double beta = c->opt.anderson_beta;
  double sa = 0.0;
  for (int j = 0; j < nh; ++j) sa += alpha[j];
  double coefs[12];
  const double *vecs[12];
  int nv = 0;
  coefs[nv] = 1.0 - sa; vecs[nv++] = c->hist_in[a.head];
  coefs[nv] = beta * (1.0 - sa); vecs[nv++] = c->hist_F[a.head];
  for (int j = 0; j < nh; ++j) {
    coefs[nv] = alpha[j]; vecs[nv++] = c->hist_in[a.jidx[j]];
    coefs[nv] = beta * alpha[j]; vecs[nv++] = c->hist_F[a.jidx[j]];
  }
  HIPCHK(hipMemcpyAsync(c->coef, coefs, sizeof(double) * nv, hipMemcpyHostToDevice, s));
  launch_lincomb(nqt, nv, c->coef, vecs, rho_in, s);
  a.head = (a.head + 1) % depth;
  a.nhist = std::min(a.nhist + 1, depth);
  return KS_OK;
}

extern "C" int ks_scf_step(ks_ctx *c, double *psi, double *lambda_host, int32_t k,
                           const double *occ_host, int32_t precision, double *rho_q,
                           ks_step_report *rep) {
  if (!c || !psi || !lambda_host || !occ_host) return fail(KS_ERR_ARG, "null argument");
  if (k < 1 || k > c->k_max) return fail(KS_ERR_ARG, "k must be in 1..k_max");
  if (precision != KS_PREC_FP64 && precision != KS_PREC_MIXED && precision != KS_PREC_FP64_BLOCK_CG)
    return fail(KS_ERR_ARG, "bad precision");
  hipStream_t s = c->s;
  const std::vector<double> lambda_in(lambda_host, lambda_host + k);  // the step's input eigenvalues
  ks_step_report R;
  std::memset(&R, 0, sizeof(R));
  const double t0 = now_s();
  const int N = c->N, nH = c->N_H, m = nH + k;
  const int64_t nqt = (int64_t)c->n_e * c->n_q;
  const bool hartree = c->opt.hartree_mode != KS_HARTREE_OFF;
  const bool nonlinear = hartree || c->opt.xc_mode != KS_XC_NONE;
  // 1. S of the input density (w_D frozen from here on)
  int piters = 0;
  launch_rows_to_storage(N, k, psi, c->PsiIn, c->int2nat, s);
  TRY(assemble_impl(c, c->PsiIn, k, occ_host, &piters, precision == KS_PREC_MIXED));
  HIPCHK(hipStreamSynchronize(s));
  const double t1 = now_s();
  // 2. BVPs
  TRY(build_rhs(c, c->PsiIn, lambda_host, k, c->Bv));
  HIPCHK(hipMemcpyAsync(c->PsiHat, c->PsiIn, sizeof(double) * N * k, hipMemcpyDeviceToDevice, s));
  int st = solve_impl(c, c->Bv, c->PsiHat, k, precision, c->opt.tol_solve, &R.solve);
  if (st < 0) return st;
  R.status_solve = st;
  const double t2 = now_s();
  // 3. augmented basis and the fixed blocks of the pencil
  TRY(build_tail(c, c->PsiHat, k));
  project_tail(c, c->M, c->GPP, k, c->FB);
  project_tail(c, c->AL, c->FAL_PP, k, c->FAL);
  TRY(orth_impl(c, c->FB, m));
  const double t3 = now_s();
  // 4. inner nonlinear iteration
  HIPCHK(hipMemcpyAsync(c->rho_in, c->rho_l, sizeof(double) * nqt, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(c->occ_d, occ_host, sizeof(double) * k, hipMemcpyHostToDevice, s));
  AndersonRing ring;
  std::vector<double> th;
  double res = 0.0;
  int it = 0, rank = 0;
  for (it = 0; it < c->opt.max_it_inner; ++it) {
    if (nonlinear) {
      if (hartree) {
        // the inner fixed point cannot settle below the error the inexact
        // Poisson solves leave in V_H: their tolerance follows the inner
        // residual (1e-4 of the last one, between 1e-4 tol_inner and
        // tol_poisson), so the last iterations solve to 1e-4 tol_inner
        const double tol_p =
            std::max(1e-4 * c->opt.tol_inner, std::min(c->opt.tol_poisson, it > 0 ? 1e-4 * res : INFINITY));
        int r = hartree_solve(c, c->rho_in, &piters, std::min(c->opt.tol_poisson, tol_p));
        if (r < 0) return r;
      } else {
        launch_fill(nqt, 0.0, c->vh_q, s);
      }
      launch_xc(nqt, c->rho_in, c->opt.xc_mode, c->exc_q, c->vxc_q, s);
      launch_add(nqt, c->vh_q, c->vxc_q, c->vnl_q, s);
      assemble_potential_all(c, c->vnl_q, c->MNL);
      project_nl(c, c->MNL, k, c->Ctmp);
      launch_combine3((int64_t)m * m, 1.0, c->FAL, 1.0, c->Ctmp, 0.0, nullptr, c->FA, s);
    } else {
      HIPCHK(hipMemcpyAsync(c->FA, c->FAL, sizeof(double) * m * m, hipMemcpyDeviceToDevice, s));
    }
    TRY(eig_impl(c, c->FA, c->FB, m, k, c->U, th, &rank, it > 0));
    launch_zu(N, c->Pidx, c->Pw, nH, c->Z, c->mp, k, c->U, k, c->PsiNew, s);
    launch_density(c->edof, c->n_loc, c->n_e, c->n_q, c->phi, c->PsiNew, k, k, c->occ_d,
                   c->rho_out, s);
    if (!nonlinear) {
      it += 1;
      break;
    }
    TRY(anderson_record(c, ring, c->rho_out, c->rho_in, &res));
    if (std::getenv("KS_TRACE_INNER")) {
      int info[8] = {0};
      (void)hipMemcpy(info, c->einfo, sizeof(int) * 8, hipMemcpyDeviceToHost);
      std::fprintf(stderr, "[ks-inner] it %d res %.3e jacobi_sweeps %d poisson_iters %d\n", it, res, info[5],
                   piters);
    }
    // converged, or the last permitted pass: no mixing, so the energies
    // below pair rho_in with the potentials it produced (Sec. 3.1)
    if (res < c->opt.tol_inner || it + 1 == c->opt.max_it_inner) {
      it += 1;
      break;
    }
    TRY(anderson_mix_next(c, ring, c->rho_in));
  }
  R.inner_iters = it;
  R.res_inner = res;
  R.rank = rank;
  const double t4 = now_s();
  // 5. outputs and energies
  launch_rows_to_api(N, k, c->PsiNew, psi, c->int2nat, s);
  if (rho_q) HIPCHK(hipMemcpyAsync(rho_q, c->rho_out, sizeof(double) * nqt, hipMemcpyDeviceToDevice, s));
  double band = 0.0;
  for (int j = 0; j < k; ++j) {
    lambda_host[j] = th[j];
    band += occ_host[j] * th[j];
  }
  R.E_band = band;
  R.E_nn = c->E_nn;
  if (nonlinear) {
    const double *a[3] = {c->vh_q, c->exc_q, c->vxc_q};
    const double *b[3] = {c->rho_in, c->rho_in, c->rho_in};
    double e[3];
    TRY(weighted_dots(c, 3, a, b, e));
    R.E_H = 0.5 * e[0];
    R.E_xc = e[1];
    R.E_vxc = e[2];
  }
  R.E_total = R.E_band - R.E_H - R.E_vxc + R.E_xc + R.E_nn;
  R.poisson_iters = piters;
  {
    // ||rho^{l+1} - rho^l||_0, the outer stopping quantity of Algorithm 3
    launch_combine3(nqt, 1.0, c->rho_out, -1.0, c->rho_l, 0.0, nullptr, c->drho, s);
    const double *d[1] = {c->drho};
    double v = 0.0;
    TRY(weighted_dots(c, 1, d, d, &v));
    R.res_outer = std::sqrt(std::max(v, 0.0));
  }
  HIPCHK(hipStreamSynchronize(s));
  const double t5 = now_s();
  R.seconds[0] = t1 - t0;
  R.seconds[1] = t2 - t1;
  R.seconds[2] = t3 - t2;
  R.seconds[3] = t4 - t3;
  R.seconds[4] = t5 - t4;
  R.seconds[5] = t5 - t0;
  if (rep) *rep = R;
  c->have_step = true;
  c->last_nonlinear = nonlinear;
  c->last_inner_converged = !nonlinear || res < c->opt.tol_inner;
  c->last_k = k;
  c->last_lam_in.assign(lambda_in.begin(), lambda_in.end());
  c->last_precision = precision;
  c->last_theta.assign(th.begin(), th.begin() + k);
  c->last_occ.assign(occ_host, occ_host + k);
  int ret = KS_OK;
  if ((int)th.size() > k && th[k] - th[k - 1] < 1e-8) ret = KS_WARN_DEGENERATE;
  if (nonlinear && res >= c->opt.tol_inner) ret = KS_NOT_CONVERGED;
  if (st == KS_NOT_CONVERGED) ret = KS_NOT_CONVERGED;
  return ret;
}

// ------------------------------------------------------ mesh to mesh
// Algorithm 1 (Sec. 3.2) between two meshes: this context's interior nodes
// located in a P1 source mesh (bucket-grid nearest vertex, barycentric
// walk), the orbitals interpolated with the barycentric weights.
extern "C" int ks_interpolate(ks_ctx *c, const ks_mesh_desc *src, const double *psi_src, int32_t k,
                              int32_t orthonormalize, double *psi) {
  if (!c || !src || !psi_src || !psi || !src->coords_host || !src->elems_host || !src->dirichlet_host)
    return fail(KS_ERR_ARG, "null argument");
  if (src->order != 1) return fail(KS_ERR_ARG, "the source mesh must be P1");
  if (k < 1 || k > c->k_max) return fail(KS_ERR_ARG, "k must be in 1..k_max");
  if (src->n_nodes < 4 || src->n_elems < 1) return fail(KS_ERR_ARG, "empty source mesh");
  for (int64_t i = 0; i < (int64_t)src->n_elems * 4; ++i)
    if (src->elems_host[i] < 0 || src->elems_host[i] >= src->n_nodes) return fail(KS_ERR_MESH, "source node id out of range");
  hipStream_t s = c->s;
  const int N = c->N;
  // source unknowns: the non-Dirichlet nodes in ascending order
  std::vector<int32_t> sint(src->n_nodes, -1);
  int ns = 0;
  for (int v = 0; v < src->n_nodes; ++v)
    if (!src->dirichlet_host[v]) sint[v] = ns++;
  int32_t *didx = nullptr, *dvid = nullptr, *dsint = nullptr;
  double *dw = nullptr, *dg = nullptr, *dwv = nullptr, *dpts = nullptr;
  const size_t kk = (size_t)k * k, n4 = (size_t)N * 4;
  auto release = [&]() {
    for (void *p : {(void *)didx, (void *)dvid, (void *)dsint, (void *)dw, (void *)dwv, (void *)dpts})
      if (p) (void)hipFree(p);
  };
  if (hipMalloc(&didx, sizeof(int32_t) * n4) != hipSuccess || hipMalloc(&dvid, sizeof(int32_t) * n4) != hipSuccess ||
      hipMalloc(&dsint, sizeof(int32_t) * sint.size()) != hipSuccess ||
      hipMalloc(&dw, sizeof(double) * (n4 + 2 * kk)) != hipSuccess || hipMalloc(&dwv, sizeof(double) * n4) != hipSuccess ||
      hipMalloc(&dpts, sizeof(double) * 3 * (size_t)N) != hipSuccess) {
    release();
    return fail(KS_ERR_NOMEM, "hipMalloc failed");
  }
  dg = dw + n4;
  int rc = KS_OK;
  hipError_t e = hipMemcpyAsync(dsint, sint.data(), sizeof(int32_t) * sint.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    // this mesh's interior nodes (storage order) located in src on the GPU
    launch_interior_coords(c->n_nodes, c->node2int, c->coords, dpts, s);
    const int r = nonnested_weights_device(src->n_nodes, src->coords_host, src->n_elems, src->elems_host, N, dpts,
                                           dvid, dwv, s);
    if (r == -1) rc = fail(KS_ERR_MESH, "source mesh: bad element vertex ids");
    else if (r == -3) rc = fail(KS_ERR_NOMEM, "hipMalloc failed");
    else if (r == -2) rc = fail(KS_ERR_MESH, "point location: degenerate weights");
    else if (r < -2) rc = fail(KS_ERR_HIP, "point location failed");
    if (rc == KS_OK) launch_ell_from_vertices(N, dvid, dwv, dsint, didx, dw, s);
  }
  if (e == hipSuccess && rc == KS_OK) {
    launch_ellP_times(N, didx, dw, psi_src, k, k, 1.0, nullptr, 0, c->Xs, k, s);
    double *out = c->Xs;
    if (orthonormalize) {
      // G = X^T M X = R^T R (Cholesky, in column order) and X <- X R^-1
      spmm_cols(c, c->M, c->Xs, k, c->PsiNew, k, k);
      launch_gemm_tn_sym(N, k, c->Xs, k, c->PsiNew, k, dg, k, c->gwork, s);
      std::vector<double> G(kk), Ri(kk, 0.0);
      e = hipMemcpyAsync(G.data(), dg, sizeof(double) * kk, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess) {
        // in place: lower triangle of G becomes L with G = L L^T (R = L^T)
        for (int j = 0; j < k && rc == KS_OK; ++j) {
          double d = G[(size_t)j * k + j];
          for (int p = 0; p < j; ++p) d -= G[(size_t)j * k + p] * G[(size_t)j * k + p];
          if (!(d > 0.0)) {
            rc = fail(KS_ERR_EIG, "interpolated orbitals are linearly dependent");
            break;
          }
          const double ljj = std::sqrt(d);
          G[(size_t)j * k + j] = ljj;
          for (int i = j + 1; i < k; ++i) {
            double t = G[(size_t)i * k + j];
            for (int p = 0; p < j; ++p) t -= G[(size_t)i * k + p] * G[(size_t)j * k + p];
            G[(size_t)i * k + j] = t / ljj;
          }
        }
        // R^-1 = (L^T)^-1, upper triangular: columns by back substitution
        for (int col = 0; col < k && rc == KS_OK; ++col)
          for (int i = col; i >= 0; --i) {
            double t = (i == col) ? 1.0 : 0.0;
            for (int p = i + 1; p <= col; ++p) t -= G[(size_t)p * k + i] * Ri[(size_t)p * k + col];
            Ri[(size_t)i * k + col] = t / G[(size_t)i * k + i];
          }
        if (rc == KS_OK) {
          e = hipMemcpyAsync(dg + kk, Ri.data(), sizeof(double) * kk, hipMemcpyHostToDevice, s);
          if (e == hipSuccess && launch_tsmm(N, k, c->Xs, k, dg + kk, k, c->PsiNew, k, s) < 0)
            rc = fail(KS_ERR_ARG, "k too large for the orthonormalisation");
          out = c->PsiNew;
        }
      }
    }
    if (e == hipSuccess && rc == KS_OK) {
      launch_rows_to_api(N, k, out, psi, c->int2nat, s);
      e = hipStreamSynchronize(s);
    }
  }
  release();
  if (e != hipSuccess) return fail(KS_ERR_HIP, hipGetErrorString(e));
  if (rc != KS_OK) return rc;
  c->have_step = false;
  return KS_OK;
}

// ------------------------------------------------------------ direct SCF
// LOBPCG work space for up to k_max orbitals (allocated on first use)
static int direct_alloc(ks_ctx *c) {
  if (c->d_k) return KS_OK;
  const int km = c->k_max;
  const size_t N = c->N;
#define DA_(p, n) \
  if (c->alloc(&c->p, (n)) < 0) return KS_ERR_NOMEM
  DA_(dS, N * 3 * km);
  DA_(dHS, N * 3 * km);
  DA_(dMS, N * 3 * km);
  DA_(dT1, N * km);
  DA_(dT2, N * km);
  DA_(dH, (size_t)c->nnz_ext + 2);
  DA_(dDinv, N);
  DA_(dDM, N);
  DA_(dGH, (size_t)9 * km * km);
  DA_(dGM, (size_t)9 * km * km);
  DA_(dC, (size_t)3 * km * km);
  DA_(dTheta, (size_t)3 * km);
#undef DA_
  launch_extract_diag(c->N, c->rowptr, c->col, c->M, c->dDM, c->s);
  c->d_k = km;
  return KS_OK;
}

// Lowest k eigenpairs of (H, M) by block LOBPCG (locally optimal block
// preconditioned CG for the generalised problem): Rayleigh-Ritz over
// [X | W | P] with W = D^-1 (H X - M X Theta), D the Jacobi preconditioner in
// c->dDinv, P the previous search directions.  X = columns [0, k) of c->dS on
// entry (any basis of the start space) and on return (M-orthonormal Ritz
// vectors, ascending theta); H X and M X in c->dHS, c->dMS.  Stops when
// every column's ||H x - theta M x||_2 / ||M x||_2 <= tol or after max_it
// iterations; *resmax receives the largest of those ratios.
//
// H X, M X and H P, M P are carried by the same linear combinations as X and
// P.  When those combinations cancel (P nearly dependent on [X | W]) the
// carried products drift from the true ones, so: they are recomputed every
// LOBPCG_REFRESH iterations, before a stop is accepted, and when a
// Rayleigh-Ritz step fails (a Gram matrix with a non-positive diagonal); if
// the step still fails, P is dropped for that iteration.
constexpr int LOBPCG_REFRESH = 16;
static int lobpcg(ks_ctx *c, const double *H, int k, double tol, int max_it, std::vector<double> &theta,
                  int *iters, double *resmax) {
  const int N = c->N, L = 3 * k;
  hipStream_t s = c->s;
  double *S = c->dS, *HS = c->dHS, *MS = c->dMS;
  auto refresh = [&](int ncols) {
    spmm_cols(c, H, S, L, HS, L, ncols);
    spmm_cols(c, c->M, S, L, MS, L, ncols);
  };
  auto rayleigh_ritz = [&](int m) {
    launch_gemm_tn_sym(N, m, S, L, HS, L, c->dGH, m, c->gwork, s);
    launch_gemm_tn_sym(N, m, S, L, MS, L, c->dGM, m, c->gwork, s);
    int r = orth_impl(c, c->dGM, m);
    if (r < 0) return r;
    int rank = 0;
    return eig_impl(c, c->dGH, c->dGM, m, k, c->dC, theta, &rank);
  };
  refresh(k);
  const int maxb = std::min(512, (1024 * 32) / (2 * k));
  std::vector<double> sums(2 * k);
  int m = k, since_refresh = 0;
  *iters = 0;
  for (int it = 0;; ++it) {
    if (m > k && ++since_refresh >= LOBPCG_REFRESH) {
      refresh(m);
      since_refresh = 0;
    }
    // Rayleigh-Ritz on the active columns [0, m)
    if (rayleigh_ritz(m) < 0) {
      refresh(m);
      since_refresh = 0;
      if (rayleigh_ritz(m) < 0) {
        if (m != 3 * k) return KS_ERR_EIG;
        m = 2 * k;
        TRY(rayleigh_ritz(m));
      }
    }
    // P <- [W | P] C[k:m];  X <- [X | W | P] C  (and the same for H S, M S)
    for (double *B : {S, HS, MS}) {
      if (m > k && launch_tsmm(N, m - k, B + k, L, c->dC + (size_t)k * k, k, c->dT1, k, s) < 0)
        return fail(KS_ERR_ARG, "block too wide for the LOBPCG update");
      if (launch_tsmm(N, m, B, L, c->dC, k, c->dT2, k, s) < 0)
        return fail(KS_ERR_ARG, "block too wide for the LOBPCG update");
      launch_copy_cols(N, k, c->dT2, k, B, L, 0, s);
      if (m > k) launch_copy_cols(N, k, c->dT1, k, B, L, 2 * k, s);
    }
    const bool haveP = m > k;
    // residuals; the preconditioned ones become W (columns [k, 2k))
    HIPCHK(hipMemcpyAsync(c->dTheta, theta.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    double rmax = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      const int nb = launch_lobpcg_resid(N, k, L, HS, MS, c->dTheta, c->dDinv, S + k, L, c->redpart, maxb, s);
      if (nb < 0) return fail(KS_ERR_ARG, "k too large for the LOBPCG residual");
      TRY(reduce_small(c, c->redpart, nb, 2 * k, sums.data()));
      rmax = 0.0;
      for (int j = 0; j < k; ++j) rmax = std::max(rmax, std::sqrt(sums[j] / std::max(sums[k + j], 1e-300)));
      // a stop is accepted on residuals from freshly computed H X and M X
      if (rmax > tol || it >= max_it || !haveP) break;
      refresh(k);
    }
    *resmax = rmax;
    *iters = it;
    if (rmax <= tol || it >= max_it) break;
    spmm_cols(c, H, S + k, L, HS + k, L, k);
    spmm_cols(c, c->M, S + k, L, MS + k, L, k);
    m = haveP ? 3 * k : 2 * k;
  }
  return KS_OK;
}

extern "C" int ks_direct_scf(ks_ctx *c, double *psi, double *lambda_host, int32_t k, const double *occ_host,
                             double tol, int32_t max_scf, double tol_eig, int32_t max_eig, double *rho_q,
                             ks_direct_report *rep_host) {
  if (!c || !psi || !lambda_host || !occ_host) return fail(KS_ERR_ARG, "null argument");
  if (k < 1 || k > c->k_max || k > 48) return fail(KS_ERR_ARG, "k must be in 1..min(k_max, 48)");
  if (!(tol > 0.0) || !(tol_eig > 0.0) || max_scf < 1 || max_eig < 1)
    return fail(KS_ERR_ARG, "tolerances must be > 0 and iteration limits >= 1");
  TRY(direct_alloc(c));
  hipStream_t s = c->s;
  const double t0 = now_s();
  const int N = c->N, L = 3 * k;
  const int64_t nqt = (int64_t)c->n_e * c->n_q;
  const bool hartree = c->opt.hartree_mode != KS_HARTREE_OFF;
  c->have_step = false;
  ks_direct_report R;
  std::memset(&R, 0, sizeof(R));
  // X = psi (storage order), rho_in = its density
  launch_rows_to_storage(N, k, psi, c->PsiNew, c->int2nat, s);
  launch_copy_cols(N, k, c->PsiNew, k, c->dS, L, 0, s);
  HIPCHK(hipMemcpyAsync(c->occ_d, occ_host, sizeof(double) * k, hipMemcpyHostToDevice, s));
  launch_density(c->edof, c->n_loc, c->n_e, c->n_q, c->phi, c->PsiNew, k, k, c->occ_d, c->rho_in, s);
  AndersonRing ring;
  std::vector<double> th(k);
  for (int j = 0; j < k; ++j) th[j] = lambda_host[j];
  double res = INFINITY, eres = 0.0;
  int it = 0, piters = 0;
  for (it = 0; it < max_scf; ++it) {
    // H(rho_in) = A^L + M[V_H(rho_in) + V_xc(rho_in)], w_D from rho_in itself
    if (hartree) {
      TRY(boundary_data(c, c->rho_in));
      const int r = hartree_solve(c, c->rho_in, &piters, std::min(c->opt.tol_poisson, 1e-4 * tol));
      if (r < 0) return r;
      R.poisson_iters += piters;
    } else {
      launch_fill(nqt, 0.0, c->vh_q, s);
    }
    launch_xc(nqt, c->rho_in, c->opt.xc_mode, c->exc_q, c->vxc_q, s);
    launch_add(nqt, c->vh_q, c->vxc_q, c->vnl_q, s);
    assemble_potential_all(c, c->vnl_q, c->dH, c->AL);
    // Jacobi preconditioner of the shifted Laplacian 1/2 K + tau M, tau = max(1, -theta_1)
    const double tau = std::max(1.0, std::isfinite(th[0]) ? -th[0] : 1.0);
    launch_prec_diag(N, 0.5, c->diagK, tau, c->dDM, c->dDinv, s);
    // eigensolve to a tolerance that follows the density residual
    const double te = std::max(tol_eig, std::min(1e-3, 0.1 * res));
    int ei = 0;
    TRY(lobpcg(c, c->dH, k, te, max_eig, th, &ei, &eres));
    R.eig_iters += ei;
    launch_copy_cols(N, k, c->dS, L, c->PsiNew, k, 0, s);
    launch_density(c->edof, c->n_loc, c->n_e, c->n_q, c->phi, c->PsiNew, k, k, c->occ_d, c->rho_out, s);
    TRY(anderson_record(c, ring, c->rho_out, c->rho_in, &res));
    // converged or the last pass: no mixing, the energies pair rho_in with
    // the operator it built (Sec. 3.1)
    if ((res < tol && eres <= tol_eig) || it + 1 == max_scf) {
      it += 1;
      break;
    }
    TRY(anderson_mix_next(c, ring, c->rho_in));
  }
  R.scf_iters = it;
  R.res = res;
  R.eig_res = eres;
  // outputs and the energy of Sec. 3.1 on the density that built H
  launch_rows_to_api(N, k, c->PsiNew, psi, c->int2nat, s);
  if (rho_q) HIPCHK(hipMemcpyAsync(rho_q, c->rho_out, sizeof(double) * nqt, hipMemcpyDeviceToDevice, s));
  double band = 0.0;
  for (int j = 0; j < k; ++j) {
    lambda_host[j] = th[j];
    band += occ_host[j] * th[j];
  }
  R.E_band = band;
  R.E_nn = c->E_nn;
  {
    const double *a[3] = {c->vh_q, c->exc_q, c->vxc_q};
    const double *b[3] = {c->rho_in, c->rho_in, c->rho_in};
    double e[3];
    TRY(weighted_dots(c, 3, a, b, e));
    R.E_H = 0.5 * e[0];
    R.E_xc = e[1];
    R.E_vxc = e[2];
  }
  R.E_total = R.E_band - R.E_H - R.E_vxc + R.E_xc + R.E_nn;
  HIPCHK(hipStreamSynchronize(s));
  R.converged = res < tol && eres <= tol_eig;
  R.seconds = now_s() - t0;
  if (rep_host) *rep_host = R;
  return R.converged ? KS_OK : KS_NOT_CONVERGED;
}

// Algorithm 3 run to convergence: repeat ks_scf_step until
// ||rho^{l+1} - rho^l||_0 < tol_outer or max_steps steps; then E_KS of the
// last step (ks_step_energy).
extern "C" int ks_scf_run(ks_ctx *c, double *psi, double *lambda_host, int32_t k, const double *occ_host,
                          int32_t precision, double tol_outer, int32_t max_steps, double *rho_q,
                          ks_run_report *rep_host) {
  if (!c || !psi || !lambda_host || !occ_host) return fail(KS_ERR_ARG, "null argument");
  if (!(tol_outer > 0.0) || max_steps < 1) return fail(KS_ERR_ARG, "tol_outer must be > 0, max_steps >= 1");
  ks_run_report R;
  std::memset(&R, 0, sizeof(R));
  const double t0 = now_s();
  int st = KS_OK;
  for (int l = 0; l < max_steps; ++l) {
    ks_step_report sr;
    st = ks_scf_step(c, psi, lambda_host, k, occ_host, precision, rho_q, &sr);
    if (st < 0) return st;
    R.steps = l + 1;
    R.inner_iters += sr.inner_iters;
    R.poisson_iters += sr.poisson_iters;
    R.res_outer = sr.res_outer;
    R.E_total = sr.E_total;
    if (sr.res_outer < tol_outer) {
      R.converged = 1;
      break;
    }
  }
  double e[6];
  const int se = ks_step_energy(c, e);
  if (se < 0) return se;
  R.E_KS = e[0];
  R.seconds = now_s() - t0;
  if (rep_host) *rep_host = R;
  if (!R.converged) return KS_NOT_CONVERGED;
  return st == KS_WARN_DEGENERATE ? KS_WARN_DEGENERATE : KS_OK;
}
