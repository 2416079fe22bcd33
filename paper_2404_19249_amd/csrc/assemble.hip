// Element geometry and element-coloured finite element assembly.
//
// Stiffness K_ij = int grad phi_i . grad phi_j and the potential-weighted
// mass M[V]_ij = int V phi_i phi_j (Sec. 3.3, eqs. st3/st4) are integrated
// with the supplied quadrature rule on affine tetrahedra.  Elements of one
// colour share no node, so one launch per colour accumulates its element
// matrices into the CSR values without atomics and in a fixed order
// (bitwise-reproducible results).  Basis tables are staged in LDS once per
// workgroup; every thread owns one element.
#include "common.h"
#include "kernels.h"

namespace ks {

__global__ void __launch_bounds__(256) k_geometry(const double *__restrict__ coords,
                                                  const int32_t *__restrict__ elems, int n_loc,
                                                  int n_e, double *__restrict__ absdet,
                                                  double *__restrict__ gl, int32_t *bad) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_e) return;
  const int32_t *el = elems + (int64_t)e * n_loc;
  double X[4][3];
  for (int v = 0; v < 4; ++v)
    for (int d = 0; d < 3; ++d) X[v][d] = coords[3 * (int64_t)el[v] + d];
  // J columns: X1-X0, X2-X0, X3-X0
  double J[3][3];
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 3; ++c) J[d][c] = X[c + 1][d] - X[0][d];
  // cofactors
  double C00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  double C01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  double C02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  double C10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  double C11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  double C12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  double C20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  double C21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  double C22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  double det = J[0][0] * C00 + J[0][1] * C01 + J[0][2] * C02;
  if (!(det > 0.0)) atomicAdd(bad, 1);
  double id = 1.0 / det;
  // inverse: Jinv[r][c] = C[c][r] / det ; grad lambda_{r+1} = row r of Jinv
  double Ji[3][3] = {{C00 * id, C10 * id, C20 * id},
                     {C01 * id, C11 * id, C21 * id},
                     {C02 * id, C12 * id, C22 * id}};
  double *g = gl + (int64_t)e * 12;
  for (int d = 0; d < 3; ++d) {
    g[3 + d] = Ji[0][d];
    g[6 + d] = Ji[1][d];
    g[9 + d] = Ji[2][d];
    g[d] = -(Ji[0][d] + Ji[1][d] + Ji[2][d]);
  }
  absdet[e] = fabs(det);
}

void launch_geometry(const double *coords, const int32_t *elems, int n_loc, int n_e,
                     double *absdet, double *gl, int32_t *bad, hipStream_t s) {
  if (n_e <= 0) return;
  hipLaunchKernelGGL(k_geometry, dim3((n_e + 255) / 256), dim3(256), 0, s, coords, elems, n_loc,
                     n_e, absdet, gl, bad);
}

// ---------------------------------------------------------------- K and M
template <int NLOC, int NQ>
__global__ void __launch_bounds__(128) k_assemble_KM(const int32_t *__restrict__ list, int count,
                                                     const int32_t *__restrict__ slot,
                                                     const double *__restrict__ absdet,
                                                     const double *__restrict__ gl,
                                                     const double *__restrict__ phi,
                                                     const double *__restrict__ dphi,
                                                     const double *__restrict__ w,
                                                     double *__restrict__ K,
                                                     double *__restrict__ M) {
  __shared__ double s_phi[NQ * NLOC];
  __shared__ double s_dphi[NQ * NLOC * 4];
  __shared__ double s_w[NQ];
  for (int i = threadIdx.x; i < NQ * NLOC; i += blockDim.x) s_phi[i] = phi[i];
  for (int i = threadIdx.x; i < NQ * NLOC * 4; i += blockDim.x) s_dphi[i] = dphi[i];
  for (int i = threadIdx.x; i < NQ; i += blockDim.x) s_w[i] = w[i];
  __syncthreads();
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int e = list[t];
  const double dj = absdet[e];
  double G[4][4];
  {
    double g[4][3];
    for (int v = 0; v < 4; ++v)
      for (int d = 0; d < 3; ++d) g[v][d] = gl[(int64_t)e * 12 + 3 * v + d];
    for (int v = 0; v < 4; ++v)
      for (int u = 0; u < 4; ++u) G[v][u] = g[v][0] * g[u][0] + g[v][1] * g[u][1] + g[v][2] * g[u][2];
  }
  const int32_t *sl = slot + (int64_t)e * NLOC * NLOC;
  for (int a = 0; a < NLOC; ++a) {
    for (int b = a; b < NLOC; ++b) {
      // slots are -1 for rows on the Dirichlet boundary; a pair may have one
      // interior row (II or IB entry) and one boundary row
      const int s_ab = sl[a * NLOC + b];
      const int s_ba = sl[b * NLOC + a];
      if (s_ab < 0 && s_ba < 0) continue;
      double kab = 0.0, mab = 0.0;
      for (int q = 0; q < NQ; ++q) {
        const double *da = s_dphi + (q * NLOC + a) * 4;
        const double *db = s_dphi + (q * NLOC + b) * 4;
        double gg = 0.0;
        for (int v = 0; v < 4; ++v) {
          double t2 = 0.0;
          for (int u = 0; u < 4; ++u) t2 += G[v][u] * db[u];
          gg += da[v] * t2;
        }
        kab += s_w[q] * gg;
        mab += s_w[q] * s_phi[q * NLOC + a] * s_phi[q * NLOC + b];
      }
      kab *= dj;
      mab *= dj;
      if (s_ab >= 0) {
        K[s_ab] += kab;
        M[s_ab] += mab;
      }
      if (b != a && s_ba >= 0) {
        K[s_ba] += kab;
        M[s_ba] += mab;
      }
    }
  }
}

void launch_assemble_KM(const int32_t *list, int count, int n_loc, int n_q, const int32_t *slot,
                        const double *absdet, const double *gl, const double *phi,
                        const double *dphi, const double *w, double *K, double *M, hipStream_t s) {
  if (count <= 0) return;
  dim3 g((count + 127) / 128), b(128);
  if (n_loc == 4 && n_q == 8)
    hipLaunchKernelGGL((k_assemble_KM<4, 8>), g, b, 0, s, list, count, slot, absdet, gl, phi,
                       dphi, w, K, M);
  else if (n_loc == 10 && n_q == 27)
    hipLaunchKernelGGL((k_assemble_KM<10, 27>), g, b, 0, s, list, count, slot, absdet, gl, phi,
                       dphi, w, K, M);
  else if (n_loc == 4 && n_q == 27)
    hipLaunchKernelGGL((k_assemble_KM<4, 27>), g, b, 0, s, list, count, slot, absdet, gl, phi,
                       dphi, w, K, M);
  else if (n_loc == 10 && n_q == 8)
    hipLaunchKernelGGL((k_assemble_KM<10, 8>), g, b, 0, s, list, count, slot, absdet, gl, phi,
                       dphi, w, K, M);
}

// ------------------------------------------------------------ M[V]
// pairtab[q][p] = phi_qa phi_qb for the p-th pair (a <= b) in row-major
// upper-triangle order.  One lane per (element, pair): EPW = 64 / NP
// elements per wave (6 for P1, 1 for P2); the lanes of an element read its
// quadrature weights w_q |J| V_q as broadcasts and their own pair column of
// the table from LDS, and add the entry into its two CSR slots (elements of
// one colour share no node, so no two lanes of a launch touch one slot).
template <int NLOC, int NQ>
__global__ void __launch_bounds__(256) k_assemble_potential(
    const int32_t *__restrict__ list, int count, const int32_t *__restrict__ slot,
    const double *__restrict__ absdet, const double *__restrict__ pairtab,
    const double *__restrict__ w, const double *__restrict__ V, double *__restrict__ out) {
  constexpr int NP = NLOC * (NLOC + 1) / 2;
  constexpr int EPW = 64 / NP;
  __shared__ double s_pt[NQ * NP];
  __shared__ double s_w[NQ];
  __shared__ unsigned char s_a[NP], s_b[NP];
  for (int i = threadIdx.x; i < NQ * NP; i += blockDim.x) s_pt[i] = pairtab[i];
  for (int i = threadIdx.x; i < NQ; i += blockDim.x) s_w[i] = w[i];
  if (threadIdx.x == 0) {
    int p = 0;
    for (int a = 0; a < NLOC; ++a)
      for (int b = a; b < NLOC; ++b, ++p) {
        s_a[p] = (unsigned char)a;
        s_b[p] = (unsigned char)b;
      }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int es = lane / NP, p = lane - es * NP;
  const int t = (blockIdx.x * (int)(blockDim.x >> 6) + wave) * EPW + es;
  if (es >= EPW || t >= count) return;
  const int e = list[t];
  const double dj = absdet[e];
  const double *Ve = V + (int64_t)e * NQ;
  double m = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) m += (s_w[q] * dj * Ve[q]) * s_pt[q * NP + p];
  const int a = s_a[p], b = s_b[p];
  const int32_t *sl = slot + (int64_t)e * NLOC * NLOC;
  const int s_ab = sl[a * NLOC + b];
  const int s_ba = sl[b * NLOC + a];
  if (s_ab >= 0) out[s_ab] += m;
  if (b != a && s_ba >= 0) out[s_ba] += m;
}

void launch_assemble_potential(const int32_t *list, int count, int n_loc, int n_q,
                               const int32_t *slot, const double *absdet, const double *pairtab,
                               const double *w, const double *V_q, double *out, hipStream_t s) {
  if (count <= 0) return;
  const int np = n_loc * (n_loc + 1) / 2, epw = 64 / np;
  const int per_block = 4 * epw;  // elements per 256-thread workgroup
  dim3 g((count + per_block - 1) / per_block), b(256);
  if (n_loc == 4 && n_q == 8)
    hipLaunchKernelGGL((k_assemble_potential<4, 8>), g, b, 0, s, list, count, slot, absdet,
                       pairtab, w, V_q, out);
  else if (n_loc == 10 && n_q == 27)
    hipLaunchKernelGGL((k_assemble_potential<10, 27>), g, b, 0, s, list, count, slot, absdet,
                       pairtab, w, V_q, out);
  else if (n_loc == 4 && n_q == 27)
    hipLaunchKernelGGL((k_assemble_potential<4, 27>), g, b, 0, s, list, count, slot, absdet,
                       pairtab, w, V_q, out);
  else if (n_loc == 10 && n_q == 8)
    hipLaunchKernelGGL((k_assemble_potential<10, 8>), g, b, 0, s, list, count, slot, absdet,
                       pairtab, w, V_q, out);
}

// Row form.  One thread per interior row, one workgroup per block of
// blockDim.x consecutive storage rows, whose CSR values are contiguous and
// accumulate in LDS.  The thread of row r walks the incidences (e, a) of r
// (the elements in which r is local node a, ascending element order) and,
// for every local node b whose column is interior, adds
//     sum_q w_q |J_e| V_eq phi_a(q) phi_b(q)
// to the slot at off[b] of its own row.  Every value slot is summed by one
// thread in a fixed order: no atomics, bitwise reproducible.  The rows of a
// block are visited longest incidence list first (rperm), so that the rows
// of one wavefront have similar trip counts.  out = base + M[V] over the
// interior pattern (base may be null), out32 = (float) out (may be null).
// At most 96 VGPRs (5 waves per SIMD): the kernel waits on its gathers, and
// the LDS image of the block's rows allows about ten waves per CU.
template <int NLOC, int NQ>
__global__ void __launch_bounds__(ASM_ROWS) __attribute__((amdgpu_waves_per_eu(5)))
k_assemble_rows(int N, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ incptr,
                const IncRec<NLOC> *__restrict__ inc, const uint8_t *__restrict__ rperm,
                const double *__restrict__ absdet, const double *__restrict__ phiq,
                const double *__restrict__ phib, const double *__restrict__ w,
                const double *__restrict__ V, const double *__restrict__ base,
                double *__restrict__ out, float *__restrict__ out32) {
  extern __shared__ double s_acc[];
  __shared__ double s_wphi[NQ * NLOC];  // w_q phi_a(q)
  // workgroups are dealt to the 8 XCDs round robin: give each XCD a
  // contiguous eighth of the row blocks, so that neighbouring blocks (which
  // share elements) meet in one L2
  const int nblk = (N + ASM_ROWS - 1) / ASM_ROWS, per = (nblk + 7) / 8;
  const int blk = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (blk >= nblk) return;
  const int r0 = blk * ASM_ROWS;
  const int nr = min(ASM_ROWS, N - r0);
  const int v0 = rowptr[r0], nv = rowptr[r0 + nr] - v0;
  for (int i = threadIdx.x; i < nv; i += ASM_ROWS) s_acc[i] = base ? base[v0 + i] : 0.0;
  for (int i = threadIdx.x; i < NQ * NLOC; i += ASM_ROWS) s_wphi[i] = w[i / NLOC] * phiq[i];
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    const int row = r0 + rperm[r0 + threadIdx.x];
    double *acc = s_acc + (rowptr[row] - v0);
    const int jb = incptr[row], j1 = incptr[row + 1];
    // quadrature points in chunks of QC: ten running sums and one chunk of
    // products live at a time (fewer registers, more waves per SIMD)
    constexpr int QC = NQ > 9 ? 9 : NQ;
    for (int j = jb; j < j1; ++j) {
      const IncRec<NLOC> rc = inc[j];
      const int e = (int)(rc.ea >> 4), a = (int)(rc.ea & 15u);
      const double dj = absdet[e];
      const double *Ve = V + (int64_t)e * NQ;
      unsigned off[NLOC];
#pragma unroll
      for (int b = 0; b < NLOC; ++b) off[b] = rc.off[b];
      double vb[NLOC];
#pragma unroll
      for (int b = 0; b < NLOC; ++b) vb[b] = 0.0;
#pragma unroll 1
      for (int q0 = 0; q0 < NQ; q0 += QC) {
        double d[QC];
#pragma unroll
        for (int u = 0; u < QC; ++u)
          d[u] = q0 + u < NQ ? dj * Ve[q0 + u] * s_wphi[(q0 + u) * NLOC + a] : 0.0;
#pragma unroll
        for (int b = 0; b < NLOC; ++b)
#pragma unroll
          for (int u = 0; u < QC; ++u)
            if (q0 + u < NQ) vb[b] += d[u] * phib[b * NQ + q0 + u];
      }
      // the incidence's slots are distinct: all reads, then all writes (one
      // LDS round trip instead of one per slot; same order of additions)
      double cur[NLOC];
#pragma unroll
      for (int b = 0; b < NLOC; ++b) cur[b] = off[b] != 255u ? acc[off[b]] : 0.0;
#pragma unroll
      for (int b = 0; b < NLOC; ++b)
        if (off[b] != 255u) acc[off[b]] = cur[b] + vb[b];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nv; i += ASM_ROWS) {
    const double v = s_acc[i];
    out[v0 + i] = v;
    if (out32) out32[v0 + i] = (float)v;
  }
}
// Load vector in two passes.  Elements: be[e][a] = |J_e| sum_q w_q f_eq
// phi_a(q), a block's elements' quadrature values read together (they are
// contiguous, so the loads coalesce) and staged in LDS.  Rows: out[r] =
// scale sum over the incidences (e, a) of interior row r of be[e][a], one
// thread per row in ascending element order (the assembly's incidence
// records): every element's values are read once, and the sum has a fixed
// order.
constexpr int LOAD_EPB = 128;  // elements per workgroup of the element pass
template <int NLOC, int NQ>
__global__ void __launch_bounds__(LOAD_EPB) k_load_elems(int n_e, const double *__restrict__ absdet,
                                                        const double *__restrict__ phiq,
                                                        const double *__restrict__ w,
                                                        const double *__restrict__ f, double *__restrict__ be) {
  __shared__ double s_wphi[NQ * NLOC];
  __shared__ double s_f[LOAD_EPB * NQ];
  for (int i = threadIdx.x; i < NQ * NLOC; i += blockDim.x) s_wphi[i] = w[i / NLOC] * phiq[i];
  const int e0 = blockIdx.x * LOAD_EPB;
  const int ne = min(LOAD_EPB, n_e - e0);
  const double *fb = f + (int64_t)e0 * NQ;
  for (int i = threadIdx.x; i < ne * NQ; i += blockDim.x) s_f[i] = fb[i];
  __syncthreads();
  if ((int)threadIdx.x >= ne) return;
  const int e = e0 + threadIdx.x;
  const double *fe = s_f + threadIdx.x * NQ;
  const double dj = absdet[e];
#pragma unroll
  for (int a = 0; a < NLOC; ++a) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q + 2 < NQ; q += 3) {
      s0 += s_wphi[q * NLOC + a] * fe[q];
      s1 += s_wphi[(q + 1) * NLOC + a] * fe[q + 1];
      s2 += s_wphi[(q + 2) * NLOC + a] * fe[q + 2];
    }
    if constexpr (NQ % 3 >= 1) s0 += s_wphi[(NQ - NQ % 3) * NLOC + a] * fe[NQ - NQ % 3];
    if constexpr (NQ % 3 == 2) s1 += s_wphi[(NQ - 1) * NLOC + a] * fe[NQ - 1];
    be[(int64_t)e * NLOC + a] = dj * ((s0 + s1) + s2);
  }
}
template <int NLOC>
__global__ void __launch_bounds__(256) k_load_gather(int N, const int32_t *__restrict__ incptr,
                                                     const IncRec<NLOC> *__restrict__ inc,
                                                     const double *__restrict__ be, double scale,
                                                     double *__restrict__ out) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < N; r += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int j = incptr[r]; j < incptr[r + 1]; ++j) {
      const uint32_t ea = inc[j].ea;
      acc += be[(int64_t)(ea >> 4) * NLOC + (ea & 15u)];
    }
    out[r] = scale * acc;
  }
}
int launch_load_rows(int N, int n_e, int n_loc, int n_q, const int32_t *incptr, const void *inc,
                     const double *absdet, const double *phi, const double *w, const double *f_q, double scale,
                     double *be, double *out, hipStream_t s) {
  if (N <= 0 || n_e <= 0) return 0;
  dim3 ge((n_e + LOAD_EPB - 1) / LOAD_EPB), bk(LOAD_EPB), gr(std::min(8192, (N + 255) / 256)), br(256);
#define KS_LR(NL, NQ)                                                                                   \
  do {                                                                                                  \
    hipLaunchKernelGGL((k_load_elems<NL, NQ>), ge, bk, 0, s, n_e, absdet, phi, w, f_q, be);             \
    hipLaunchKernelGGL((k_load_gather<NL>), gr, br, 0, s, N, incptr, static_cast<const IncRec<NL> *>(inc), \
                       be, scale, out);                                                                 \
  } while (0)
  if (n_loc == 4 && n_q == 8) KS_LR(4, 8);
  else if (n_loc == 10 && n_q == 27) KS_LR(10, 27);
  else if (n_loc == 4 && n_q == 27) KS_LR(4, 27);
  else if (n_loc == 10 && n_q == 8) KS_LR(10, 8);
  else return -1;
#undef KS_LR
  return 0;
}

size_t assemble_rows_lds_limit() { return 160 * 1024 - 27 * 10 * sizeof(double) - 1024; }
int launch_assemble_rows(int N, int n_loc, int n_q, const int32_t *rowptr, const int32_t *incptr, const void *inc,
                         const uint8_t *rperm, size_t lds_bytes, const double *absdet, const double *phi,
                         const double *phib, const double *w, const double *V_q, const double *base, double *out,
                         float *out32, hipStream_t s) {
  if (N <= 0) return 0;
  const int nblk = (N + ASM_ROWS - 1) / ASM_ROWS;
  dim3 g(8 * ((nblk + 7) / 8)), b(ASM_ROWS);
#define KS_AR(NL, NQ)                                                                                           \
  do {                                                                                                          \
    static bool attr = false;                                                                                   \
    if (!attr) {                                                                                                \
      if (hipFuncSetAttribute((const void *)k_assemble_rows<NL, NQ>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                              (int)assemble_rows_lds_limit()) != hipSuccess)                                    \
        return -1;                                                                                              \
      attr = true;                                                                                              \
    }                                                                                                           \
    hipLaunchKernelGGL((k_assemble_rows<NL, NQ>), g, b, lds_bytes, s, N, rowptr, incptr,                        \
                       static_cast<const IncRec<NL> *>(inc), rperm, absdet, phi, phib, w, V_q, base, out,    \
                       out32);     \
    return 0;                                                                                                   \
  } while (0)
  if (n_loc == 4 && n_q == 8) KS_AR(4, 8);
  if (n_loc == 10 && n_q == 27) KS_AR(10, 27);
  if (n_loc == 4 && n_q == 27) KS_AR(4, 27);
  if (n_loc == 10 && n_q == 8) KS_AR(10, 8);
#undef KS_AR
  return -1;
}

// ------------------------------------------------------------ load vector
template <int NLOC, int NQ>
__global__ void __launch_bounds__(256) k_load_vector(const int32_t *__restrict__ list, int count,
                                                     const int32_t *__restrict__ edof,
                                                     const double *__restrict__ absdet,
                                                     const double *__restrict__ phi,
                                                     const double *__restrict__ w,
                                                     const double *__restrict__ f, double scale,
                                                     double *__restrict__ out) {
  __shared__ double s_phi[NQ * NLOC];
  __shared__ double s_w[NQ];
  for (int i = threadIdx.x; i < NQ * NLOC; i += blockDim.x) s_phi[i] = phi[i];
  for (int i = threadIdx.x; i < NQ; i += blockDim.x) s_w[i] = w[i];
  __syncthreads();
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int e = list[t];
  const double dj = absdet[e] * scale;
  double c[NQ];
  const double *fe = f + (int64_t)e * NQ;
#pragma unroll
  for (int q = 0; q < NQ; ++q) c[q] = s_w[q] * dj * fe[q];
#pragma unroll
  for (int a = 0; a < NLOC; ++a) {
    const int d = edof[(int64_t)e * NLOC + a];
    if (d < 0) continue;
    double b = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) b += c[q] * s_phi[q * NLOC + a];
    out[d] += b;
  }
}

void launch_load_vector(const int32_t *list, int count, int n_loc, int n_q, const int32_t *edof,
                        const double *absdet, const double *phi, const double *w,
                        const double *f_q, double scale, double *out, hipStream_t s) {
  if (count <= 0) return;
  dim3 g((count + 255) / 256), b(256);
  if (n_loc == 4 && n_q == 8)
    hipLaunchKernelGGL((k_load_vector<4, 8>), g, b, 0, s, list, count, edof, absdet, phi, w, f_q,
                       scale, out);
  else if (n_loc == 10 && n_q == 27)
    hipLaunchKernelGGL((k_load_vector<10, 27>), g, b, 0, s, list, count, edof, absdet, phi, w,
                       f_q, scale, out);
  else if (n_loc == 4 && n_q == 27)
    hipLaunchKernelGGL((k_load_vector<4, 27>), g, b, 0, s, list, count, edof, absdet, phi, w,
                       f_q, scale, out);
  else if (n_loc == 10 && n_q == 8)
    hipLaunchKernelGGL((k_load_vector<10, 8>), g, b, 0, s, list, count, edof, absdet, phi, w,
                       f_q, scale, out);
}

// ------------------------------------------------------------ BLAS-1
__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b,
                        double *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}
__global__ void k_fill(int64_t n, double v, double *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}
__global__ void k_combine3(int64_t n, double a, const double *__restrict__ x, double b,
                           const double *__restrict__ y, double c, const double *__restrict__ z,
                           double *__restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double r = a * x[i];
    if (y) r += b * y[i];
    if (z) r += c * z[i];
    out[i] = r;
  }
}
__global__ void k_to_float(int64_t n, const double *__restrict__ x, float *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
static inline dim3 grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}
void launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_axpby, grid_for(n), dim3(256), 0, s, n, a, x, b, y);
}
void launch_fill(int64_t n, double v, double *y, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill, grid_for(n), dim3(256), 0, s, n, v, y);
}
void launch_combine3(int64_t n, double a, const double *x, double b, const double *y, double c,
                     const double *z, double *out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_combine3, grid_for(n), dim3(256), 0, s, n, a, x, b, y, c, z, out);
}
void launch_to_float(int64_t n, const double *x, float *y, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_to_float, grid_for(n), dim3(256), 0, s, n, x, y);
}

__global__ void k_extract_diag(int N, const int32_t *__restrict__ rowptr,
                               const int32_t *__restrict__ col, const double *__restrict__ val,
                               double *__restrict__ diag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double d = 0.0;
  for (int j = rowptr[i]; j < rowptr[i + 1]; ++j)
    if (col[j] == i) d = val[j];
  diag[i] = d;
}
void launch_extract_diag(int N, const int32_t *rowptr, const int32_t *col, const double *val,
                         double *diag, hipStream_t s) {
  if (N > 0)
    hipLaunchKernelGGL(k_extract_diag, dim3((N + 255) / 256), dim3(256), 0, s, N, rowptr, col, val,
                       diag);
}

}  // namespace ks
