// Multi-right-hand-side CSR SpMM and the block Jacobi-preconditioned CG of
// the boundary value problems of Algorithm 3 (eq. Aux_Linear_Problem).
//
// Layout: every [N][k] block is row-major with the k right-hand sides
// contiguous, so the k values of one gathered row form one coalesced
// segment.  A group of CG = k/VW lanes owns one matrix row, each lane VW
// consecutive columns; for k = 1 (Hartree Poisson) NG lanes split the
// nonzeros of a row instead and combine them with cross-lane shuffles.
//
// One PCG iteration is three streaming launches, each followed (A, B) by a
// one-workgroup reduction of its per-block column partials:
//   A  q = S p                      partials p.q        -> alpha
//   B  r -= alpha q                 partials r.z, r.r   -> beta, convergence
//   C  x += alpha p,  p = D^{-1} r + beta p
// Per-column scalars live on the device and are combined in a fixed order
// (bitwise-reproducible results, no device-scope fences in the streaming
// kernels).  Converged columns are frozen (alpha = 0).  Launches after
// convergence return at once; the host polls the state every few iterations.
#include "common.h"
#include "kernels.h"
#include <vector>
#include <type_traits>
#include <algorithm>

namespace ks {

// per-column scalars and control words
struct ColState {
  double rz, pq, alpha, beta, rr, bb, rz_new;
  double alpha_prev;  // the previous iteration's alpha (its x update is deferred to this one)
  int active, iters;
};
struct Control {
  int stop;       // set when no column is active (or breakdown)
  int skip;       // iteration in which stop was set (its x/p update still runs)
  int breakdown;  // p^T S p <= 0 or NaN in an active column
  int pad;
};
// workgroups of an elementwise phase: 512 (2 per CU, each sweeping many row
// groups).  On the 2M-row, 24-column FP32 solve 512 streams as fast as 2048
// and leaves a quarter of the column partials for the one-workgroup
// reductions between phases.
static int pcg_blocks() { return 512; }
constexpr int SPMM_BLOCKS = 2048; // workgroups of the SpMM phase (8 waves per SIMD)
size_t pcg_state_bytes(int k) { return sizeof(Control) + sizeof(ColState) * (size_t)k + 64; }

template <typename T, int VW>
struct alignas(sizeof(T) * VW) VecT {
  T v[VW];
};

// ------------------------------------------------------------------ mapping
struct RowMap {
  int lane, wave, LPR, RPW, slot, cg, ng;
  bool valid;  // lane owns a (row slot, column group)
};
template <int NG>
__device__ __forceinline__ RowMap row_map(int CG) {
  RowMap m;
  m.lane = threadIdx.x & 63;
  m.wave = threadIdx.x >> 6;
  m.LPR = CG * NG;
  m.RPW = 64 / m.LPR;
  m.slot = m.lane / m.LPR;
  const int r = m.lane % m.LPR;
  m.cg = r / NG;
  m.ng = r % NG;
  m.valid = m.slot < m.RPW;
  return m;
}

// Row groups (one per workgroup iteration) are dealt to the 8 XCDs in
// contiguous eighths: workgroup b runs on XCD b % 8 (round-robin dispatch), so
// the workgroups of one XCD sweep one contiguous slab of rows and the gathered
// neighbour rows of the block vector stay in that XCD's L2.
struct GroupIter {
  int g, end, step;
};
__device__ __forceinline__ GroupIter group_iter(int n_groups) {
  const int nx = (gridDim.x >= 8 && (gridDim.x & 7) == 0) ? 8 : 1;
  const int x = blockIdx.x % nx, lb = blockIdx.x / nx, per = gridDim.x / nx;
  const int chunk = (n_groups + nx - 1) / nx;
  GroupIter it;
  it.g = x * chunk + lb;
  it.end = min(n_groups, (x + 1) * chunk);
  it.step = per;
  return it;
}

// Block reduction of per-lane column partials (VW columns per lane) into
// part[blockIdx][col] for col < k.  s_red: 256 * VW doubles.
template <int VW, int NG>
__device__ __forceinline__ void block_cols(const double (&acc)[VW], const RowMap &m, int k, int CG,
                                           double *s_red, double *part, int stride, int off) {
  for (int v = 0; v < VW; ++v) s_red[threadIdx.x * VW + v] = (m.valid && m.ng == 0) ? acc[v] : 0.0;
  __syncthreads();
  const int nw = blockDim.x >> 6;
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    const int cg = c / VW, v = c % VW;
    double s = 0.0;
    for (int w = 0; w < nw; ++w)
      for (int sl = 0; sl < m.RPW; ++sl) s += s_red[(w * 64 + sl * m.LPR + cg * NG) * VW + v];
    part[(int64_t)blockIdx.x * stride + off + c] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- SpMM row
// Nonzeros are taken U at a time: U independent (col, val) loads, then U
// independent gathers of the VW-wide row segments, so one row costs about
// nnz/(U*NG) dependent memory round trips.  Slots past the row end reuse the
// chunk's first nonzero (index j < row end, so its column is a valid column
// of this matrix, square or not) with weight zero; every load index stays in
// [row start, row end).
template <typename T, int VW> struct Unroll { static constexpr int U = (sizeof(T) * VW >= 32) ? 4 : 8; };

template <typename T, int VW, int NG>
__device__ __forceinline__ void row_product(int row, const RowMap &m,
                                            const int32_t *__restrict__ rowptr,
                                            const int32_t *__restrict__ col,
                                            const T *__restrict__ val, const T *__restrict__ X,
                                            int ldx, int k, T (&acc)[VW]) {
  constexpr int U = Unroll<T, VW>::U;
  for (int v = 0; v < VW; ++v) acc[v] = T(0);
  const int c0 = m.cg * VW;
  const bool colok = c0 < k;
  const bool vec = VW > 1 && (ldx % VW) == 0 && c0 + VW <= k;
  const int jb = rowptr[row], je = rowptr[row + 1];
  for (int j = jb + m.ng; j < je; j += U * NG) {
    int ci[U];
    T vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int jj = j + u * NG;
      const bool ok = jj < je;
      const int jc = ok ? jj : j;
      ci[u] = col[jc];
      const T vload = val[jc];
      vv[u] = ok ? vload : T(0);
    }
    if (colok) {
      if (vec) {
        VecT<T, VW> xs[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
          xs[u] = *reinterpret_cast<const VecT<T, VW> *>(X + (int64_t)ci[u] * ldx + c0);
#pragma unroll
        for (int u = 0; u < U; ++u)
          for (int v = 0; v < VW; ++v) acc[v] += vv[u] * xs[u].v[v];
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
          for (int v = 0; v < VW; ++v)
            if (c0 + v < k) acc[v] += vv[u] * X[(int64_t)ci[u] * ldx + c0 + v];
      }
    }
  }
  if (NG > 1) {
    for (int off = 1; off < NG; off <<= 1)
      for (int v = 0; v < VW; ++v) acc[v] += __shfl_xor(acc[v], off, 64);
  }
}

template <typename T, int VW>
__device__ __forceinline__ void load_row(const T *__restrict__ A, int64_t row, int ld, int c0, int k,
                                         T (&x)[VW]) {
  if (VW > 1 && (ld % VW) == 0 && c0 + VW <= k) {
    const VecT<T, VW> t = *reinterpret_cast<const VecT<T, VW> *>(A + row * ld + c0);
    for (int v = 0; v < VW; ++v) x[v] = t.v[v];
  } else {
    for (int v = 0; v < VW; ++v) x[v] = (c0 + v < k) ? A[row * ld + c0 + v] : T(0);
  }
}
template <typename T, int VW>
__device__ __forceinline__ void store_row(T *__restrict__ A, int64_t row, int ld, int c0, int k,
                                          const T (&x)[VW]) {
  if (VW > 1 && (ld % VW) == 0 && c0 + VW <= k) {
    VecT<T, VW> t;
    for (int v = 0; v < VW; ++v) t.v[v] = x[v];
    *reinterpret_cast<VecT<T, VW> *>(A + row * ld + c0) = t;
  } else {
    for (int v = 0; v < VW; ++v)
      if (c0 + v < k) A[row * ld + c0 + v] = x[v];
  }
}

// -------------------------------------------------------- generic SpMM
template <typename T, int VW, int NG>
__global__ void __launch_bounds__(256) k_spmm(int N, const int32_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ col,
                                              const T *__restrict__ val, const T *__restrict__ X,
                                              int ldx, T *__restrict__ Y, int ldy, int k, int CG,
                                              const T *__restrict__ B, int ldb, int mode,
                                              const int32_t *__restrict__ ord) {
  const RowMap m = row_map<NG>(CG);
  const int rows_per_block = (blockDim.x >> 6) * m.RPW;
  // uniform trip count per workgroup: every lane of a row group stays in the loop
  const int n_groups = (N + rows_per_block - 1) / rows_per_block;
  for (GroupIter gi = group_iter(n_groups); gi.g < gi.end; gi.g += gi.step) {
    const int pos = gi.g * rows_per_block + m.wave * m.RPW + m.slot;
    const bool rv = m.valid && pos < N;
    const int row = rv ? (ord ? ord[pos] : pos) : 0;
    T acc[VW];
    if (rv) row_product<T, VW, NG>(row, m, rowptr, col, val, X, ldx, k, acc);
    else {
      for (int v = 0; v < VW; ++v) acc[v] = T(0);
      if (NG > 1)
        for (int off = 1; off < NG; off <<= 1)
          for (int v = 0; v < VW; ++v) acc[v] += __shfl_xor(acc[v], off, 64);
    }
    if (rv && m.ng == 0 && m.cg * VW < k) {
      if (mode == 1) {
        T b[VW];
        load_row<T, VW>(B, row, ldb, m.cg * VW, k, b);
        for (int v = 0; v < VW; ++v) acc[v] = b[v] - acc[v];
      }
      store_row<T, VW>(Y, row, ldy, m.cg * VW, k, acc);
    }
  }
}

struct Shape {
  int VW, CG, NG;
};
static Shape pick_shape(int k, int ld) {
  Shape s;
  if (k == 1) {
    s.VW = 1; s.CG = 1; s.NG = 8;
    return s;
  }
  if (k % 4 == 0 && ld % 4 == 0 && k / 4 <= 64) s.VW = 4;
  else if (k % 2 == 0 && ld % 2 == 0 && k / 2 <= 64) s.VW = 2;
  else s.VW = 1;
  if (k > 64 * s.VW) s.VW = 4;  // wide blocks: VW=4 covers up to 256 columns
  s.CG = (k + s.VW - 1) / s.VW;
  s.NG = 1;
  return s;
}
// workgroups for N rows at RPW rows per wave (4 waves per workgroup); a
// multiple of 8 once there is more than one per XCD
static int grid_rows(int N, int RPW, int cap = 4096) {
  int rows_per_block = 4 * RPW;
  int b = (N + rows_per_block - 1) / rows_per_block;
  b = std::max(1, std::min(b, cap));
  if (b > 8) b = (b + 7) / 8 * 8;
  return b;
}

template <typename T>
static void spmm_dispatch(int N, const int32_t *rowptr, const int32_t *col, const T *val, const T *X,
                          int ldx, T *Y, int ldy, int k, const T *B, int ldb, int mode,
                          const int32_t *ord, hipStream_t s) {
  if (N <= 0 || k <= 0) return;
  Shape sh = pick_shape(k, std::min(ldx, ldy));
  // vector loads need VW-aligned rows: drop to scalar access otherwise
  auto aligned = [&](const void *p, int ld) {
    return p == nullptr || ((reinterpret_cast<uintptr_t>(p) % (sizeof(T) * sh.VW)) == 0 &&
                            (ld % sh.VW) == 0);
  };
  if (sh.VW > 1 && (!aligned(X, ldx) || !aligned(Y, ldy) || (mode == 1 && !aligned(B, ldb)))) {
    if (k > 64) sh = Shape{4, (k + 3) / 4, 1};  // wide: scalar fallback inside the kernel
    else sh = Shape{1, k, 1};
  }
  if (sh.CG > 64) sh = Shape{4, (k + 3) / 4, 1};
  const int RPW = 64 / (sh.CG * sh.NG);
  dim3 g(grid_rows(N, RPW)), b(256);
  if (sh.NG == 8)
    hipLaunchKernelGGL((k_spmm<T, 1, 8>), g, b, 0, s, N, rowptr, col, val, X, ldx, Y, ldy, k, 1, B,
                       ldb, mode, ord);
  else if (sh.VW == 4)
    hipLaunchKernelGGL((k_spmm<T, 4, 1>), g, b, 0, s, N, rowptr, col, val, X, ldx, Y, ldy, k, sh.CG,
                       B, ldb, mode, ord);
  else if (sh.VW == 2)
    hipLaunchKernelGGL((k_spmm<T, 2, 1>), g, b, 0, s, N, rowptr, col, val, X, ldx, Y, ldy, k, sh.CG,
                       B, ldb, mode, ord);
  else
    hipLaunchKernelGGL((k_spmm<T, 1, 1>), g, b, 0, s, N, rowptr, col, val, X, ldx, Y, ldy, k, sh.CG,
                       B, ldb, mode, ord);
}

void launch_spmm(int N, const int32_t *rowptr, const int32_t *col, const double *val,
                 const double *X, int ldx, double *Y, int ldy, int k, const double *B, int ldb,
                 int mode, const int32_t *ord, hipStream_t s) {
  spmm_dispatch<double>(N, rowptr, col, val, X, ldx, Y, ldy, k, B, ldb, mode, ord, s);
}
void launch_spmm_f32(int N, const int32_t *rowptr, const int32_t *col, const float *val,
                     const float *X, float *Y, int k, const int32_t *ord, hipStream_t s) {
  spmm_dispatch<float>(N, rowptr, col, val, X, k, Y, k, k, nullptr, k, 0, ord, s);
}

__global__ void k_scale_cols(int64_t n, int k, double *__restrict__ Y, const double *__restrict__ sc) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    Y[i] *= sc[i % k];
}
void launch_scale_cols(int N, int k, double *Y, const double *scale_dev, hipStream_t s) {
  int64_t n = (int64_t)N * k;
  if (n > 0)
    hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)),
                       dim3(256), 0, s, n, k, Y, scale_dev);
}

__global__ void k_refine_update(int64_t n, int k, const float *__restrict__ D,
                                const double *__restrict__ sc, double *__restrict__ X) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    X[i] += sc[i % k] * (double)D[i];
}
void launch_refine_update(int N, int k, const float *D, const double *scale, double *X, hipStream_t s) {
  int64_t n = (int64_t)N * k;
  if (n > 0)
    hipLaunchKernelGGL(k_refine_update, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)),
                       dim3(256), 0, s, n, k, D, scale, X);
}


// ============================================================ tiled SpMM
// q = S p for one block of BR consecutive rows at a time.  Everything the
// block reads is first copied into LDS with direct global->LDS loads (each
// lane moves one 16-byte chunk, a wave fills 64 consecutive chunks): the rows
// of p the block references (its halo, typically 2.5-6x BR rows) as a
// row-major [halo][k] image, and the block's contiguous runs of matrix values
// and 16-bit local column indices.  Then every (row, VW-column group) lane
// walks its row's nonzeros entirely in LDS.  The matrix is streamed once,
// the block vector is read from HBM about once (neighbouring blocks of one
// XCD share halo rows in L2), and no gather goes through the vector L1.
// Several workgroups per CU overlap one block's copies with another's math.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef const __attribute__((address_space(1))) void gbl_void_t;

// nchunks CB-byte chunks (CB = 16 or 4): chunk c comes from src_of(c) and
// lands at lds + CB c
template <int CB, typename F>
__device__ __forceinline__ void dma(int nchunks, unsigned char *lds, F src_of) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c0 = wave * 64; c0 < nchunks; c0 += nw * 64) {
    const int c = c0 + lane;
    if (c < nchunks) {
      lds_void_t *d = (lds_void_t *)(lds + (size_t)c0 * CB);
      if constexpr (CB == 16) __builtin_amdgcn_global_load_lds((gbl_void_t *)src_of(c), d, 16, 0, 0);
      else __builtin_amdgcn_global_load_lds((gbl_void_t *)src_of(c), d, 4, 0, 0);
    }
  }
}

// LDS layout of one block: halo image (max_halo rows, then one row of zeros
// that the index runs' padding points at), values, local indices; every
// region a whole number of 1 KB wave fills.  Several workgroups per CU
// overlap one block's copies with another block's arithmetic.
struct TLayout {
  int halo, vals, idx;  // byte offsets
  int total;
};
__host__ __device__ __forceinline__ int round_kb(int b) { return (b + 1023) / 1024 * 1024; }
__host__ __device__ __forceinline__ TLayout tile_layout(int max_halo, int max_nnz, int max_pnz, int rowbytes,
                                                        int elem) {
  TLayout L;
  L.halo = 0;
  L.vals = round_kb((max_halo + 1) * rowbytes);
  L.idx = L.vals + round_kb(max_nnz * elem + 32);
  L.total = L.idx + round_kb(max_pnz * 2 + 32);
  return L;
}

// Q = S P for the rows of the tiling, partial p.q per workgroup.  VW columns
// per lane (k % VW == 0); halo rows copied in HCB-byte chunks, HCB = 16 when
// k * sizeof(T) % 16 == 0, else 4; N * k * sizeof(T) < 2^32 (byte offsets
// into P are 32-bit).  All checked by the host.
// MODE 0: the PCG phase (Q = S P, p.q partials, skipped once the solver
// stopped); MODE 1: Q = S P; MODE 2: Q = B - S P, with per-workgroup column
// partials of the squared residual when part is given.
// SC: lcol holds LDS byte offsets of the halo rows (local index x rowbytes)
// instead of local indices, which saves one address instruction per nonzero.
//
// Every address a block's copies need is in registers before the block
// starts: while block i is computed from LDS, each lane fetches the halo
// list entries of its first PC copy chunks of block i+1 (and that block's
// CSR range and its first row slot), so that the copies of block i+1 issue
// back to back instead of one dependent index load each.
template <typename T, int VW, int HCB, int TB, int MODE, bool SC>
__global__ void __launch_bounds__(TB) k_tpcg_A(int N, int k, int ldp, int ldq, int BR, int nblk, int max_halo,
                                                int max_nnz, int max_pnz,
                                                const int32_t *__restrict__ halo_ptr,
                                                const int32_t *__restrict__ halo_col,
                                                const int32_t *__restrict__ hself,
                                                const int32_t *__restrict__ rowptr,
                                                const uint16_t *__restrict__ lcol,
                                                const int32_t *__restrict__ pptr,
                                                const uint32_t *__restrict__ rmeta,
                                                const T *__restrict__ val, const T *__restrict__ P,
                                                T *__restrict__ Q, double *__restrict__ part,
                                                const Control *ctl, const T *__restrict__ Bm) {
  if (MODE == 0 && ctl && ctl->stop) return;
  extern __shared__ __align__(16) unsigned char t_smem[];
  constexpr int PC = 8;  // copy chunks per lane whose halo rows are fetched one block ahead
  const int CG = k / VW;
  const unsigned rowbytes = (unsigned)k * sizeof(T);   // one halo row in LDS
  const unsigned pitch = (unsigned)ldp * sizeof(T);     // one row of P in memory
  const int CH = (int)rowbytes / HCB;
  const TLayout L = tile_layout(max_halo, max_nnz, max_pnz, (int)rowbytes, (int)sizeof(T));
  // fixed (row slot, column group) per thread: RPP rows per pass
  const int RPP = (int)blockDim.x / CG;
  const int cg = threadIdx.x % CG, rslot = threadIdx.x / CG;
  const bool active = rslot < RPP;
  // copy chunk c = wave 64 + lane + i TB of a block is byte (c % CH) HCB of
  // halo row c / CH; for i < PC: hpb[i] = (c / CH) << 10 | (c % CH) HCB
  // (a halo row is at most 512 bytes)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned hpb[PC];
#pragma unroll
  for (int i = 0; i < PC; ++i) {
    const int c = wave * 64 + lane + i * TB;
    const int h = c / CH;
    hpb[i] = ((unsigned)h << 10) | (unsigned)((c - h * CH) * HCB);
  }
  // chunks from i = PC on (rare: halos above PC TB / CH rows) walk on from here
  const int cr = wave * 64 + lane + PC * TB;
  const int hr0 = cr / CH, chr0 = cr - hr0 * CH;
  const int dh = TB / CH, dch = TB - dh * CH;
  double apq[VW];
  for (int v = 0; v < VW; ++v) apq[v] = 0.0;
  const unsigned char *Pb = reinterpret_cast<const unsigned char *>(P);
  const unsigned char *Vb = reinterpret_cast<const unsigned char *>(val);
  const unsigned char *Ib = reinterpret_cast<const unsigned char *>(lcol);
  const GroupIter gi = group_iter(nblk);
  // the zero halo row, and the value region (read up to 7 entries past a
  // row's end, always finite after this)
  for (unsigned o = threadIdx.x * 4; o < rowbytes; o += TB * 4)
    *reinterpret_cast<float *>(t_smem + L.halo + (unsigned)max_halo * rowbytes + o) = 0.f;
  for (int o = threadIdx.x * 16; o < L.idx - L.vals; o += TB * 16)
    *reinterpret_cast<uint4 *>(t_smem + L.vals + o) = make_uint4(0u, 0u, 0u, 0u);
  // the block about to be copied: halo list start and size, CSR range,
  // padded index range, halo rows of this lane's first PC chunks, first row
  // slot of this lane
  int hb0 = 0, nh = 0, j0 = 0, j1 = 0, p0 = 0, p1 = 0;
  int hrow[PC];
  uint2 rm0 = make_uint2(0u, 0u);
  const uint2 *rm2 = reinterpret_cast<const uint2 *>(rmeta);
  if (gi.g < gi.end) {
    const int b = gi.g, r0 = b * BR, nr = min(BR, N - r0);
    hb0 = halo_ptr[b];
    nh = halo_ptr[b + 1] - hb0;
    j0 = rowptr[r0];
    j1 = rowptr[r0 + nr];
    p0 = pptr[b];
    p1 = pptr[b + 1];
#pragma unroll
    for (int i = 0; i < PC; ++i) {
      const int h = (int)(hpb[i] >> 10);
      hrow[i] = halo_col[hb0 + (h < nh ? h : 0)];  // unconditional loads: one wait covers all
    }
    if (active && rslot < nr) rm0 = rm2[r0 + rslot];
  }
  for (int b = gi.g; b < gi.end; b += gi.step) {
    const int r0 = b * BR, nr = min(BR, N - r0);
    const int hs = hself[b];  // halo position of row r0; rows r0.. are consecutive there
    __syncthreads();          // the previous block is done with the LDS image
    // the fetched halo rows are in (one wait here, none between the copies)
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    {
      unsigned char *dst = t_smem + L.halo + (unsigned)(wave * 64) * HCB;
#pragma unroll
      for (int i = 0; i < PC; ++i) {
        if ((int)(hpb[i] >> 10) < nh) {
          const unsigned off = (unsigned)hrow[i] * pitch + (hpb[i] & 1023u);
          lds_void_t *d = (lds_void_t *)(dst + (unsigned)(i * TB) * HCB);
          if constexpr (HCB == 16) __builtin_amdgcn_global_load_lds((gbl_void_t *)(Pb + off), d, 16, 0, 0);
          else __builtin_amdgcn_global_load_lds((gbl_void_t *)(Pb + off), d, 4, 0, 0);
        }
      }
      const int total = nh * CH;
      if (wave * 64 + PC * TB < total) {
        const int32_t *hl = halo_col + hb0;
        int h = hr0, ch = chr0;
        for (int c0 = wave * 64 + PC * TB; c0 < total; c0 += TB) {
          if (c0 + lane < total) {
            const unsigned off = (unsigned)hl[h] * pitch + (unsigned)(ch * HCB);
            lds_void_t *d = (lds_void_t *)(t_smem + L.halo + (unsigned)c0 * HCB);
            if constexpr (HCB == 16) __builtin_amdgcn_global_load_lds((gbl_void_t *)(Pb + off), d, 16, 0, 0);
            else __builtin_amdgcn_global_load_lds((gbl_void_t *)(Pb + off), d, 4, 0, 0);
          }
          h += dh;
          ch += dch;
          if (ch >= CH) {
            ch -= CH;
            h += 1;
          }
        }
      }
    }
    const int64_t va = ((int64_t)j0 * sizeof(T)) & ~(int64_t)15;
    const int64_t vb = ((int64_t)j1 * sizeof(T) + 15) & ~(int64_t)15;
    dma<16>((int)((vb - va) / 16), t_smem + L.vals, [&](int c) { return Vb + va + (int64_t)c * 16; });
    // padded index runs: 16-byte aligned at both ends
    dma<16>((p1 - p0) / 8, t_smem + L.idx, [&](int c) { return Ib + (int64_t)p0 * 2 + (int64_t)c * 16; });
    // this block's values in LDS, addressed from its first nonzero; its
    // index runs from the image start
    const T *vs = reinterpret_cast<const T *>(t_smem + L.vals + ((int64_t)j0 * sizeof(T) - va));
    const uint16_t *is = reinterpret_cast<const uint16_t *>(t_smem + L.idx);
    const uint2 m0 = rm0;
    // the next block's list range and CSR range (scalar loads, land with the copies)
    const int bn = b + gi.step;
    const bool more = bn < gi.end;
    int r0n = 0, nrn = 0;
    if (more) {
      r0n = bn * BR;
      nrn = min(BR, N - r0n);
      hb0 = halo_ptr[bn];
      nh = halo_ptr[bn + 1] - hb0;
      j0 = rowptr[r0n];
      j1 = rowptr[r0n + nrn];
      p0 = pptr[bn];
      p1 = pptr[bn + 1];
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies have landed
    __syncthreads();                // ... and every wave's
    // the next block's halo rows and first row slot, in flight while this
    // block is computed
    if (more) {
#pragma unroll
      for (int i = 0; i < PC; ++i) {
        const int h = (int)(hpb[i] >> 10);
        hrow[i] = halo_col[hb0 + (h < nh ? h : 0)];
      }
      rm0 = (active && rslot < nrn) ? rm2[r0n + rslot] : make_uint2(0u, 0u);
    }
    const T *xs = reinterpret_cast<const T *>(t_smem + L.halo) + cg * VW;
    const unsigned char *xsb = t_smem + L.halo + cg * VW * sizeof(T);
    auto do_row = [&](const uint2 m) {
      const int rr = (int)(m.x >> 24);  // longest rows first
      const int row = r0 + rr;
      const int jb = (int)(m.x & 0xffffu), len = (int)((m.x >> 16) & 0xffu);
      const uint16_t *ir = is + m.y;  // this row's index run, 16-byte aligned
      T acc[VW];
      for (int v = 0; v < VW; ++v) acc[v] = T(0);
      // eight nonzeros per step: one aligned 16-byte read of their local
      // indices, issued one step ahead so that it overlaps the previous
      // step's gathers; a tail of at most four takes one four-wide step.
      // Slots past the row's end point at the zero halo row; their weights
      // (the following entries of the LDS value image, finite) then add
      // exact zeros.  The run is padded to a multiple of eight entries, so
      // the read ahead stays inside it.
      auto step = [&](auto nu, const uint4 iw, int j) {
        constexpr int NU = decltype(nu)::value;
        unsigned li[8];
        li[0] = iw.x & 0xffffu; li[1] = iw.x >> 16; li[2] = iw.y & 0xffffu; li[3] = iw.y >> 16;
        li[4] = iw.z & 0xffffu; li[5] = iw.z >> 16; li[6] = iw.w & 0xffffu; li[7] = iw.w >> 16;
        T vv[NU];
        VecT<T, VW> x[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) vv[u] = vs[jb + j + u];
#pragma unroll
        for (int u = 0; u < NU; ++u)
          x[u] = SC ? *reinterpret_cast<const VecT<T, VW> *>(xsb + li[u])
                    : *reinterpret_cast<const VecT<T, VW> *>(xs + __umul24(li[u], (unsigned)k));
        // all of the step's LDS reads are issued before the first product
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < NU; ++u)
          for (int v = 0; v < VW; ++v) acc[v] += vv[u] * x[u].v[v];
      };
      uint4 iw = make_uint4(0u, 0u, 0u, 0u);
      if (len > 0) iw = *reinterpret_cast<const uint4 *>(ir);
      int j = 0;
      for (; j + 8 <= len; j += 8) {
        const uint4 cur = iw;
        if (j + 8 < len) iw = *reinterpret_cast<const uint4 *>(ir + j + 8);
        step(std::integral_constant<int, 8>{}, cur, j);
      }
      if (len - j > 4) step(std::integral_constant<int, 8>{}, iw, j);
      else if (len - j > 0) step(std::integral_constant<int, 4>{}, iw, j);
      if constexpr (MODE == 0) {
        const VecT<T, VW> p = *reinterpret_cast<const VecT<T, VW> *>(xs + __umul24(hs + rr, k));
        for (int v = 0; v < VW; ++v) apq[v] += (double)p.v[v] * (double)acc[v];
      } else if constexpr (MODE == 2) {
        T b[VW];
        load_row<T, VW>(Bm, row, ldq, cg * VW, k, b);
        for (int v = 0; v < VW; ++v) acc[v] = b[v] - acc[v];
        for (int v = 0; v < VW; ++v) apq[v] += (double)acc[v] * (double)acc[v];
      }
      store_row<T, VW>(Q, row, ldq, cg * VW, k, acc);
    };
    // the first row of every lane comes with the block (no memory wait
    // here: the next block's halo rows stay in flight during the compute);
    // blocks taller than one pass load the later row slots
    if (active && rslot < nr) do_row(m0);
    for (int rs = rslot + RPP; active && rs < nr; rs += RPP) do_row(rm2[r0 + rs]);
  }
  if (MODE == 1 || part == nullptr) return;
  // per-workgroup column partials (fixed order): thread t holds columns
  // [(t % CG) VW, (t % CG) VW + VW) of its rows; the LDS image is free now
  __syncthreads();
  double *s_red = reinterpret_cast<double *>(t_smem);
  for (int v = 0; v < VW; ++v) s_red[threadIdx.x * VW + v] = active ? apq[v] : 0.0;
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    const int g = c / VW, v = c % VW;
    double sum = 0.0;
    for (int t = g; t < RPP * CG; t += CG) sum += s_red[t * VW + v];
    part[(int64_t)blockIdx.x * k + c] = sum;
  }
}

size_t tiled_lds_bytes(const Tiling &t, int k, size_t elem) {
  if (!t.nblk || (k * elem) % 4 != 0) return 0;
  return (size_t)tile_layout(t.max_halo, t.max_nnz, t.max_pnz, k * (int)elem, (int)elem).total;
}

// launch shape of the tiled SpMM for this operator: VW, halo chunk, grid, LDS
struct TShape {
  int VW = 1, HCB = 16, grid = 0, TB = 256;
  size_t lds = 0;
};
constexpr size_t TILE_LDS_MAX = 160 * 1024 - 512;
// tb: threads per workgroup (256, 512 or 1024; the waves share one block)
// ld: row pitch (elements) of the gathered operand; a16: its base address and
// pitch allow 16-byte halo chunks
template <typename T>
static TShape tiled_shape(const Tiling &t, int k, int N, int nblk_max, int tb, int ld = 0, bool a16 = true) {
  TShape sh;
  if (ld <= 0) ld = k;
  const int vw16 = 16 / (int)sizeof(T);
  sh.VW = (k % vw16 == 0) ? vw16 : 1;
  sh.TB = (tb == 512 || tb == 1024) ? tb : 256;
  sh.HCB = ((k * sizeof(T)) % 16 == 0 && (ld * sizeof(T)) % 16 == 0 && a16) ? 16 : 4;
  sh.lds = tiled_lds_bytes(t, k, sizeof(T));
  if (sh.lds) sh.lds = std::max(sh.lds, (size_t)sh.TB * sh.VW * sizeof(double));  // final column reduction
  if (sh.lds == 0 || sh.lds > TILE_LDS_MAX || (double)N * ld * sizeof(T) >= 4294967296.0) return sh;
  const int per_cu = std::max(1, std::min(2048 / sh.TB, (int)(TILE_LDS_MAX / sh.lds)));
  int g = std::min(t.nblk, 256 * per_cu);
  if (g > 8) g = g / 8 * 8;
  sh.grid = std::max(1, std::min(g, nblk_max));
  return sh;
}

template <typename T, int VW, int HCB, int TB, int MODE, bool SC = false>
static int launch_tpcg_A_t(int N, int k, int ldp, int ldq, const Tiling &t, const TShape &sh,
                           const int32_t *rowptr, const T *val, const T *P, T *Q, double *part, const Control *ctl,
                           const T *Bm, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void *)k_tpcg_A<T, VW, HCB, TB, MODE, SC>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)TILE_LDS_MAX) != hipSuccess)
      return -1;
    attr = true;
  }
  hipLaunchKernelGGL((k_tpcg_A<T, VW, HCB, TB, MODE, SC>), dim3(sh.grid), dim3(TB), sh.lds, s, N, k, ldp, ldq,
                     t.BR, t.nblk, t.max_halo, t.max_nnz, t.max_pnz, t.halo_ptr, t.halo_col, t.hself, rowptr,
                     SC ? t.lbyte : t.lcol, t.pptr, t.rmeta, val, P, Q, part, ctl, Bm);
  return 0;
}
// the byte-offset index runs serve FP32 halo rows of exactly lb_rowbytes
template <typename T>
static bool use_lbyte(const Tiling &t, const TShape &sh, int k) {
  return sizeof(T) == 4 && sh.VW == 4 && sh.HCB == 16 && t.lbyte && k * (int)sizeof(T) == t.lb_rowbytes;
}
template <typename T, int MODE>
static int launch_tpcg_A_m(int N, int k, int ldp, int ldq, const Tiling &t, const TShape &sh,
                           const int32_t *rowptr, const T *val, const T *P, T *Q, double *part, const Control *ctl,
                           const T *Bm, hipStream_t s) {
  constexpr int V16 = 16 / sizeof(T);
#define KS_TL(VW, HCB, TB) \
  return launch_tpcg_A_t<T, VW, HCB, TB, MODE>(N, k, ldp, ldq, t, sh, rowptr, val, P, Q, part, ctl, Bm, s)
#define KS_TLS(TB) \
  return launch_tpcg_A_t<T, V16, 16, TB, MODE, true>(N, k, ldp, ldq, t, sh, rowptr, val, P, Q, part, ctl, Bm, s)
  if constexpr (sizeof(T) == 4) {
    if (use_lbyte<T>(t, sh, k)) {
      if (sh.TB == 1024) KS_TLS(1024);
      if (sh.TB == 512) KS_TLS(512);
      KS_TLS(256);
    }
  }
#undef KS_TLS
  if (sh.TB == 1024) {
    if (sh.VW == V16) KS_TL(V16, 16, 1024);
    if (sh.HCB == 16) KS_TL(1, 16, 1024);
    KS_TL(1, 4, 1024);
  }
  if (sh.TB == 512) {
    if (sh.VW == V16) KS_TL(V16, 16, 512);
    if (sh.HCB == 16) KS_TL(1, 16, 512);
    KS_TL(1, 4, 512);
  }
  if (sh.VW == V16) KS_TL(V16, 16, 256);
  if (sh.HCB == 16) KS_TL(1, 16, 256);
  KS_TL(1, 4, 256);
#undef KS_TL
}
template <typename T>
static int launch_tpcg_A(int N, int k, const Tiling &t, const TShape &sh, const int32_t *rowptr,
                         const T *val, const T *P, T *Q, double *part, const Control *ctl, hipStream_t s) {
  return launch_tpcg_A_m<T, 0>(N, k, k, k, t, sh, rowptr, val, P, Q, part, ctl, nullptr, s);
}

// Y = S X (B == nullptr) or Y = B - S X with the halo-tile kernel (FP64, X
// and Y row-major [N][k]); -1 when the tiling cannot serve this k
int launch_spmm_tiled(int N, int k, const Tiling &t, int tb, const int32_t *rowptr, const double *val,
                      const double *X, double *Y, const double *B, hipStream_t s) {
  const TShape sh = tiled_shape<double>(t, k, N, 1 << 30, tb);
  if (sh.grid <= 0) return -1;
  if (B) return launch_tpcg_A_m<double, 2>(N, k, k, k, t, sh, rowptr, val, X, Y, nullptr, nullptr, B, s);
  return launch_tpcg_A_m<double, 1>(N, k, k, k, t, sh, rowptr, val, X, Y, nullptr, nullptr, nullptr, s);
}

// Y = B - S X through the halo tiles with per-workgroup column partials of
// sum_i Y[i][c]^2 in part[b][c] (FP64, [N][k]); returns the number of
// partial rows, or -1 (nothing launched) when the tiling cannot serve k
int launch_residual_tiled_norms(int N, int k, const Tiling &t, int tb, const int32_t *rowptr, const double *val,
                                const double *X, double *Y, const double *B, double *part, hipStream_t s) {
  const TShape sh = tiled_shape<double>(t, k, N, 1 << 30, tb);
  if (sh.grid <= 0 || !B || !part) return -1;
  if (launch_tpcg_A_m<double, 2>(N, k, k, k, t, sh, rowptr, val, X, Y, part, nullptr, B, s) < 0) return -1;
  return sh.grid;
}

// FP32 form (Y = S X or Y = B - S X, [N][k] row-major); -1 when the tiling
// cannot serve k FP32 columns
int launch_spmm_tiled_f32(int N, int k, const Tiling &t, int tb, const int32_t *rowptr, const float *val,
                          const float *X, float *Y, const float *B, hipStream_t s) {
  const TShape sh = tiled_shape<float>(t, k, N, 1 << 30, tb);
  if (sh.grid <= 0) return -1;
  if (B) return launch_tpcg_A_m<float, 2>(N, k, k, k, t, sh, rowptr, val, X, Y, nullptr, nullptr, B, s);
  return launch_tpcg_A_m<float, 1>(N, k, k, k, t, sh, rowptr, val, X, Y, nullptr, nullptr, nullptr, s);
}
bool tiled_fits_f32(int N, int k, const Tiling &t, int tb) { return tiled_shape<float>(t, k, N, 1 << 30, tb).grid > 0; }

// The same over column chunks of width kc: X, Y (and B) with row pitches
// ldx, ldy (elements); -1 (nothing launched) when the tiling cannot serve a
// chunk
int launch_spmm_tiled_cols(int N, int k, int ldx, int ldy, int kc, const Tiling &t, int tb, const int32_t *rowptr,
                           const double *val, const double *X, double *Y, const double *B, hipStream_t s) {
  if (kc < 1 || ldx < k || ldy < k) return -1;
  auto shape = [&](int c0) {
    const int w = std::min(kc, k - c0);
    const bool a16 = ((c0 * sizeof(double)) % 16 == 0) && ((uintptr_t)X % 16 == 0);
    return tiled_shape<double>(t, w, N, 1 << 30, tb, ldx, a16);
  };
  for (int c0 = 0; c0 < k; c0 += kc)
    if (shape(c0).grid <= 0) return -1;
  for (int c0 = 0; c0 < k; c0 += kc) {
    const int w = std::min(kc, k - c0);
    const TShape sh = shape(c0);
    const int r = B ? launch_tpcg_A_m<double, 2>(N, w, ldx, ldy, t, sh, rowptr, val, X + c0, Y + c0, nullptr,
                                                 nullptr, B + c0, s)
                    : launch_tpcg_A_m<double, 1>(N, w, ldx, ldy, t, sh, rowptr, val, X + c0, Y + c0, nullptr,
                                                 nullptr, nullptr, s);
    if (r < 0) return -1;
  }
  return 0;
}

// ================================================================== PCG
// Every phase writes per-block column partials; a one-workgroup kernel then
// combines them in a fixed order (deterministic, and no device-scope fences
// inside the streaming kernels: on a multi-XCD chip those write back L2).
constexpr int RED_THREADS = 1024;

// sums[c] = sum_b part[b][c] for c < W (W <= 192), fixed order
__device__ __forceinline__ void reduce_partials(const double *__restrict__ part, int nblk, int W,
                                                double *s_sum) {
  __shared__ double s_red[RED_THREADS];
  const int G = max(1, RED_THREADS / W);
  const int t = threadIdx.x;
  double acc = 0.0;
  if (t < G * W) {
    // partials b = g, g + G, g + 2G, ... added in that order; sixteen
    // loads in flight per step
    const int c = t % W, g = t / W;
    for (int b = g; b < nblk; b += 16 * G) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = (b + u * G < nblk) ? part[(int64_t)(b + u * G) * W + c] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += v[u];
    }
  }
  s_red[t] = acc;
  __syncthreads();
  if (t < W) {
    double tot = 0.0;
    for (int g = 0; g < G; ++g) tot += s_red[g * W + t];
    s_sum[t] = tot;
  }
  __syncthreads();
}

// I: R = B - S X, P = D^{-1} R; partials of b.b, r.r, r.z
template <typename T, int VW, int NG>
__global__ void __launch_bounds__(256) k_pcg_init(int N, int k, int CG,
                                                  const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col,
                                                  const T *__restrict__ val,
                                                  const T *__restrict__ diag,
                                                  const T *__restrict__ Bm, const T *__restrict__ X,
                                                  T *__restrict__ R, T *__restrict__ P,
                                                  double *__restrict__ part,
                                                  const int32_t *__restrict__ ord, int have_r) {
  __shared__ double s_red[256 * VW];
  const RowMap m = row_map<NG>(CG);
  const int rows_per_block = (blockDim.x >> 6) * m.RPW;
  double abb[VW], arr[VW], arz[VW];
  for (int v = 0; v < VW; ++v) abb[v] = arr[v] = arz[v] = 0.0;
  const int n_groups = (N + rows_per_block - 1) / rows_per_block;
  for (GroupIter gi = group_iter(n_groups); gi.g < gi.end; gi.g += gi.step) {
    const int pos = gi.g * rows_per_block + m.wave * m.RPW + m.slot;
    const bool rv = m.valid && pos < N;
    const int row = rv ? (ord ? ord[pos] : pos) : 0;
    T acc[VW];
    if (have_r) {
      // R already holds b - S x (halo-tile kernel), or x = 0: no S x needed
      for (int v = 0; v < VW; ++v) acc[v] = T(0);
    } else if (rv) row_product<T, VW, NG>(row, m, rowptr, col, val, X, k, k, acc);
    else {
      for (int v = 0; v < VW; ++v) acc[v] = T(0);
      if (NG > 1)
        for (int off = 1; off < NG; off <<= 1)
          for (int v = 0; v < VW; ++v) acc[v] += __shfl_xor(acc[v], off, 64);
    }
    if (rv && m.ng == 0 && m.cg * VW < k) {
      T b[VW], r[VW], p[VW];
      load_row<T, VW>(Bm, row, k, m.cg * VW, k, b);
      if (have_r == 1) load_row<T, VW>(R, row, k, m.cg * VW, k, r);
      const T d = diag[row];
      for (int v = 0; v < VW; ++v) {
        if (have_r != 1) r[v] = b[v] - acc[v];  // acc = 0 when x = 0 (have_r == 2)
        p[v] = r[v] / d;
        abb[v] += (double)b[v] * (double)b[v];
        arr[v] += (double)r[v] * (double)r[v];
        arz[v] += (double)r[v] * (double)p[v];
      }
      store_row<T, VW>(R, row, k, m.cg * VW, k, r);
      store_row<T, VW>(P, row, k, m.cg * VW, k, p);
    }
  }
  block_cols<VW, NG>(abb, m, k, CG, s_red, part, 3 * k, 0);
  block_cols<VW, NG>(arr, m, k, CG, s_red, part, 3 * k, k);
  block_cols<VW, NG>(arz, m, k, CG, s_red, part, 3 * k, 2 * k);
}

// Start of the FP32 correction solve of the mixed-precision refinement,
// from the FP64 residual W and the column scales sc: R = float(W sc) (the
// right-hand side; the correction starts from X = 0), P = D^{-1} R, X = 0,
// and the b.b, r.r, r.z partials in k_pcg_init's layout.  sc[k + c] >= 1
// relaxes column c's stopping test: b.b is recorded times sc[k + c]^2, so
// the column stops at relative residual tol sc[k + c].
template <int VW>
__global__ void __launch_bounds__(256) k_refine_prep(int N, int k, int CG, const double *__restrict__ W,
                                                     const double *__restrict__ sc, const float *__restrict__ diag,
                                                     float *__restrict__ R, float *__restrict__ P,
                                                     float *__restrict__ X, double *__restrict__ part) {
  __shared__ double s_red[256 * VW];
  const RowMap m = row_map<1>(CG);
  const int rows_per_block = (blockDim.x >> 6) * m.RPW;
  const int c0 = m.cg * VW;
  double sv[VW], arr[VW], arz[VW];
  for (int v = 0; v < VW; ++v) {
    sv[v] = (c0 + v < k) ? sc[c0 + v] : 0.0;
    arr[v] = arz[v] = 0.0;
  }
  double rx[VW];
  for (int v = 0; v < VW; ++v) rx[v] = (c0 + v < k) ? sc[k + c0 + v] * sc[k + c0 + v] : 1.0;
  const int n_groups = (N + rows_per_block - 1) / rows_per_block;
  for (GroupIter gi = group_iter(n_groups); gi.g < gi.end; gi.g += gi.step) {
    const int row = gi.g * rows_per_block + m.wave * m.RPW + m.slot;
    if (!m.valid || c0 >= k || row >= N) continue;
    double w[VW];
    load_row<double, VW>(W, row, k, c0, k, w);
    const float d = diag[row];
    float r[VW], p[VW], z[VW];
    for (int v = 0; v < VW; ++v) {
      r[v] = (float)(w[v] * sv[v]);
      p[v] = r[v] / d;
      z[v] = 0.f;
      arr[v] += (double)r[v] * (double)r[v];
      arz[v] += (double)r[v] * (double)p[v];
    }
    store_row<float, VW>(R, row, k, c0, k, r);
    store_row<float, VW>(P, row, k, c0, k, p);
    store_row<float, VW>(X, row, k, c0, k, z);
  }
  double abb[VW];
  for (int v = 0; v < VW; ++v) abb[v] = arr[v] * rx[v];
  block_cols<VW, 1>(abb, m, k, CG, s_red, part, 3 * k, 0);
  block_cols<VW, 1>(arr, m, k, CG, s_red, part, 3 * k, k);
  block_cols<VW, 1>(arz, m, k, CG, s_red, part, 3 * k, 2 * k);
}

int launch_refine_prep(int N, int k, const double *W, const double *sc, const float *diag, float *X, PCGWork &w,
                       hipStream_t s) {
  if (N <= 0 || k <= 0 || k > MAX_K) return -1;
  const int VW = (k % 4 == 0) ? 4 : 1;
  const int CG = k / VW;
  if (CG > 64) return -1;
  const int nb = std::min(grid_rows(N, 64 / CG, pcg_blocks()), w.nblk_max);
  float *R = reinterpret_cast<float *>(w.R), *P = reinterpret_cast<float *>(w.P);
  double *part = reinterpret_cast<double *>(w.part);
  if (VW == 4)
    hipLaunchKernelGGL(k_refine_prep<4>, dim3(nb), dim3(256), 0, s, N, k, CG, W, sc, diag, R, P, X, part);
  else
    hipLaunchKernelGGL(k_refine_prep<1>, dim3(nb), dim3(256), 0, s, N, k, CG, W, sc, diag, R, P, X, part);
  w.prep_nblk = nb;
  return 0;
}

__global__ void __launch_bounds__(RED_THREADS) k_red_init(int k, int nblk, const double *part,
                                                          Control *ctl, ColState *cs, double tol) {
  __shared__ double s_sum[192];
  reduce_partials(part, nblk, 3 * k, s_sum);
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    ColState st;
    st.bb = s_sum[c]; st.rr = s_sum[k + c]; st.rz = s_sum[2 * k + c]; st.rz_new = st.rz;
    st.pq = 0.0; st.alpha = 0.0; st.alpha_prev = 0.0; st.beta = 0.0; st.iters = 0;
    st.active = (st.bb > 0.0) && (st.rr > tol * tol * st.bb);
    cs[c] = st;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int any = 0;
    for (int c = 0; c < k; ++c) any |= cs[c].active;
    ctl->stop = !any;
    ctl->skip = -1;   // iteration in which the solver stopped (none yet)
    ctl->breakdown = 0;
  }
}

// A: Q = S P, partial p.q
template <typename T, int VW, int NG>
__global__ void __launch_bounds__(256) k_pcg_A(int N, int k, int CG, const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col,
                                               const T *__restrict__ val, const T *__restrict__ P,
                                               T *__restrict__ Q, double *__restrict__ part,
                                               const Control *ctl,
                                               const int32_t *__restrict__ ord) {
  if (ctl->stop) return;
  __shared__ double s_red[256 * VW];
  const RowMap m = row_map<NG>(CG);
  const int rows_per_block = (blockDim.x >> 6) * m.RPW;
  double apq[VW];
  for (int v = 0; v < VW; ++v) apq[v] = 0.0;
  const int n_groups = (N + rows_per_block - 1) / rows_per_block;
  for (GroupIter gi = group_iter(n_groups); gi.g < gi.end; gi.g += gi.step) {
    const int pos = gi.g * rows_per_block + m.wave * m.RPW + m.slot;
    const bool rv = m.valid && pos < N;
    const int row = rv ? (ord ? ord[pos] : pos) : 0;
    T acc[VW];
    if (rv) row_product<T, VW, NG>(row, m, rowptr, col, val, P, k, k, acc);
    else {
      for (int v = 0; v < VW; ++v) acc[v] = T(0);
      if (NG > 1)
        for (int off = 1; off < NG; off <<= 1)
          for (int v = 0; v < VW; ++v) acc[v] += __shfl_xor(acc[v], off, 64);
    }
    if (rv && m.ng == 0 && m.cg * VW < k) {
      T p[VW];
      load_row<T, VW>(P, row, k, m.cg * VW, k, p);
      for (int v = 0; v < VW; ++v) apq[v] += (double)p[v] * (double)acc[v];
      store_row<T, VW>(Q, row, k, m.cg * VW, k, acc);
    }
  }
  block_cols<VW, NG>(apq, m, k, CG, s_red, part, k, 0);
}

__global__ void __launch_bounds__(RED_THREADS) k_red_A(int k, int nblk, const double *part,
                                                       Control *ctl, ColState *cs) {
  if (ctl->stop) return;
  __shared__ double s_sum[192];
  reduce_partials(part, nblk, k, s_sum);
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    const double pq = s_sum[c];
    ColState st = cs[c];
    st.pq = pq;
    st.alpha_prev = st.alpha;
    st.alpha = 0.0;
    if (st.active) {
      if (!(pq > 0.0)) ctl->breakdown = 1;
      else st.alpha = st.rz / pq;
    }
    cs[c] = st;
  }
}

// B: R -= alpha Q; partials r.z and r.r
template <typename T, int VW>
__global__ void __launch_bounds__(256) k_pcg_B(int N, int k, int CG, const T *__restrict__ diag,
                                               const T *__restrict__ Q, T *__restrict__ R,
                                               double *__restrict__ part, const Control *ctl,
                                               const ColState *cs) {
  if (ctl->stop) return;
  __shared__ double s_red[256 * VW];
  __shared__ double s_alpha[MAX_K];
  for (int c = threadIdx.x; c < k; c += blockDim.x) s_alpha[c] = cs[c].alpha;
  __syncthreads();
  const RowMap m = row_map<1>(CG);
  const int rows_per_block = (blockDim.x >> 6) * m.RPW;
  double arz[VW], arr[VW];
  for (int v = 0; v < VW; ++v) arz[v] = arr[v] = 0.0;
  const int c0 = m.cg * VW;
  T al[VW];
  for (int v = 0; v < VW; ++v) al[v] = (c0 + v < k) ? (T)s_alpha[c0 + v] : T(0);
  const int n_groups = (N + rows_per_block - 1) / rows_per_block;
  for (GroupIter gi = group_iter(n_groups); gi.g < gi.end; gi.g += gi.step) {
    const int row = gi.g * rows_per_block + m.wave * m.RPW + m.slot;
    if (!m.valid || c0 >= k || row >= N) continue;
    T q[VW], r[VW];
    load_row<T, VW>(Q, row, k, c0, k, q);
    load_row<T, VW>(R, row, k, c0, k, r);
    const T d = diag[row];
    for (int v = 0; v < VW; ++v) {
      r[v] -= al[v] * q[v];
      arr[v] += (double)r[v] * (double)r[v];
      arz[v] += (double)r[v] * (double)(r[v] / d);
    }
    store_row<T, VW>(R, row, k, c0, k, r);
  }
  block_cols<VW, 1>(arz, m, k, CG, s_red, part, 2 * k, 0);
  block_cols<VW, 1>(arr, m, k, CG, s_red, part, 2 * k, k);
}

__global__ void __launch_bounds__(RED_THREADS) k_red_B(int k, int nblk, const double *part,
                                                       Control *ctl, ColState *cs, double tol,
                                                       int it) {
  if (ctl->stop) return;
  __shared__ double s_sum[192];
  reduce_partials(part, nblk, 2 * k, s_sum);
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    ColState st = cs[c];
    if (st.active) {
      const double rz = s_sum[c], rr = s_sum[k + c];
      st.beta = rz / st.rz;
      st.rz = rz;
      st.rr = rr;
      st.iters += 1;
      if (!(rr > tol * tol * st.bb)) st.active = 0;
    } else {
      st.beta = 0.0;
    }
    cs[c] = st;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int any = 0;
    for (int c = 0; c < k; ++c) any |= cs[c].active;
    if (!any || ctl->breakdown) {
      ctl->stop = 1;
      ctl->skip = it;   // the x/p update of this iteration still runs
    }
  }
}

// C: X += alpha P ; P = D^{-1} R + beta P   (runs in the stopping iteration too)
// The directions alternate between two buffers: iteration it reads p_it from
// Pc and writes p_{it+1} to Pn.  The x update of an even iteration is
// deferred to the next one, which reads p_{it-1} from Pn (before overwriting
// it) and applies both terms in order: one pass over X per two iterations.
// An even iteration that stops the solver applies its own term.
template <typename T, int VW>
__global__ void __launch_bounds__(256) k_pcg_C(int N, int k, int CG, const T *__restrict__ diag,
                                               const T *__restrict__ R, T *__restrict__ X,
                                               const T *__restrict__ Pc, T *__restrict__ Pn,
                                               const Control *ctl, const ColState *cs, int it) {
  if (ctl->stop && ctl->skip != it) return;
  const bool odd = it & 1;
  const bool upd_x = odd || ctl->stop;  // an even iteration updates X only when it is the last
  __shared__ double s_ab[3 * MAX_K];
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    s_ab[c] = cs[c].alpha;
    s_ab[MAX_K + c] = cs[c].beta;
    s_ab[2 * MAX_K + c] = cs[c].alpha_prev;
  }
  __syncthreads();
  const RowMap m = row_map<1>(CG);
  const int rows_per_block = (blockDim.x >> 6) * m.RPW;
  const int c0 = m.cg * VW;
  T al[VW], be[VW], ap[VW];
  for (int v = 0; v < VW; ++v) {
    al[v] = (c0 + v < k) ? (T)s_ab[c0 + v] : T(0);
    be[v] = (c0 + v < k) ? (T)s_ab[MAX_K + c0 + v] : T(0);
    ap[v] = (c0 + v < k) ? (T)s_ab[2 * MAX_K + c0 + v] : T(0);
  }
  const int n_groups = (N + rows_per_block - 1) / rows_per_block;
  for (GroupIter gi = group_iter(n_groups); gi.g < gi.end; gi.g += gi.step) {
    const int row = gi.g * rows_per_block + m.wave * m.RPW + m.slot;
    if (!m.valid || c0 >= k || row >= N) continue;
    T p[VW], r[VW];
    load_row<T, VW>(Pc, row, k, c0, k, p);
    load_row<T, VW>(R, row, k, c0, k, r);
    if (upd_x) {
      T x[VW];
      load_row<T, VW>(X, row, k, c0, k, x);
      if (odd) {
        T q[VW];
        load_row<T, VW>(Pn, row, k, c0, k, q);
        for (int v = 0; v < VW; ++v) x[v] += ap[v] * q[v];
      }
      for (int v = 0; v < VW; ++v) x[v] += al[v] * p[v];
      store_row<T, VW>(X, row, k, c0, k, x);
    }
    const T d = diag[row];
    for (int v = 0; v < VW; ++v) p[v] = r[v] / d + be[v] * p[v];
    store_row<T, VW>(Pn, row, k, c0, k, p);
  }
}

// After the last launched iteration it (even) when the solver did not stop:
// its deferred X += alpha p_it
template <typename T, int VW>
__global__ void __launch_bounds__(256) k_pcg_flush(int N, int k, int CG, T *__restrict__ X,
                                                   const T *__restrict__ Pc, const Control *ctl,
                                                   const ColState *cs) {
  if (ctl->stop) return;
  __shared__ double s_a[MAX_K];
  for (int c = threadIdx.x; c < k; c += blockDim.x) s_a[c] = cs[c].alpha;
  __syncthreads();
  const RowMap m = row_map<1>(CG);
  const int rows_per_block = (blockDim.x >> 6) * m.RPW;
  const int c0 = m.cg * VW;
  T al[VW];
  for (int v = 0; v < VW; ++v) al[v] = (c0 + v < k) ? (T)s_a[c0 + v] : T(0);
  const int n_groups = (N + rows_per_block - 1) / rows_per_block;
  for (GroupIter gi = group_iter(n_groups); gi.g < gi.end; gi.g += gi.step) {
    const int row = gi.g * rows_per_block + m.wave * m.RPW + m.slot;
    if (!m.valid || c0 >= k || row >= N) continue;
    T x[VW], p[VW];
    load_row<T, VW>(X, row, k, c0, k, x);
    load_row<T, VW>(Pc, row, k, c0, k, p);
    for (int v = 0; v < VW; ++v) x[v] += al[v] * p[v];
    store_row<T, VW>(X, row, k, c0, k, x);
  }
}

template <typename T, int VW, int NG>
static int pcg_launch_iters(int N, int k, int CG, int nblkA, int nblkE, const int32_t *rowptr,
                             const int32_t *col, const T *val, const int32_t *ord, const T *diag,
                             T *X, T *R, T *P0, T *P1,
                             T *Q, double *part, Control *ctl, ColState *cs, double tol, int it0,
                             int iters, hipStream_t s, const Tiling *til, const TShape &tsh) {
  for (int it = it0; it < it0 + iters; ++it) {
    T *P = (it & 1) ? P1 : P0, *Pn = (it & 1) ? P0 : P1;
    if (til) {
      if (launch_tpcg_A<T>(N, k, *til, tsh, rowptr, val, P, Q, part, ctl, s) < 0) return -1;
      hipLaunchKernelGGL(k_red_A, dim3(1), dim3(RED_THREADS), 0, s, k, tsh.grid, part, ctl, cs);
    } else {
      hipLaunchKernelGGL((k_pcg_A<T, VW, NG>), dim3(nblkA), dim3(256), 0, s, N, k, CG, rowptr, col, val,
                         P, Q, part, ctl, ord);
      hipLaunchKernelGGL(k_red_A, dim3(1), dim3(RED_THREADS), 0, s, k, nblkA, part, ctl, cs);
    }
    hipLaunchKernelGGL((k_pcg_B<T, VW>), dim3(nblkE), dim3(256), 0, s, N, k, CG, diag, Q, R, part,
                       ctl, cs);
    hipLaunchKernelGGL(k_red_B, dim3(1), dim3(RED_THREADS), 0, s, k, nblkE, part, ctl, cs, tol, it);
    hipLaunchKernelGGL((k_pcg_C<T, VW>), dim3(nblkE), dim3(256), 0, s, N, k, CG, diag, R, X, P, Pn, ctl,
                       cs, it);
  }
  return 0;
}

template <typename T, int VW, int NG>
static int pcg_run(int N, int k, const int32_t *rowptr, const int32_t *col, const T *val,
                   const int32_t *ord, const T *diag, const T *B, T *X, double tol, int max_iter, PCGWork &w,
                   int *iters_out, double *relres_out, int *converged_out, int *breakdown_out,
                   hipStream_t s, int x_zero) {
  const int CG = (k + VW - 1) / VW;
  const int RPWA = 64 / (CG * NG);
  const int RPWE = 64 / CG;
  const int nblkA = std::min(grid_rows(N, RPWA, SPMM_BLOCKS), w.nblk_max);
  const int nblkE = std::min(grid_rows(N, RPWE, pcg_blocks()), w.nblk_max);
  Control *ctl = reinterpret_cast<Control *>(w.state);
  ColState *cs = reinterpret_cast<ColState *>(reinterpret_cast<char *>(w.state) + sizeof(Control));
  T *R = reinterpret_cast<T *>(w.R), *P = reinterpret_cast<T *>(w.P), *Q = reinterpret_cast<T *>(w.Q);
  T *P2 = reinterpret_cast<T *>(w.P2);
  double *part = reinterpret_cast<double *>(w.part);
  TShape tsh;
  const Tiling *til = nullptr;
  if (w.til) {
    tsh = tiled_shape<T>(*w.til, k, N, w.nblk_max, w.til_tb);
    if (tsh.grid > 0) til = w.til;
  }
  int have_r = 0;
  if (x_zero == 2) {
    // R, P, X and the start partials written by launch_refine_prep
    hipLaunchKernelGGL(k_red_init, dim3(1), dim3(RED_THREADS), 0, s, k, w.prep_nblk, part, ctl, cs, tol);
  } else {
    if (x_zero) {
      have_r = 2;  // r = b
    } else if (til) {  // R = B - S X through the halo tiles
      if (launch_tpcg_A_m<T, 2>(N, k, k, k, *til, tsh, rowptr, val, X, R, nullptr, nullptr, B, s) < 0) return -1;
      have_r = 1;
    }
    hipLaunchKernelGGL((k_pcg_init<T, VW, NG>), dim3(nblkA), dim3(256), 0, s, N, k, CG, rowptr, col, val,
                       diag, B, X, R, P, part, ord, have_r);
    hipLaunchKernelGGL(k_red_init, dim3(1), dim3(RED_THREADS), 0, s, k, nblkA, part, ctl, cs, tol);
  }
  std::vector<ColState> hcs(k);
  Control hctl{};
  // host polls of the stop flag: the first after as many iterations as the
  // previous solve took, then every 2 (iterations launched after
  // convergence return at once, but still cost a launch each); without a
  // history, after 4, 8, 16, 32, ... iterations
  // (the first chunk goes out unpolled: a start that already meets the
  // tolerance costs only launches that return at once)
  const bool hist = w.last_iters > 0;
  int done_iters = 0, chunk = hist ? std::max(2, w.last_iters) : 4;
  for (;;) {
    if (done_iters > 0) {
      if (hipMemcpyAsync(&hctl, ctl, sizeof(Control), hipMemcpyDeviceToHost, s) != hipSuccess) return -2;
      if (hipStreamSynchronize(s) != hipSuccess) return -2;
    }
    if (hctl.stop || done_iters >= max_iter) break;
    int n = std::min(chunk, max_iter - done_iters);
    if (pcg_launch_iters<T, VW, NG>(N, k, CG, nblkA, nblkE, rowptr, col, val, ord, diag, X, R, P, P2, Q, part,
                                    ctl, cs, tol, done_iters, n, s, til, tsh) < 0)
      return -1;
    done_iters += n;
    chunk = hist ? 2 : std::min(chunk * 2, 32);
  }
  // iteration limit reached after an even iteration: its deferred x update
  if (!hctl.stop && done_iters > 0 && ((done_iters - 1) & 1) == 0)
    hipLaunchKernelGGL((k_pcg_flush<T, VW>), dim3(nblkE), dim3(256), 0, s, N, k, CG, X, P, ctl, cs);
  if (hipMemcpyAsync(hcs.data(), cs, sizeof(ColState) * k, hipMemcpyDeviceToHost, s) != hipSuccess)
    return -2;
  if (hipStreamSynchronize(s) != hipSuccess) return -2;
  int conv = 1, itmax = 0;
  for (int c = 0; c < k; ++c) itmax = std::max(itmax, hcs[c].iters);
  w.last_iters = itmax;
  for (int c = 0; c < k; ++c) {
    if (iters_out) iters_out[c] = hcs[c].iters;
    if (relres_out) relres_out[c] = hcs[c].bb > 0 ? sqrt(hcs[c].rr / hcs[c].bb) : 0.0;
    if (hcs[c].active) conv = 0;
  }
  if (converged_out) *converged_out = conv;
  if (breakdown_out) *breakdown_out = hctl.breakdown;
  return 0;
}

// Average duration of `reps` back-to-back launches of one PCG phase
// (0 = A: q = S p with p.q, 1 = B: r update, 2 = C: x/p update) in the
// launch configuration pcg_solve uses, on the workspace's current contents.
template <typename T, int VW, int NG>
static int time_phase_t(int N, int k, int phase, const int32_t *rowptr, const int32_t *col,
                        const T *val, const int32_t *ord, const T *diag, T *X, PCGWork &w, int reps, float *ms,
                        hipStream_t s) {
  const int CG = (k + VW - 1) / VW;
  const int RPWA = 64 / (CG * NG);
  const int RPWE = 64 / CG;
  const int nblkA = std::min(grid_rows(N, RPWA, SPMM_BLOCKS), w.nblk_max);
  const int nblkE = std::min(grid_rows(N, RPWE, pcg_blocks()), w.nblk_max);
  Control *ctl = reinterpret_cast<Control *>(w.state);
  ColState *cs = reinterpret_cast<ColState *>(reinterpret_cast<char *>(w.state) + sizeof(Control));
  T *R = reinterpret_cast<T *>(w.R), *P = reinterpret_cast<T *>(w.P), *Q = reinterpret_cast<T *>(w.Q);
  T *P2 = reinterpret_cast<T *>(w.P2);
  double *part = reinterpret_cast<double *>(w.part);
  TShape tsh;
  const Tiling *til = nullptr;
  if (w.til) {
    tsh = tiled_shape<T>(*w.til, k, N, w.nblk_max, w.til_tb);
    if (tsh.grid > 0) til = w.til;
    else return -3;  // this tiling cannot serve k columns of T
  }
  int nc = 0;  // C launches alternate even and odd iterations (the average cost)
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -2;
  if (hipMemsetAsync(ctl, 0, sizeof(Control), s) != hipSuccess) return -2;
  auto launch = [&]() {
    if (phase == 0 && til)
      (void)launch_tpcg_A<T>(N, k, *til, tsh, rowptr, val, P, Q, part, ctl, s);
    else if (phase == 0)
      hipLaunchKernelGGL((k_pcg_A<T, VW, NG>), dim3(nblkA), dim3(256), 0, s, N, k, CG, rowptr, col,
                         val, P, Q, part, ctl, ord);
    else if (phase == 1)
      hipLaunchKernelGGL((k_pcg_B<T, VW>), dim3(nblkE), dim3(256), 0, s, N, k, CG, diag, Q, R, part,
                         ctl, cs);
    else {
      const int it = nc++;
      hipLaunchKernelGGL((k_pcg_C<T, VW>), dim3(nblkE), dim3(256), 0, s, N, k, CG, diag, R, X, (it & 1) ? P2 : P,
                         (it & 1) ? P : P2, ctl, cs, it);
    }
  };
  launch();  // warm
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, s);
  (void)hipEventSynchronize(e1);
  float t = 0.f;
  (void)hipEventElapsedTime(&t, e0, e1);
  *ms = t / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // leave the solver state stopped
  Control stop{1, -1, 0, 0};
  (void)hipMemcpyAsync(ctl, &stop, sizeof(Control), hipMemcpyHostToDevice, s);
  return hipStreamSynchronize(s) == hipSuccess ? 0 : -2;
}



// Vector width: 8 (FP32) / 4 / 2 / 1 values per lane, the widest that divides
// k and fits the pointer alignment.  NG lanes share a row's nonzeros
// (ng <= 0 picks the default: 8 for k = 1, 1 otherwise).
template <typename T>
static int pick_vw(int k, const void *B, const void *X) {
  auto al = [](const void *p, size_t bytes) { return (reinterpret_cast<uintptr_t>(p) % bytes) == 0; };
  if (k == 1) return 1;
  if (sizeof(T) == 4 && k % 8 == 0 && al(B, 32) && al(X, 32)) return 8;
  if (k % 4 == 0 && al(B, 4 * sizeof(T)) && al(X, 4 * sizeof(T))) return 4;
  if (k % 2 == 0 && al(B, 2 * sizeof(T)) && al(X, 2 * sizeof(T))) return 2;
  return 1;
}
static int fit_ng(int k, int vw, int ng) {
  if (ng <= 0) ng = (k == 1) ? 8 : 1;
  const int cg = (k + vw - 1) / vw;
  while (ng > 1 && cg * ng > 64) ng >>= 1;
  return ng;
}

#define KS_PCG_DISPATCH(FN, ...)                                                 \
  switch (vw * 16 + ng) {                                                        \
    case 8 * 16 + 1: return FN<T, (sizeof(T) == 4 ? 8 : 4), 1>(__VA_ARGS__);     \
    case 8 * 16 + 2: return FN<T, (sizeof(T) == 4 ? 8 : 4), 2>(__VA_ARGS__);     \
    case 8 * 16 + 4: return FN<T, (sizeof(T) == 4 ? 8 : 4), 4>(__VA_ARGS__);     \
    case 8 * 16 + 8: return FN<T, (sizeof(T) == 4 ? 8 : 4), 8>(__VA_ARGS__);     \
    case 4 * 16 + 1: return FN<T, 4, 1>(__VA_ARGS__);                             \
    case 4 * 16 + 2: return FN<T, 4, 2>(__VA_ARGS__);                             \
    case 4 * 16 + 4: return FN<T, 4, 4>(__VA_ARGS__);                             \
    case 4 * 16 + 8: return FN<T, 4, 8>(__VA_ARGS__);                             \
    case 2 * 16 + 1: return FN<T, 2, 1>(__VA_ARGS__);                             \
    case 2 * 16 + 2: return FN<T, 2, 2>(__VA_ARGS__);                             \
    case 2 * 16 + 4: return FN<T, 2, 4>(__VA_ARGS__);                             \
    case 2 * 16 + 8: return FN<T, 2, 8>(__VA_ARGS__);                             \
    case 1 * 16 + 2: return FN<T, 1, 2>(__VA_ARGS__);                             \
    case 1 * 16 + 4: return FN<T, 1, 4>(__VA_ARGS__);                             \
    case 1 * 16 + 8: return FN<T, 1, 8>(__VA_ARGS__);                             \
    default: return FN<T, 1, 1>(__VA_ARGS__);                                     \
  }

template <typename T>
int pcg_solve(int N, int k, const int32_t *rowptr, const int32_t *col, const T *val,
              const int32_t *ord, const T *diag, const T *B, T *X, double tol, int max_iter,
              PCGWork &w, int *iters_out, double *relres_out, int *converged_out,
              int *breakdown_out, hipStream_t s, int ng, int x_zero) {
  const int vw = pick_vw<T>(k, B, X);
  ng = fit_ng(k, vw, ng);
  KS_PCG_DISPATCH(pcg_run, N, k, rowptr, col, val, ord, diag, B, X, tol, max_iter, w, iters_out,
                  relres_out, converged_out, breakdown_out, s, x_zero)
}

template int pcg_solve<double>(int, int, const int32_t *, const int32_t *, const double *,
                               const int32_t *, const double *, const double *, double *, double, int,
                               PCGWork &, int *, double *, int *, int *, hipStream_t, int, int);
template int pcg_solve<float>(int, int, const int32_t *, const int32_t *, const float *,
                              const int32_t *, const float *, const float *, float *, double, int,
                              PCGWork &, int *, double *, int *, int *, hipStream_t, int, int);

template <typename T>
int pcg_time_phase(int N, int k, int phase, const int32_t *rowptr, const int32_t *col, const T *val,
                   const int32_t *ord, const T *diag, T *X, PCGWork &w, int reps, float *ms,
                   hipStream_t s, int ng) {
  const int vw = pick_vw<T>(k, w.R, X);
  ng = fit_ng(k, vw, ng);
  KS_PCG_DISPATCH(time_phase_t, N, k, phase, rowptr, col, val, ord, diag, X, w, reps, ms, s)
}
// Autotuner check of the SpMM phase: a fixed input block p, the output of
// the reference kernel kept, and every candidate's output compared with it.
template <typename T>
__global__ void k_fill_pattern(int64_t n, T *__restrict__ p) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = (T)(1.0 + 0.5 * sin(0.37 * (double)(i % 100003)));
}
template <typename T>
__global__ void k_max_dev(int64_t n, const T *__restrict__ q, const T *__restrict__ ref, double *out) {
  __shared__ double sd[256], sr[256];
  double d = 0.0, r = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double a = (double)q[i], b = (double)ref[i];
    d = fmax(d, (a == a) ? fabs(a - b) : INFINITY);  // NaN counts as a mismatch
    r = fmax(r, fabs(b));
  }
  sd[threadIdx.x] = d;
  sr[threadIdx.x] = r;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + o]);
      sr[threadIdx.x] = fmax(sr[threadIdx.x], sr[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = sd[0];
    out[2 * blockIdx.x + 1] = sr[0];
  }
}
template <typename T>
int pcg_phase_check(PCGWork &w, int N, int k, int mode, void *ref, double *dev_host, hipStream_t s) {
  const int64_t n = (int64_t)N * k;
  const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
  if (mode == 0) {
    hipLaunchKernelGGL(k_fill_pattern<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       reinterpret_cast<T *>(w.P));
    return hipGetLastError() == hipSuccess ? 0 : -2;
  }
  if (mode == 1)
    return hipMemcpyAsync(ref, w.Q, sizeof(T) * n, hipMemcpyDeviceToDevice, s) == hipSuccess ? 0 : -2;
  double *part = reinterpret_cast<double *>(w.part);  // at least 2 x 1024 doubles
  hipLaunchKernelGGL(k_max_dev<T>, dim3(g), dim3(256), 0, s, n, reinterpret_cast<const T *>(w.Q),
                     reinterpret_cast<const T *>(ref), part);
  std::vector<double> h(2 * g);
  if (hipMemcpyAsync(h.data(), part, sizeof(double) * 2 * g, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return -2;
  double d = 0.0, r = 0.0;
  for (unsigned b = 0; b < g; ++b) {
    d = std::max(d, h[2 * b]);
    r = std::max(r, h[2 * b + 1]);
  }
  *dev_host = r > 0.0 ? d / r : d;
  return 0;
}
template int pcg_phase_check<double>(PCGWork &, int, int, int, void *, double *, hipStream_t);
template int pcg_phase_check<float>(PCGWork &, int, int, int, void *, double *, hipStream_t);

template int pcg_time_phase<double>(int, int, int, const int32_t *, const int32_t *, const double *,
                                    const int32_t *, const double *, double *, PCGWork &, int, float *,
                                    hipStream_t, int);
template int pcg_time_phase<float>(int, int, int, const int32_t *, const int32_t *, const float *,
                                   const int32_t *, const float *, float *, PCGWork &, int, float *,
                                   hipStream_t, int);

}  // namespace ks
