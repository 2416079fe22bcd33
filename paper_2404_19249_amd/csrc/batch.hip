// Batched block BVP solves: many independent systems of uneven size
// (each S_s X_s = B_s with k_s columns, Jacobi-PCG per column) in ONE
// persistent launch.
//
// The grid is sized to what the device keeps resident.  Workgroups are
// dealt to systems in teams proportional to each system's work (nnz_s k_s),
// at least one per system; a team owns contiguous row ranges of its system
// and runs the same recurrences as the single-system solver, separated by
// team barriers.  Team reductions are done redundantly by every workgroup
// of the team from per-workgroup partials in a fixed order, so all members
// take identical decisions (convergence, stop) without a broadcast.  Every
// wait is bounded: a barrier that spins past its limit sets the system's
// status to -2 and the workgroup leaves, so the grid always drains.
//
// Memory coherence.  The L2 caches of the eight XCDs are not coherent with
// each other, and an agent-scope acquire/release fence per barrier (an L2
// write-back plus an L2 invalidate for every workgroup) thrashes the caches
// of every team on the XCD.  Instead, the only data one workgroup writes and
// another reads -- the search directions P and the reduction partials --
// are stored and loaded with agent-scope atomic (coherent) accesses, which
// the hardware completes at the device coherence point.  Each wave waits for
// its own accesses to complete before the barrier arrival, and a workgroup
// issues loads of other workgroups' data only after it has observed every
// arrival.  Everything else (the matrix, B, and the R, Q, X rows a
// workgroup owns) uses ordinary cached accesses.
//
// Halo tiles.  A system whose context carries a row-block tiling (blocks of
// BR consecutive storage rows, each with the sorted list of rows its
// nonzeros touch and 16-bit local column indices) runs its products
// through it: the team owns whole blocks, each block's halo rows of P are
// loaded once, coherently, into LDS, and the rows then gather from LDS.
// The coherent traffic per product drops from one load per nonzero and
// column to one per halo row and column.
#include "common.h"
#include "kernels.h"
#include <algorithm>
#include <vector>

namespace ks {

struct BatchSys {
  const int32_t *rowptr, *col;
  const double *val, *diag, *B;
  double *X, *R, *P, *Q;
  double *part;          // shared by all systems: [grid][3 phases][3 MAX_K]
  unsigned int *bar;     // [2]: arrival count since launch start, unused
  int N, k, ng, team0, team, max_iter;
  // halo tiling (tile_br = 0: row products from the CSR arrays)
  int tile_br, tile_nblk;
  const int32_t *halo_ptr, *halo_col, *hself, *pptr;
  const uint16_t *lcol;
  const uint32_t *rmeta;
  double tol;
  int *iters;            // [k]
  double *relres;        // [k]
  unsigned long long *t_done;
  int *status;           // 0 converged, 1 iteration limit, -1 breakdown, -2 barrier timeout
};

constexpr long long SPIN_LIMIT = 1LL << 24;
constexpr int VU = 4;  // rows per lane per round of the vector phases

__device__ __forceinline__ double ld_coh(const double *p) {
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ bool team_barrier(unsigned int *bar, int team, int *status) {
  // bar[0] counts arrivals since the launch started (cleared before each
  // launch); every episode adds exactly `team` arrivals, so the episode a
  // workgroup joins ends when the count reaches the next multiple of team.
  __shared__ int s_ok;
  __builtin_amdgcn_s_waitcnt(0);  // this wave's coherent stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    s_ok = 1;
    const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = (arrived / (unsigned)team + 1u) * (unsigned)team;
    long long spins = 0;
    // relaxed polling: no cache invalidation per poll, one acquire after
    while (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > SPIN_LIMIT) {
        s_ok = 0;
        atomicExch(status, -2);
        break;
      }
    }
  }
  __syncthreads();
  return s_ok != 0;
}

// row product with k columns (one value per lane), NG lanes per row's
// nonzeros; COH: the gathered block is written by other workgroups
template <bool COH>
__device__ __forceinline__ double batch_row(int row, int c, int ng, int NG, const int32_t *rowptr,
                                            const int32_t *col, const double *val, const double *X,
                                            int k) {
  constexpr int U = 8;  // gathers in flight per lane
  double acc = 0.0;
  const int jb = rowptr[row], je = rowptr[row + 1];
  for (int j = jb + ng; j < je; j += U * NG) {
    int ci[U];
    double vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int jj = j + u * NG;
      const bool ok = jj < je;
      const int jc = ok ? jj : j;
      ci[u] = col[jc];
      const double v = val[jc];
      vv[u] = ok ? v : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double *xp = X + (int64_t)ci[u] * k + c;
      acc += vv[u] * (COH ? ld_coh(xp) : *xp);
    }
  }
  return acc;
}

// per-workgroup column sums of `a` (one column per lane group) -> out[c]
__device__ __forceinline__ void wg_cols(double a, bool own, int c, int k, int LPR, int RPW,
                                        double *s_red, double *out) {
  s_red[threadIdx.x] = own ? a : 0.0;
  __syncthreads();
  for (int cc = threadIdx.x; cc < k; cc += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
      for (int sl = 0; sl < RPW; ++sl) s += s_red[w * 64 + sl * LPR + cc * (LPR / k)];
    out[cc] = s;
  }
  __syncthreads();
}

// sum of the team's partials for W <= blockDim values -> s_sum.  The
// workgroup's threads split the members into S = blockDim / W strided
// slices (four loads in flight per thread), then S partial sums per value
// are added in slice order: the order depends only on (team, W, blockDim),
// so every member of the team forms the same sums.  s_tmp: blockDim doubles.
__device__ __forceinline__ void team_sum(const double *part, int team, int W, double *s_tmp,
                                         double *s_sum) {
  const int S = (int)blockDim.x / W, tid = threadIdx.x;
  if (tid < S * W) {
    const int j = tid % W;
    const double *p = part + j;
    const int64_t ps = 9 * MAX_K;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int t = tid / W;
    for (; t + 3 * S < team; t += 4 * S) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] += ld_coh(p + (int64_t)(t + u * S) * ps);
    }
    for (; t < team; t += S) a[0] += ld_coh(p + (int64_t)t * ps);
    s_tmp[tid] = (a[0] + a[1]) + (a[2] + a[3]);
  }
  __syncthreads();
  for (int j = tid; j < W; j += blockDim.x) {
    double v = 0.0;
    for (int q = 0; q < S; ++q) v += s_tmp[q * W + j];
    s_sum[j] = v;
  }
  __syncthreads();
}

// Q = S P on the rows of tile blocks [b0, b1) of system d through LDS
// (s_halo: at least max_halo * k doubles), with this lane's share of the
// p.q partial of column c added to apq
__device__ __forceinline__ void batch_tiled_product(const BatchSys &d, int b0, int b1, int k, int c, int ng,
                                                    int NG, bool valid, int slot, int wave, int RPW,
                                                    double *s_halo, double &apq) {
  const int BR = d.tile_br, rows_per_iter = (blockDim.x >> 6) * RPW;
  for (int blk = b0; blk < b1; ++blk) {
    const int hb = d.halo_ptr[blk], tot = (d.halo_ptr[blk + 1] - hb) * k;
    // eight coherent loads in flight per thread before the LDS writes
    constexpr int SU = 8;
    for (int i0 = threadIdx.x; i0 < tot; i0 += SU * (int)blockDim.x) {
      double v[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int i = i0 + u * (int)blockDim.x;
        const int h = i / k, cc = i - h * k;
        v[u] = i < tot ? ld_coh(d.P + (int64_t)d.halo_col[hb + (i < tot ? h : 0)] * k + cc) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int i = i0 + u * (int)blockDim.x;
        if (i < tot) s_halo[i] = v[u];
      }
    }
    __syncthreads();
    const int rb = blk * BR, nr = min(BR, d.N - rb);
    const int nz0 = d.rowptr[rb], p0 = d.pptr[blk], hs = d.hself[blk];
    for (int sb = 0; sb < nr; sb += rows_per_iter) {
      const int sl = sb + wave * RPW + slot;
      const bool rv = valid && sl < nr;
      double acc = 0.0;
      int rr = 0;
      if (rv) {
        const uint32_t m0 = d.rmeta[2 * (int64_t)(rb + sl)], m1 = d.rmeta[2 * (int64_t)(rb + sl) + 1];
        const int len = (int)((m0 >> 16) & 0xffu);
        rr = (int)(m0 >> 24);
        const double *v = d.val + nz0 + (m0 & 0xffffu);
        const uint16_t *lc = d.lcol + p0 + m1;
        double a1 = 0.0;
        int j = ng;
        for (; j + NG < len; j += 2 * NG) {
          acc += v[j] * s_halo[(int)lc[j] * k + c];
          a1 += v[j + NG] * s_halo[(int)lc[j + NG] * k + c];
        }
        if (j < len) acc += v[j] * s_halo[(int)lc[j] * k + c];
        acc += a1;
      }
      for (int off = 1; off < NG; off <<= 1) acc += __shfl_xor(acc, off, 64);
      if (rv && ng == 0) {
        d.Q[(int64_t)(rb + rr) * k + c] = acc;
        apq += s_halo[(hs + rr) * k + c] * acc;
      }
    }
    __syncthreads();  // the next block's halo overwrites s_halo
  }
}

__global__ void __launch_bounds__(256) k_batch_pcg(const BatchSys *__restrict__ systems,
                                                   const int *__restrict__ wg_sys) {
  extern __shared__ double s_halo[];
  __shared__ double s_red[256];
  __shared__ double s_sum[3 * MAX_K];
  __shared__ double s_part[3 * MAX_K];
  __shared__ double s_rz[MAX_K], s_bb[MAX_K], s_alpha[MAX_K], s_beta[MAX_K], s_rr[MAX_K];
  __shared__ int s_active[MAX_K], s_iters[MAX_K];
  __shared__ int s_flags[2];  // any active, breakdown
  const int sidx = wg_sys[blockIdx.x];
  if (sidx < 0) return;
  const BatchSys &d = systems[sidx];
  const int rank = blockIdx.x - d.team0, team = d.team, k = d.k, NG = d.ng;
  const int LPR = k * NG, RPW = 64 / LPR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot = lane / LPR, rem = lane % LPR, c = rem / NG, ng = rem % NG;
  const bool valid = slot < RPW;
  const int rows_per_iter = (blockDim.x >> 6) * RPW;
  // contiguous row range of this workgroup (whole tile blocks when tiled)
  int r0, r1, b0 = 0, b1 = 0;
  if (d.tile_br > 0) {
    const int per = (d.tile_nblk + team - 1) / team;
    b0 = min(d.tile_nblk, rank * per);
    b1 = min(d.tile_nblk, b0 + per);
    r0 = min(d.N, b0 * d.tile_br);
    r1 = min(d.N, b1 * d.tile_br);
  } else {
    const int chunk = (d.N + team - 1) / team;
    r0 = min(d.N, rank * chunk);
    r1 = min(d.N, r0 + chunk);
  }
  // partials of team member t (global workgroup team0 + t), phase ph
  const int W3 = 3 * k;
  constexpr int PS = 9 * MAX_K;
  double *partI = d.part + (int64_t)d.team0 * PS, *partA = partI + 3 * MAX_K, *partB = partI + 6 * MAX_K;

  // ---- init: R = B - S X, P = D^{-1} R; b.b, r.r, r.z
  double abb = 0.0, arr = 0.0, arz = 0.0;
  for (int base = r0; base < r1; base += rows_per_iter) {
    const int row = base + wave * RPW + slot;
    const bool rv = valid && row < r1;
    double acc = rv ? batch_row<false>(row, c, ng, NG, d.rowptr, d.col, d.val, d.X, k) : 0.0;
    for (int off = 1; off < NG; off <<= 1) acc += __shfl_xor(acc, off, 64);
    if (rv && ng == 0) {
      const int64_t ix = (int64_t)row * k + c;
      const double b = d.B[ix], r = b - acc, p = r / d.diag[row];
      d.R[ix] = r;
      st_coh(d.P + ix, p);
      abb += b * b;
      arr += r * r;
      arz += r * p;
    }
  }
  const bool own = valid && ng == 0;
  wg_cols(abb, own, c, k, LPR, RPW, s_red, s_part);
  wg_cols(arr, own, c, k, LPR, RPW, s_red, s_part + k);
  wg_cols(arz, own, c, k, LPR, RPW, s_red, s_part + 2 * k);
  for (int i = threadIdx.x; i < W3; i += blockDim.x) st_coh(partI + (int64_t)rank * PS + i, s_part[i]);
  if (!team_barrier(d.bar, team, d.status)) return;
  team_sum(partI, team, W3, s_red, s_sum);
  for (int cc = threadIdx.x; cc < k; cc += blockDim.x) {
    s_bb[cc] = s_sum[cc];
    s_rr[cc] = s_sum[k + cc];
    s_rz[cc] = s_sum[2 * k + cc];
    s_active[cc] = (s_bb[cc] > 0.0) && (s_rr[cc] > d.tol * d.tol * s_bb[cc]);
    s_iters[cc] = 0;
    s_alpha[cc] = s_beta[cc] = 0.0;
  }
  if (threadIdx.x == 0) s_flags[1] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    int any = 0;
    for (int cc = 0; cc < k; ++cc) any |= s_active[cc];
    s_flags[0] = any;
  }
  __syncthreads();

  int it = 0;
  for (; it < d.max_iter && s_flags[0] && !s_flags[1]; ++it) {
    // ---- A: Q = S P, p.q
    double apq = 0.0;
    if (d.tile_br > 0)
      batch_tiled_product(d, b0, b1, k, c, ng, NG, valid, slot, wave, RPW, s_halo, apq);
    else
    for (int base = r0; base < r1; base += rows_per_iter) {
      const int row = base + wave * RPW + slot;
      const bool rv = valid && row < r1;
      double acc = rv ? batch_row<true>(row, c, ng, NG, d.rowptr, d.col, d.val, d.P, k) : 0.0;
      for (int off = 1; off < NG; off <<= 1) acc += __shfl_xor(acc, off, 64);
      if (rv && ng == 0) {
        const int64_t ix = (int64_t)row * k + c;
        d.Q[ix] = acc;
        apq += ld_coh(d.P + ix) * acc;
      }
    }
    wg_cols(apq, own, c, k, LPR, RPW, s_red, s_part);
    for (int i = threadIdx.x; i < k; i += blockDim.x) st_coh(partA + (int64_t)rank * PS + i, s_part[i]);
    if (!team_barrier(d.bar, team, d.status)) return;
    team_sum(partA, team, k, s_red, s_sum);
    for (int cc = threadIdx.x; cc < k; cc += blockDim.x) {
      const double pq = s_sum[cc];
      s_alpha[cc] = 0.0;
      if (s_active[cc]) {
        if (!(pq > 0.0)) s_flags[1] = 1;
        else s_alpha[cc] = s_rz[cc] / pq;
      }
    }
    __syncthreads();
    // ---- B: R -= alpha Q ; r.z, r.r
    double brz = 0.0, brr = 0.0;
    // VU rows per lane per round, their loads issued together
    for (int base = r0; base < r1; base += VU * rows_per_iter) {
      double rv[VU], qv[VU], dv[VU];
#pragma unroll
      for (int u = 0; u < VU; ++u) {
        const int row = base + u * rows_per_iter + wave * RPW + slot;
        const bool ok = valid && row < r1 && ng == 0;
        const int64_t ix = (int64_t)(ok ? row : 0) * k + (ok ? c : 0);
        rv[u] = ok ? d.R[ix] : 0.0;
        qv[u] = ok ? d.Q[ix] : 0.0;
        dv[u] = ok ? d.diag[row] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < VU; ++u) {
        const int row = base + u * rows_per_iter + wave * RPW + slot;
        if (!(valid && row < r1 && ng == 0)) continue;
        const double r = rv[u] - s_alpha[c] * qv[u];
        d.R[(int64_t)row * k + c] = r;
        brr += r * r;
        brz += r * (r / dv[u]);
      }
    }
    wg_cols(brz, own, c, k, LPR, RPW, s_red, s_part);
    wg_cols(brr, own, c, k, LPR, RPW, s_red, s_part + k);
    for (int i = threadIdx.x; i < 2 * k; i += blockDim.x) st_coh(partB + (int64_t)rank * PS + i, s_part[i]);
    if (!team_barrier(d.bar, team, d.status)) return;
    team_sum(partB, team, 2 * k, s_red, s_sum);
    for (int cc = threadIdx.x; cc < k; cc += blockDim.x) {
      const double rz = s_sum[cc], rr = s_sum[k + cc];
      if (s_active[cc]) {
        s_beta[cc] = rz / s_rz[cc];
        s_rz[cc] = rz;
        s_rr[cc] = rr;
        s_iters[cc] += 1;
        if (!(rr > d.tol * d.tol * s_bb[cc])) s_active[cc] = 0;
      } else {
        s_beta[cc] = 0.0;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int any = 0;
      for (int cc = 0; cc < k; ++cc) any |= s_active[cc];
      s_flags[0] = any;
    }
    __syncthreads();
    // ---- C: X += alpha P ; P = D^{-1} R + beta P
    for (int base = r0; base < r1; base += VU * rows_per_iter) {
      double pv[VU], xv[VU], rv[VU], dv[VU];
#pragma unroll
      for (int u = 0; u < VU; ++u) {
        const int row = base + u * rows_per_iter + wave * RPW + slot;
        const bool ok = valid && row < r1 && ng == 0;
        const int64_t ix = (int64_t)(ok ? row : 0) * k + (ok ? c : 0);
        pv[u] = ok ? ld_coh(d.P + ix) : 0.0;
        xv[u] = ok ? d.X[ix] : 0.0;
        rv[u] = ok ? d.R[ix] : 0.0;
        dv[u] = ok ? d.diag[row] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < VU; ++u) {
        const int row = base + u * rows_per_iter + wave * RPW + slot;
        if (!(valid && row < r1 && ng == 0)) continue;
        const int64_t ix = (int64_t)row * k + c;
        d.X[ix] = xv[u] + s_alpha[c] * pv[u];
        st_coh(d.P + ix, rv[u] / dv[u] + s_beta[c] * pv[u]);
      }
    }
    if (s_flags[0] && !s_flags[1])
      if (!team_barrier(d.bar, team, d.status)) return;
  }
  if (rank == 0 && threadIdx.x == 0) {
    for (int cc = 0; cc < k; ++cc) {
      d.iters[cc] = s_iters[cc];
      d.relres[cc] = s_bb[cc] > 0.0 ? sqrt(s_rr[cc] / s_bb[cc]) : 0.0;
    }
    int st = 0;
    if (s_flags[1]) st = -1;
    else if (s_flags[0]) st = 1;
    if (atomicCAS(d.status, 0, st) != 0) { /* keep an earlier barrier timeout */ }
    *d.t_done = wall_clock64();
  }
}

// start of a launch: clears status and arrival counters and stamps the
// device clock
__global__ void k_batch_reset(BatchSys *systems, int n, unsigned long long *t0) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    *systems[i].status = 0;
    systems[i].bar[0] = 0u;
  }
  if (threadIdx.x == 0) *t0 = wall_clock64();
}
void launch_batch_reset(void *systems, int n, unsigned long long *t0, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(256), 0, s, reinterpret_cast<BatchSys *>(systems), n, t0);
}
void launch_batch_pcg(int grid, const void *systems, const int *wg_sys, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_pcg, dim3(grid), dim3(256), lds, s,
                     reinterpret_cast<const BatchSys *>(systems), wg_sys);
}
size_t batch_sys_bytes() { return sizeof(BatchSys); }
size_t batch_part_stride() { return 9 * MAX_K; }
int batch_resident_grid() {
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_batch_pcg, 256, 0) != hipSuccess)
    return -1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  return per_cu * cus;
}
// Largest dynamic LDS (bytes, multiple of 1 KiB, at most 64 KiB) with which
// a grid of `grid` workgroups stays resident; -1 if the query fails.
int64_t batch_lds_budget(int grid) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return -1;
  const int need = (grid + cus - 1) / cus;  // workgroups per CU
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void *)k_batch_pcg, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024) !=
        hipSuccess)
      return -1;
    attr_set = true;
  }
  for (int64_t lds = 64 * 1024; lds > 0; lds -= 1024) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_batch_pcg, 256, (size_t)lds) !=
        hipSuccess)
      return -1;
    if (per_cu >= need) return lds;
  }
  return 0;
}

// Host-side description of one system (filled by the runtime), packed into
// the device table by pack_batch.
void pack_batch_sys(void *dst, const int32_t *rowptr, const int32_t *col, const double *val,
                    const double *diag, const double *B, double *X, double *R, double *P, double *Q,
                    double *part, unsigned int *bar, int N, int k, int ng, int team0, int team,
                    int max_iter, double tol, int *iters, double *relres,
                    unsigned long long *t_done, int *status, const Tiling *til) {
  BatchSys s;
  s.tile_br = til ? til->BR : 0;
  s.tile_nblk = til ? til->nblk : 0;
  s.halo_ptr = til ? til->halo_ptr : nullptr;
  s.halo_col = til ? til->halo_col : nullptr;
  s.hself = til ? til->hself : nullptr;
  s.pptr = til ? til->pptr : nullptr;
  s.lcol = til ? til->lcol : nullptr;
  s.rmeta = til ? til->rmeta : nullptr;
  s.rowptr = rowptr; s.col = col; s.val = val; s.diag = diag; s.B = B;
  s.X = X; s.R = R; s.P = P; s.Q = Q; s.part = part; s.bar = bar;
  s.N = N; s.k = k; s.ng = ng; s.team0 = team0; s.team = team; s.max_iter = max_iter;
  s.tol = tol; s.iters = iters; s.relres = relres; s.t_done = t_done; s.status = status;
  *reinterpret_cast<BatchSys *>(dst) = s;
}

}  // namespace ks
