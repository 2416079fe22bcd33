// HBM streaming probes: the bandwidth that plain, perfectly coalesced
// streams reach on this device, as the practical ceiling next to the nominal
// peak for the memory-bound kernels of the library.  Each thread moves
// 16-byte vectors, UNROLL independent ones in flight, grid-stride over the
// buffer; the grid covers every CU several times.
#include "../../include/ks.h"
#include "common.h"
#include "kernels.h"
#include <algorithm>

namespace ks {

namespace {
constexpr int PR_THREADS = 256;
constexpr int PR_UNROLL = 4;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// kind 0: read (sum per block), 1: copy b = a, 2: triad c = a + s b
template <int KIND, bool NT>
__global__ void __launch_bounds__(PR_THREADS) k_stream(int64_t n4, const f32x4 *__restrict__ a,
                                                       const f32x4 *__restrict__ b, f32x4 *__restrict__ c,
                                                       float s, float *__restrict__ part) {
  const int64_t stride = (int64_t)gridDim.x * PR_THREADS;
  int64_t i = (int64_t)blockIdx.x * PR_THREADS + threadIdx.x;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (; i + (PR_UNROLL - 1) * stride < n4; i += PR_UNROLL * stride) {
    f32x4 x[PR_UNROLL], y[PR_UNROLL];
#pragma unroll
    for (int u = 0; u < PR_UNROLL; ++u) x[u] = NT ? __builtin_nontemporal_load(a + i + u * stride) : a[i + u * stride];
    if constexpr (KIND == 2) {
#pragma unroll
      for (int u = 0; u < PR_UNROLL; ++u)
        y[u] = NT ? __builtin_nontemporal_load(b + i + u * stride) : b[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < PR_UNROLL; ++u) {
      if constexpr (KIND == 0) acc += x[u];
      else {
        const f32x4 v = KIND == 1 ? x[u] : x[u] + s * y[u];
        if (NT) __builtin_nontemporal_store(v, c + i + u * stride);
        else c[i + u * stride] = v;
      }
    }
  }
  for (; i < n4; i += stride) {
    const f32x4 x = a[i];
    if constexpr (KIND == 0) acc += x;
    else c[i] = KIND == 1 ? x : x + s * b[i];
  }
  if constexpr (KIND == 0) {
    __shared__ float sh[PR_THREADS / 64];
    float v = acc.x + acc.y + acc.z + acc.w;
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      float t = 0.f;
      for (int w = 0; w < PR_THREADS / 64; ++w) t += sh[w];
      part[blockIdx.x] = t;
    }
  }
}

template <int KIND>
void launch_stream(int nt, int grid, int64_t n4, const f32x4 *a, const f32x4 *b, f32x4 *c, float *part,
                   hipStream_t s) {
  if (nt) hipLaunchKernelGGL((k_stream<KIND, true>), dim3(grid), dim3(PR_THREADS), 0, s, n4, a, b, c, 1.5f, part);
  else hipLaunchKernelGGL((k_stream<KIND, false>), dim3(grid), dim3(PR_THREADS), 0, s, n4, a, b, c, 1.5f, part);
}
}  // namespace

}  // namespace ks

using namespace ks;

extern "C" int ks_stream_probe(int64_t bytes, int32_t kind, int32_t nontemporal, int32_t reps, double *gbs_host,
                               hipStream_t stream) {
  if (!gbs_host || kind < 0 || kind > 2 || reps < 1 || bytes < (1 << 20) || bytes > ((int64_t)1 << 36))
    return set_error(KS_ERR_ARG, "ks_stream_probe: kind 0..2, reps >= 1, 1 MiB <= bytes <= 64 GiB");
  const int64_t n4 = bytes / 16;
  const int nbuf = kind == 0 ? 1 : (kind == 1 ? 2 : 3);
  f32x4 *buf[3] = {nullptr, nullptr, nullptr};
  float *part = nullptr;
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int grid = std::max(1, ncu) * 16;
  auto cleanup = [&]() {
    for (auto *p : buf)
      if (p) (void)hipFree(p);
    if (part) (void)hipFree(part);
  };
  for (int i = 0; i < nbuf; ++i)
    if (hipMalloc(&buf[i], (size_t)n4 * 16) != hipSuccess) {
      cleanup();
      return set_error(KS_ERR_NOMEM, "ks_stream_probe: hipMalloc failed");
    }
  if (hipMalloc(&part, sizeof(float) * grid) != hipSuccess) {
    cleanup();
    return set_error(KS_ERR_NOMEM, "ks_stream_probe: hipMalloc failed");
  }
  hipError_t e = hipSuccess;
  for (int i = 0; i < nbuf && e == hipSuccess; ++i) e = hipMemsetAsync(buf[i], 0, (size_t)n4 * 16, stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto run = [&]() {
    if (kind == 0) launch_stream<0>(nontemporal, grid, n4, buf[0], nullptr, nullptr, part, stream);
    else if (kind == 1) launch_stream<1>(nontemporal, grid, n4, buf[0], nullptr, buf[1], part, stream);
    else launch_stream<2>(nontemporal, grid, n4, buf[0], buf[1], buf[2], part, stream);
  };
  float ms = 0.f;
  if (e == hipSuccess) {
    run();  // warm-up
    e = hipEventRecord(e0, stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) run();
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  cleanup();
  if (e != hipSuccess) return set_error(KS_ERR_HIP, hipGetErrorString(e));
  const double moved = (double)n4 * 16 * nbuf;  // read + write streams
  *gbs_host = moved * reps / (ms * 1e-3) / 1e9;
  return KS_OK;
}
