// Small generalised eigensolve (eq. st1) for callers that cannot allocate
// device memory: the same two-stage packed Jacobi kernels as ks_small_eig,
// with every work buffer carved out of one fixed device array per GPU
// instead of a context's workspace.
#include "../../include/ks.h"
#include "common.h"
#include "kernels.h"

#include <mutex>
#include <string>

using namespace ks;

namespace {
constexpr int NA_MAX_M = 190;                        // the packed eigensolver's limit
constexpr size_t NA_SCRATCH_DOUBLES = (size_t)19 << 17;  // 19 MiB
constexpr int NA_MAX_DEVICES = 64;
}  // namespace

// One copy per GPU, alive until the process ends.  Host code never passes
// this name to a kernel: it uses the device address from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[NA_SCRATCH_DOUBLES];

namespace {
std::mutex g_mu;
double *g_scratch[NA_MAX_DEVICES] = {};

__global__ void k_zero_ints(int n, int *p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

size_t up32(size_t n) { return (n + 31) & ~(size_t)31; }

// Device address of the current GPU's scratch array, looked up once per
// device with that device current.
int scratch_address(double **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(KS_ERR_HIP, "hipGetDevice failed");
  if (dev < 0 || dev >= NA_MAX_DEVICES) return set_error(KS_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(KS_ERR_HIP, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
    g_scratch[dev] = static_cast<double *>(p);
  }
  *out = g_scratch[dev];
  return KS_OK;
}
}  // namespace

extern "C" int ks_small_eig_noalloc(const double *FA, const double *FB, int32_t m, int32_t k, double *U,
                                    double *lambda_host, int32_t *rank_host, hipStream_t stream) {
  if (!FA || !FB || !U || !lambda_host) return set_error(KS_ERR_ARG, "null argument");
  if (m < 1 || m > NA_MAX_M || k < 1 || k > m)
    return set_error(KS_ERR_ARG, "need 1 <= k <= m <= 190");
  double *base = nullptr;
  if (int r = scratch_address(&base); r != KS_OK) return r;
  // layout: D, lam, theta [m]; V, X, W, S, T1, T2 [m][m]; the rotation log;
  // 8 status ints
  const size_t mm = (size_t)m * m;
  double *D = base;
  double *lam = D + up32(m);
  double *theta = lam + up32(m);
  double *V = theta + up32(m);
  double *X = V + up32(mm);
  double *W = X + up32(mm);
  double *S = W + up32(mm);
  double *T1 = S + up32(mm);
  double *T2 = T1 + up32(mm);
  double *work = T2 + up32(mm);
  int *info = reinterpret_cast<int *>(work + up32(jacobi_work_doubles(m)));
  if ((size_t)((reinterpret_cast<double *>(info) + 4) - base) > NA_SCRATCH_DOUBLES)
    return set_error(KS_ERR_ARG, "scratch too small for this m");
  hipStream_t s = stream;
  // the array keeps the previous call's contents: clear the status words
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, s, 8, info);
  if (launch_orth(m, FB, m, D, V, X, work, info, s) < 0)
    return set_error(KS_ERR_HIP, "cannot enable the LDS size of the eigensolver");
  int h[8];
  hipError_t e = hipMemcpyAsync(h, info, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(KS_ERR_HIP, hipGetErrorString(e));
  if (h[2]) return set_error(KS_ERR_EIG, "F_B has a non-positive diagonal entry");
  const int r = h[0];
  if (r < k) return set_error(KS_ERR_EIG, ("pencil has rank " + std::to_string(r) + " < k").c_str());
  if (launch_reduced_eig_split(m, k, r, FA, m, D, X, W, 0, S, T1, T2, work, lam, theta, U, info + 4, s) < 0)
    return set_error(KS_ERR_HIP, "cannot enable the LDS size of the eigensolver");
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(lambda_host, theta, sizeof(double) * k, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(KS_ERR_HIP, hipGetErrorString(e));
  if (rank_host) *rank_host = r;
  return KS_OK;
}
