// dp_force_error_noalloc: the audit's force-error reduction without any
// device allocation, for callers that cannot allocate (code under HIP graph
// capture, tight serving loops).
//
// dp_force_error allocates a buffer for the per-block partial sums of its
// reduction on every call and copies them to the host.  This variant keeps
// the partial sums in a fixed file-scope device array, reduces them on the
// device in the same fixed order as dp_force_error does on the host, and
// writes (RMSE, max) to a caller-owned device buffer, asynchronously on the
// caller's stream.
//
// The array is 256 (sum of squares, max) pairs, 4 KiB per device: the
// reduction's grid is capped at 256 blocks for every n, so every accepted n
// fits.  Each device holds its own copy until the process ends; its address
// is looked up once per device with hipGetSymbolAddress and only that
// address is handed to kernels.  Every block of the first kernel writes its
// pair before the second kernel reads them, so nothing needs clearing
// between calls.  Calls that overlap on one device (two streams, two host
// threads) share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dpa1.h"
#include "dpa1_model.h"
#include "dpa1_train.h"
#include "train_internal.h"

namespace {

constexpr int kMaxParts = 256;
static __device__ __align__(256) double scratch[2 * kMaxParts];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices];  // device address of scratch, per device

// (RMSE, max) from the partial pairs, summed in block order in FP64 as
// dp_force_error does on the host.
__global__ void k_force_error_finish(const double *__restrict__ part, int nb, int n,
                                     double *__restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double sq = 0.0, mx = 0.0;
  for (int b = 0; b < nb; ++b) {
    sq += part[2 * b];
    mx = fmax(mx, part[2 * b + 1]);
  }
  out[0] = sqrt(sq / (3.0 * (double)n));
  out[1] = mx;
}

__global__ void k_zero2(double *out) {
  if (threadIdx.x < 2) out[threadIdx.x] = 0.0;
}

// Address of this device's scratch array, looked up on the first call on the
// device (with that device current).
int scratch_address(double **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return dpa1::fail(DP_ERR_DEVICE, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch[dev] = (double *)p;
  }
  *out = g_scratch[dev];
  return DP_OK;
}

}  // namespace

extern "C" int dp_force_error_noalloc(const double *d_a, const double *d_b, int n,
                                      double *d_rmse_max, void *hip_stream) {
  if (!d_rmse_max || n < 0 || (n > 0 && (!d_a || !d_b)))
    return dpa1::fail(DP_ERR_ARG, "bad arguments");
  if (n > DP_FORCE_ERROR_MAX_ATOMS)
    return dpa1::fail(DP_ERR_ARG, "n = %d exceeds DP_FORCE_ERROR_MAX_ATOMS (%d)", n,
                      DP_FORCE_ERROR_MAX_ATOMS);
  hipStream_t s = (hipStream_t)hip_stream;
  if (n == 0) {
    hipLaunchKernelGGL(k_zero2, dim3(1), dim3(64), 0, s, d_rmse_max);
    HIP_TRY(hipGetLastError());
    return DP_OK;
  }
  const int nb = dpa1::force_error_blocks(n);
  if (nb > kMaxParts)
    return dpa1::fail(DP_ERR_ARG, "reduction needs %d partial sums, scratch holds %d", nb,
                      kMaxParts);
  double *part = nullptr;
  int rc = scratch_address(&part);
  if (rc) return rc;
  dpa1::launch_force_error(d_a, d_b, n, part, s);
  hipLaunchKernelGGL(k_force_error_finish, dim3(1), dim3(64), 0, s, part, nb, n, d_rmse_max);
  HIP_TRY(hipGetLastError());
  return DP_OK;
}
