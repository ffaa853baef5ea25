// vmc_probe.hip -- calibration of the LDS FP64 atomic-add rate that bounds
// the per-bin histogram of the sample pass (2 dim LDS atomics per sample).
// Every lane adds into its own LDS double, 8 independent adds per loop
// trip, so the rate is set by the LDS atomic pipeline alone.
#include <hip/hip_runtime.h>

#include "vmc.h"
#include "vmc_device.hpp"
#include "vmc_error.hpp"

namespace {

__device__ double g_probe_sink;  // written only if a sum came out -1 (never)

__global__ __launch_bounds__(vmc::kBlock) void k_probe_lds_add(int iters) {
  __shared__ double s[8 * vmc::kBlock];
  for (int i = 0; i < 8; ++i) s[i * vmc::kBlock + threadIdx.x] = 0.0;
  __syncthreads();
  const double v = 1.0 + 1e-3 * threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) vmc::lds_add(&s[i * vmc::kBlock + threadIdx.x], v);
  }
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < 8; ++i) t += s[i * vmc::kBlock + threadIdx.x];
  if (t == -1.0) g_probe_sink = t;  // keeps the adds alive; the sum is positive
}

}  // namespace

extern "C" int vmc_probe_lds_atomics(int blocks, int iters, double* rate, void* stream) {
  if (!rate) return vmc::set_error(VMC_E_INVALID, "rate is NULL");
  if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20))
    return vmc::set_error(VMC_E_INVALID, "blocks %d / iters %d outside [1, 2^20]", blocks, iters);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return vmc::set_error(VMC_E_HIP, "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return vmc::set_error(VMC_E_HIP, "hipEventCreate");
  }
  int rc = VMC_OK;
  hipLaunchKernelGGL(k_probe_lds_add, dim3(blocks), dim3(vmc::kBlock), 0, st, 16);  // warm-up
  hipEventRecord(e0, st);
  hipLaunchKernelGGL(k_probe_lds_add, dim3(blocks), dim3(vmc::kBlock), 0, st, iters);
  hipEventRecord(e1, st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e != hipSuccess)
    rc = vmc::set_error(VMC_E_HIP, "LDS probe: %s", hipGetErrorString(e));
  else
    *rate = static_cast<double>(blocks) * vmc::kBlock * 8.0 * iters / (ms * 1e-3);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}
