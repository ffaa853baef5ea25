// vmc_probe.hip -- calibration kernels for the two rates that bound the
// sample pass: the LDS FP64 atomic add (the per-bin histogram, 2 dim adds
// per sample) and the FP32 fused multiply-add of the vector ALU (the
// integrand).  Each lane runs 8 independent chains per loop trip, so each
// rate is set by its own pipeline alone.
#include <hip/hip_runtime.h>

#include "vmc.h"
#include "vmc_device.hpp"
#include "vmc_error.hpp"

namespace vmc {
// Written only if a probe's sum hits its sentinel (never).  External
// linkage, so the compiler must keep the store and the work that feeds it.
__device__ double probe_sink;
}  // namespace vmc

namespace {

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
  if (t == -1.0) vmc::probe_sink = t;  // keeps the adds alive; the sum is positive
}

// a, b and sentinel are arguments so that the compiler cannot bound the sum
// and drop the chains; the host passes a = 0.9999, b = 1e-4, sentinel = -1.
__global__ __launch_bounds__(vmc::kBlock) void k_probe_fma(int iters, float a, float b, float sentinel) {
  float f[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) f[i] = 1.0f + 1e-3f * static_cast<float>(threadIdx.x + i);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = fmaf(f[i], a, b);
  }
  float t = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) t += f[i];
  if (t == sentinel) vmc::probe_sink = t;  // keeps the chains alive; the sum is positive
}

// Duration (ms) of one launch after a short warm-up launch, on `st`.
template <class Launch>
int timed(hipStream_t st, Launch launch, const char* what, float* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return vmc::set_error(VMC_E_HIP, "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return vmc::set_error(VMC_E_HIP, "hipEventCreate");
  }
  int rc = VMC_OK;
  launch(16);  // warm-up
  hipEventRecord(e0, st);
  launch(0);
  hipEventRecord(e1, st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  if (e != hipSuccess) rc = vmc::set_error(VMC_E_HIP, "%s probe: %s", what, hipGetErrorString(e));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}

int check_args(int blocks, int iters, const double* rate) {
  if (!rate) return vmc::set_error(VMC_E_INVALID, "rate is NULL");
  if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20))
    return vmc::set_error(VMC_E_INVALID, "blocks %d / iters %d outside [1, 2^20]", blocks, iters);
  return VMC_OK;
}

}  // namespace

extern "C" int vmc_probe_lds_atomics(int blocks, int iters, double* rate, void* stream) {
  if (int rc = check_args(blocks, iters, rate)) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float ms = 0.f;
  const int rc = timed(
      st,
      [&](int warm) {
        hipLaunchKernelGGL(k_probe_lds_add, dim3(blocks), dim3(vmc::kBlock), 0, st, warm ? warm : iters);
      },
      "LDS", &ms);
  if (rc == VMC_OK) *rate = static_cast<double>(blocks) * vmc::kBlock * 8.0 * iters / (ms * 1e-3);
  return rc;
}

extern "C" int vmc_probe_fp32_fma(int blocks, int iters, double* flops, void* stream) {
  if (int rc = check_args(blocks, iters, flops)) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float ms = 0.f;
  const int rc = timed(
      st,
      [&](int warm) {
        hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(vmc::kBlock), 0, st, warm ? warm : iters, 0.9999f,
                           1e-4f, -1.0f);
      },
      "FMA", &ms);
  if (rc == VMC_OK) *flops = static_cast<double>(blocks) * vmc::kBlock * 8.0 * 2.0 * iters / (ms * 1e-3);
  return rc;
}
