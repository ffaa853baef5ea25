// vmc_small.hpp -- the FP64 kernels around the sample pass: clearing the
// accumulators, the per-iteration estimate and the running combination of
// iterations, grid refinement (step 5 of the six-step structure of
// Kanzaki, arXiv:1010.2107, Sec. 3.1) and the FP32 table build.
#pragma once

#include "vmc_kernels.hpp"

namespace vmc {
// internal linkage: every unit that launches these kernels gets its own copy
namespace {

__global__ __launch_bounds__(kBlock) void k_clear(double* bins, int nbins_total, double* scal, int s_lo,
                                                  int s_hi) {
  const int tid = blockIdx.x * kBlock + threadIdx.x;
  const int stride = gridDim.x * kBlock;
  for (int i = tid; i < nbins_total; i += stride) bins[i] = 0.0;
  for (int i = s_lo + tid; i < s_hi; i += stride) scal[i] = 0.0;
}

// Estimate of one iteration and its variance,
//   plain:      I = S1/n, var = (S2/n - I^2)/(n-1)
//   stratified: I = S1/(kM), var = sum_c (k S2_c - S1_c^2)/(k^2 (k-1) M^2),
// then the running combination with weights 1/var, updated with West's
// weighted incremental mean so that chi^2 needs no stored history.
// Iterations with var = 0 are exact; when any exist the combined value is
// their mean with zero error.
__device__ void finalize_one(double* scal, int strat, double n, double kd, double Md, int fwd, int ngrad) {
  const double denom = kd * kd * (kd - 1.0) * Md * Md;
  if (fwd) {
    const double I = scal[S_S1] / n;
    const double var = strat ? scal[S_V] / denom : (scal[S_S2] / n - I * I) / (n - 1.0);
    scal[S_I] = I;
    scal[S_VAR] = var;
    scal[S_NEFF] = n;
    scal[S_NTOTAL] += n;
    scal[S_NITER] += 1.0;
    if (var == 0.0) {
      scal[S_NEXACT] += 1.0;
      scal[S_SUMEXACT] += I;
    } else {
      const double w = 1.0 / var;
      const double W = scal[S_W] + w;
      const double delta = I - scal[S_MEAN];
      const double mean = scal[S_MEAN] + delta * (w / W);
      scal[S_M2] += w * delta * (I - mean);
      scal[S_MEAN] = mean;
      scal[S_W] = W;
    }
    if (scal[S_NEXACT] > 0.0) {
      scal[S_IBAR] = scal[S_SUMEXACT] / scal[S_NEXACT];
      scal[S_SIGBAR] = 0.0;
      scal[S_CHI2] = 0.0;
    } else {
      scal[S_IBAR] = scal[S_MEAN];
      scal[S_SIGBAR] = 1.0 / sqrt(scal[S_W]);
      scal[S_CHI2] = scal[S_NITER] > 1.0 ? scal[S_M2] / (scal[S_NITER] - 1.0) : __builtin_nan("");
    }
  }
  for (int q = 0; q < ngrad; ++q) {
    double* g = scal + S_GRAD + 5 * q;
    const double G = g[0] / n;
    g[3] = G;
    g[4] = strat ? g[2] / denom : (g[1] / n - G * G) / (n - 1.0);
  }
}

__global__ void k_finalize(double* scal, int strat, double n, double kd, double Md, int fwd, int ngrad) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  finalize_one(scal, strat, n, kd, Md, fwd, ngrad);
}

__global__ void k_combine_reset(double* scal) {
  const int i = threadIdx.x;
  if (i >= S_W && i <= S_NTOTAL) scal[i] = 0.0;
}

// Uniform grid, its table, and cleared accumulators.
__global__ __launch_bounds__(kBlock) void k_reset(double* edges, float* table, double* bins, double* scal,
                                                  int d, int N) {
  const int tid = blockIdx.x * kBlock + threadIdx.x;
  const int stride = gridDim.x * kBlock;
  for (int i = tid; i < d * (N + 1); i += stride) {
    const int j = i % (N + 1);
    edges[i] = static_cast<double>(j) / static_cast<double>(N);
  }
  for (int i = tid; i < d * N; i += stride) {
    const int j = i % N;
    const double lo = static_cast<double>(j) / static_cast<double>(N);
    const double hi = static_cast<double>(j + 1) / static_cast<double>(N);
    table[2 * i] = static_cast<float>(lo);
    table[2 * i + 1] = static_cast<float>(hi - lo);
  }
  for (int i = tid; i < 2 * d * N; i += stride) bins[i] = 0.0;
  for (int i = tid; i < S_LEN; i += stride) scal[i] = 0.0;
}

// FP32 (lower edge, width) per bin, both rounded from FP64 values (the
// width is differenced in FP64 first so narrow bins keep their precision).
__global__ __launch_bounds__(kBlock) void k_table(const double* edges, float* table, int d, int N) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= d * N) return;
  const int a = i / N, j = i - a * N;
  const double* e = edges + static_cast<size_t>(a) * (N + 1);
  table[2 * i] = static_cast<float>(e[j]);
  table[2 * i + 1] = static_cast<float>(e[j + 1] - e[j]);
}

// Refinement of one axis per block (N <= 256 bins, one thread per bin):
//  d_j = sum of w^2 in bin j; smoothed with its neighbours (3-point mean,
//  2-point at the ends); rho_j = dbar_j / sum dbar; damped weight
//  r_j = ((1-rho_j)/(-ln rho_j))^alpha (0 at rho = 0, 1 at rho = 1); the new
//  edges cut the piecewise-uniform density r_j/width_j into N pieces of
//  equal weight.  An axis with zero (or non-finite) smoothed sum is kept.
// The two short sums run in order on one thread; everything else is one
// thread per bin / per new edge.
// ea: the axis' N+1 edges; ta: its N (lo, width) table entries; b2: its N
// plane-1 bin sums.  Called by a whole block.
__device__ void refine_axis(double* ea, float* ta, const double* b2, int N, double alpha) {
  __shared__ double e[257], r[256], C[257], en[257];
  __shared__ double Dsum, Tshare;
  __shared__ int keep;
  const int t = threadIdx.x;
  for (int i = t; i <= N; i += kBlock) e[i] = ea[i];
  for (int i = t; i < N; i += kBlock) C[i] = b2[i];
  __syncthreads();
  for (int i = t; i < N; i += kBlock) {
    double sm;
    if (i == 0)
      sm = (C[0] + C[1]) / 2.0;
    else if (i == N - 1)
      sm = (C[N - 2] + C[N - 1]) / 2.0;
    else
      sm = (C[i - 1] + C[i] + C[i + 1]) / 3.0;
    r[i] = sm;
  }
  __syncthreads();
  if (t == 0) {
    double D = 0.0;
    for (int i = 0; i < N; ++i) D += r[i];
    Dsum = D;
    keep = !(D > 0.0) || !isfinite(D);
  }
  __syncthreads();
  if (keep) return;
  for (int i = t; i < N; i += kBlock) {
    const double rho = r[i] / Dsum;
    double base;
    if (rho <= 0.0)
      base = 0.0;
    else if (rho >= 1.0)
      base = 1.0;
    else
      base = (1.0 - rho) / (-log(rho));
    r[i] = pow(base, alpha);
  }
  __syncthreads();
  if (t == 0) {
    C[0] = 0.0;
    for (int i = 0; i < N; ++i) C[i + 1] = C[i] + r[i];
    Tshare = C[N] / N;
  }
  __syncthreads();
  const double T = Tshare;
  for (int k = t; k <= N; k += kBlock) {
    if (k == 0 || k == N) {
      en[k] = e[k];
      continue;
    }
    const double target = k * T;
    int lo = 0, hi = N - 1;  // smallest j with C[j+1] > target, else N-1
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (C[mid + 1] > target)
        hi = mid;
      else
        lo = mid + 1;
    }
    en[k] = e[lo] + ((target - C[lo]) / r[lo]) * (e[lo + 1] - e[lo]);
  }
  __syncthreads();
  for (int k = t; k <= N; k += kBlock) ea[k] = en[k];
  for (int j = t; j < N; j += kBlock) {
    ta[2 * j] = static_cast<float>(en[j]);
    ta[2 * j + 1] = static_cast<float>(en[j + 1] - en[j]);
  }
}

__global__ __launch_bounds__(kBlock) void k_refine(double* edges, float* table, const double* bins, int d,
                                                   int N, double alpha) {
  const int a = blockIdx.x;
  refine_axis(edges + static_cast<size_t>(a) * (N + 1), table + static_cast<size_t>(2) * a * N,
              bins + static_cast<size_t>(d + a) * N, N, alpha);
}

}  // namespace
}  // namespace vmc
