// vmc_small.hpp -- the FP64 kernels around the sample pass: clearing the
// accumulators, resetting the combination of iterations, grid refinement
// (step 5 of the six-step structure of Kanzaki, arXiv:1010.2107, Sec. 3.1)
// and the FP32 table build.
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

// Publish a sample launch: add up the kStripes copies of the partial sums
// (and clear them), write the bin sums (forward passes), the scalar sums,
// the estimate and the running combination.
// Thread i of the grid owns bin i; block 0 also owns the scalar slots.
__global__ __launch_bounds__(kBlock) void k_publish(double* bins, double* stripes, int stripe_len, int nb,
                                                    double* scal, int fwd, int strat, int ngrad, double n, double kd,
                                                    double Md) {
  __shared__ double tot[kStripeScal];
  // all kStripes loads of a slot are issued before any store
  auto gather = [&](int slot) {
    double c[kStripes];
#pragma unroll
    for (int s = 0; s < kStripes; ++s) c[s] = stripes[static_cast<size_t>(s) * stripe_len + slot];
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < kStripes; ++s) {
      v += c[s];
      stripes[static_cast<size_t>(s) * stripe_len + slot] = 0.0;
    }
    return v;
  };
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < nb) {
    const double v = gather(i);
    if (fwd) bins[i] = v;
  }
  if (blockIdx.x != 0) return;
  if (threadIdx.x < kStripeScal) tot[threadIdx.x] = gather(nb + threadIdx.x);
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (fwd) {
    scal[S_S1] = tot[T_S1];
    scal[S_S2] = tot[T_S2];
    scal[S_NONFIN] = tot[T_NONFIN];
    scal[S_NZERO] = tot[T_NZERO];
    scal[S_V] = tot[T_V];
  }
  for (int q = 0; q < ngrad; ++q) {
    scal[S_GRAD + 5 * q + 0] = tot[T_G + q];
    scal[S_GRAD + 5 * q + 1] = tot[T_G + ngrad + q];
    scal[S_GRAD + 5 * q + 2] = tot[T_G + 2 * ngrad + q];
  }
  finalize_one(scal, strat, n, kd, Md, fwd, ngrad);
}

__global__ void k_combine_reset(double* scal) {
  const int i = threadIdx.x;
  if (i >= S_W && i <= S_NTOTAL) scal[i] = 0.0;
}

// Uniform grid, its table, and cleared accumulators.
__global__ __launch_bounds__(kBlock) void k_reset(double* edges, float* table, double* bins, int nbins_total,
                                                  double* scal, int d, int N) {
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
    table[2 * i + 1] = static_cast<float>((hi - lo) * kWidthScale);
  }
  for (int i = tid; i < nbins_total; i += stride) bins[i] = 0.0;
  for (int i = tid; i < S_LEN; i += stride) scal[i] = 0.0;
}

// FP32 (lower edge, width x kWidthScale) per bin, both rounded from FP64
// values (the width is differenced in FP64 first so narrow bins keep their
// precision).
__global__ __launch_bounds__(kBlock) void k_table(const double* edges, float* table, int d, int N) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= d * N) return;
  const int a = i / N, j = i - a * N;
  const double* e = edges + static_cast<size_t>(a) * (N + 1);
  table[2 * i] = static_cast<float>(e[j]);
  table[2 * i + 1] = static_cast<float>((e[j + 1] - e[j]) * kWidthScale);
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
    ta[2 * j + 1] = static_cast<float>((en[j + 1] - en[j]) * kWidthScale);
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
