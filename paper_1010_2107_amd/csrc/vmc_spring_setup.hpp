// vmc_spring_setup.hpp -- the set-up of SPRING event generation from the
// per-cube maxima of the BASES integration phase (Kanzaki, arXiv:1010.2107,
// Sec. 3.1): the largest cube maximum, the integer envelope q_c, its
// running sums P (an exact 64-bit scan) and the guide table of the cube
// search.  The trial kernel is in vmc_spring.hpp.
#pragma once

#include "vmc_spring.hpp"

namespace vmc {
namespace {

constexpr int kScanItems = 8;                        // cubes per thread in the scan
constexpr uint64_t kScanChunk = kBlock * kScanItems;  // cubes per scan block

// Envelope quanta of a cube: ceil(wmax/gmax 2^20) for a positive maximum.
__device__ __forceinline__ uint64_t quanta(double v, double gmax) {
  return (v > 0.0 && v <= gmax) ? static_cast<uint64_t>(ceil((v / gmax) * kSpringQuanta)) : 0ull;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Inclusive scan over the lanes of a wave.
__device__ __forceinline__ uint64_t wave_scan_u64(uint64_t v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint64_t o = __shfl_up(v, off, kWave);
    if (lane >= off) v += o;
  }
  return v;
}

// Exclusive scan of one value per thread over the block; *total gets the sum.
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* lds, uint64_t* total) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint64_t inc = wave_scan_u64(v);
  if (lane == kWave - 1) lds[wave] = inc;
  __syncthreads();
  uint64_t before = 0, all = 0;
  for (int w = 0; w < kBlock / kWave; ++w) {
    if (w < wave) before += lds[w];
    all += lds[w];
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

__global__ void k_sp_init(uint64_t* st, uint64_t M, uint32_t kbits) {
  for (int i = threadIdx.x; i < SP_HDR; i += blockDim.x) st[i] = 0ull;
  __syncthreads();
  if (threadIdx.x == 0) {
    st[SP_KBITS] = kbits;
    st[SP_NCUBES] = M;
  }
}

// Largest positive finite maximum: the bit patterns of positive doubles are
// ordered as unsigned integers, so an integer atomic max finds it.  NaN,
// zero and negative maxima are ignored; +Inf maxima are counted.
__global__ __launch_bounds__(kBlock) void k_sp_gmax(const double* wmax, uint64_t M, uint64_t* st) {
  double m = 0.0;
  uint64_t bad = 0;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < M;
       i += static_cast<uint64_t>(gridDim.x) * kBlock) {
    const double v = wmax[i];
    if (isinf(v) && v > 0.0)
      ++bad;
    else if (v > m)
      m = v;
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, kWave));
  bad = wave_sum_u64(bad);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (m > 0.0)
      atomicMax(reinterpret_cast<unsigned long long*>(st + SP_GMAX),
                static_cast<unsigned long long>(__double_as_longlong(m)));
    if (bad) atomicAdd(reinterpret_cast<unsigned long long*>(st + SP_BADMAX), static_cast<unsigned long long>(bad));
  }
}

// Sum of q over scan block b's cubes -> st[SP_HDR + b].
__global__ __launch_bounds__(kBlock) void k_sp_blocksum(const double* wmax, uint64_t M, uint64_t* st) {
  __shared__ uint64_t lds[kBlock / kWave];
  const double gmax = __longlong_as_double(static_cast<long long>(st[SP_GMAX]));
  const uint64_t c0 = static_cast<uint64_t>(blockIdx.x) * kScanChunk + static_cast<uint64_t>(threadIdx.x) * kScanItems;
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (c0 + i < M) s += quanta(wmax[c0 + i], gmax);
  uint64_t total;
  (void)block_exclusive_scan(s, lds, &total);
  if (threadIdx.x == 0) st[SP_HDR + blockIdx.x] = total;
}

// Exclusive scan of the nblk block sums in place (one block), then the
// header: T, one quantum (headroom x gmax / 2^20), the envelope integral.
__global__ __launch_bounds__(kBlock) void k_sp_scan_blocks(uint64_t* st, uint64_t nblk, double headroom) {
  __shared__ uint64_t lds[kBlock / kWave];
  uint64_t carry = 0;
  for (uint64_t base = 0; base < nblk; base += kBlock) {
    const uint64_t i = base + threadIdx.x;
    const uint64_t v = i < nblk ? st[SP_HDR + i] : 0ull;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(v, lds, &total);
    if (i < nblk) st[SP_HDR + i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    const double gmax = __longlong_as_double(static_cast<long long>(st[SP_GMAX]));
    const double unit = gmax / kSpringQuanta * headroom;
    st[SP_TOTAL] = carry;
    st[SP_UNIT] = static_cast<uint64_t>(__double_as_longlong(unit));
    st[SP_ENV] = static_cast<uint64_t>(
        __double_as_longlong(static_cast<double>(carry) * unit / static_cast<double>(st[SP_NCUBES])));
  }
}

// Running sums P[c] (c <= M) from the scanned block offsets.
__global__ __launch_bounds__(kBlock) void k_sp_scan(const double* wmax, uint64_t M, const uint64_t* st,
                                                    uint64_t* prefix) {
  __shared__ uint64_t lds[kBlock / kWave];
  const double gmax = __longlong_as_double(static_cast<long long>(st[SP_GMAX]));
  const uint64_t c0 = static_cast<uint64_t>(blockIdx.x) * kScanChunk + static_cast<uint64_t>(threadIdx.x) * kScanItems;
  uint64_t q[kScanItems], s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    q[i] = (c0 + i < M) ? quanta(wmax[c0 + i], gmax) : 0ull;
    s += q[i];
  }
  uint64_t total;
  uint64_t run = st[SP_HDR + blockIdx.x] + block_exclusive_scan(s, lds, &total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (c0 + i < M) prefix[c0 + i] = run;
    run += q[i];
    if (c0 + i + 1 == M) prefix[M] = run;
  }
}

// guide[b] = cube of the smallest r64 of bucket b (b < K), guide[K] = cube
// of r = T - 1: the last c with P[c] <= r.
__global__ __launch_bounds__(kBlock) void k_sp_guide(const uint64_t* prefix, uint64_t M, const uint64_t* st,
                                                     uint32_t* guide) {
  const uint32_t kbits = static_cast<uint32_t>(st[SP_KBITS]);
  const uint64_t K = 1ull << kbits, T = st[SP_TOTAL];
  for (uint64_t b = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; b <= K;
       b += static_cast<uint64_t>(gridDim.x) * kBlock) {
    uint64_t r;
    if (b == K)
      r = T - 1;
    else
      r = __umul64hi(kbits ? (b << (64 - kbits)) : 0ull, T);
    uint64_t lo = 0, hi = M - 1;
    while (lo < hi) {
      const uint64_t mid = (lo + hi + 1) >> 1;
      if (prefix[mid] <= r)
        lo = mid;
      else
        hi = mid - 1;
    }
    guide[b] = static_cast<uint32_t>(lo);
  }
}

__global__ void k_sp_clear_counts(uint64_t* st) {
  if (threadIdx.x == 0) st[SP_TRIALS] = st[SP_KEPT] = st[SP_OVER] = st[SP_SLOT] = 0ull;
}

}  // namespace
}  // namespace vmc
