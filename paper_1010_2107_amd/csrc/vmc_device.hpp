// vmc_device.hpp -- device primitives of the sample-and-accumulate pass
// (steps 2-4 of the six-step structure of Kanzaki, arXiv:1010.2107,
// Sec. 3.1) for gfx950: counter-based random words, exact bin index,
// LDS-resident grid table, and block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vmc {

constexpr int kBlock = 256;  // 4 wave64 per block
constexpr int kWave = 64;
constexpr int kMaxGrad = 17;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products and xors; the key advances by the Weyl increments between
// rounds.  The key words are kernel arguments, so the key schedule lives in
// scalar registers; the products map onto v_mad_u64_u32.
// ---------------------------------------------------------------------------
struct Key {
  uint32_t k0, k1;
};

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96); c may be a scalar.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Rounds 2-10 of Philox4x32-10 given the first round's products.
__device__ __forceinline__ void philox10_from_round1(uint32_t hi0, uint32_t lo0, uint32_t hi1, uint32_t lo1,
                                                     uint32_t c1, uint32_t c3, Key key, uint32_t (&out)[4]) {
  uint32_t k0 = key.k0, k1 = key.k1;
  uint32_t c0 = hi1 ^ c1 ^ k0;
  uint32_t c2 = hi0 ^ c3 ^ k1;
  c1 = lo1;
  c3 = lo0;
#pragma unroll
  for (int r = 1; r < 10; ++r) {
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t x0 = xor3(static_cast<uint32_t>(pb >> 32), c1, k0);
    const uint32_t x2 = xor3(static_cast<uint32_t>(pa >> 32), c3, k1);
    c1 = static_cast<uint32_t>(pb);
    c3 = static_cast<uint32_t>(pa);
    c0 = x0;
    c2 = x2;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// NW words of the block sequence with counter (c0, g | tag, c2, c3),
// g = 0, 1, ...: word i is word i%4 of block g = i/4.  The first round
// multiplies only c0 and c2, which all blocks share, so its products are
// formed once.
template <int NW>
__device__ __forceinline__ void philox_words(uint32_t c0, uint32_t tag, uint32_t c2, uint32_t c3, Key key,
                                             uint32_t (&w)[NW]) {
  const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
  const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
  const uint32_t hi0 = static_cast<uint32_t>(pa >> 32), lo0 = static_cast<uint32_t>(pa);
  const uint32_t hi1 = static_cast<uint32_t>(pb >> 32), lo1 = static_cast<uint32_t>(pb);
#pragma unroll
  for (int g = 0; g < (NW + 3) / 4; ++g) {
    uint32_t blk[4];
    philox10_from_round1(hi0, lo0, hi1, lo1, static_cast<uint32_t>(g) | tag, c3, key, blk);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (4 * g + q < NW) w[4 * g + q] = blk[q];
  }
}

// The D words of sample s of iteration it (stream tag 0).
template <int D>
__device__ __forceinline__ void sample_words(uint32_t s, uint32_t it, uint32_t kid, Key key,
                                             uint32_t (&w)[D]) {
  philox_words<D>(s, 0u, it, kid, key, w);
}

// ---------------------------------------------------------------------------
// Bin index.  The uniform is u = (2m+1) 2^-24 with m the top 23 bits of the
// word.  With y N = (2m+1) N 2^-24 the bin is its integer part and the
// in-bin offset its fraction, both exact in 32-bit integer arithmetic for
// N <= 256.  Stratified: y = (c + u)/ng, so y N = (c 2^24 + 2m+1) N /
// (ng 2^24); when ng divides N this is c (N/ng) + (2m+1)(N/ng) 2^-24.
// The helpers return the offset scaled by 2^32 (a 24-bit integer times 2^8,
// exact in FP32), to be multiplied by a width stored times kWidthScale.
// ---------------------------------------------------------------------------
// Division of 32-bit words by a launch-constant divisor d >= 2 through a
// precomputed multiplier (Granlund and Montgomery, "Division by invariant
// integers using multiplication", PLDI 1994, Sec. 4): with l = ceil(log2 d)
// and m = floor(2^32 (2^l - d) / d) + 1, t = mulhi(m, n) gives
// n / d = (t + ((n - t) >> 1)) >> (l - 1) exactly for every 32-bit n.
// m = 1 exactly when d is a power of two.
struct DivU32 {
  uint32_t d, m, sh;  // divisor, multiplier, l - 1
};
inline DivU32 make_divu32(uint32_t d) {  // d >= 2
  uint32_t l = 0;
  while ((uint64_t{1} << l) < d) ++l;
  const uint64_t m = ((uint64_t{1} << 32) * ((uint64_t{1} << l) - d)) / d + 1;
  return DivU32{d, static_cast<uint32_t>(m), l - 1};
}

__device__ __forceinline__ uint32_t divu32(uint32_t n, const DivU32& v) {
  const uint32_t t = __umulhi(n, v.m);
  return (t + ((n - t) >> 1)) >> v.sh;
}

// The D base-d digits of c (least significant first).  The branch on the
// divisor's form is uniform across the launch.
template <int D>
__device__ __forceinline__ void digits(uint32_t c, const DivU32& v, uint32_t (&cc)[D]) {
  if (v.m == 1) {
    const uint32_t mask = v.d - 1, l = v.sh + 1;
#pragma unroll
    for (int a = 0; a < D; ++a) cc[a] = (c >> (l * a)) & mask;
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const uint32_t q = divu32(c, v);
      cc[a] = c - q * v.d;
      c = q;
    }
  }
}

// (2m+1) N 2^8 as m (N 2^9) + N 2^8, one 32 x 32 + 64-bit multiply-add
// (m < 2^23, N <= 256, the result below 2^40): its high word is the integer
// part of (2m+1) N 2^-24, its low word the 24-bit fraction shifted up by 8.
__device__ __forceinline__ uint64_t odd_times(uint32_t word, uint32_t n) {
  return static_cast<uint64_t>(word >> 9) * (n << 9) + (n << 8);
}

template <typename T>
__device__ __forceinline__ void bin_plain(uint32_t word, uint32_t nbins, int& j, T& off) {
  const uint64_t P = odd_times(word, nbins);
  j = static_cast<int>(P >> 32);
  off = static_cast<T>(static_cast<uint32_t>(P));
}

template <typename T>
__device__ __forceinline__ void bin_strat_div(uint32_t word, uint32_t ca, uint32_t per_cube, int& j, T& off) {
  // ng divides nbins; per_cube = nbins / ng
  const uint64_t P = odd_times(word, per_cube);
  j = static_cast<int>(__umul24(ca, per_cube) + static_cast<uint32_t>(P >> 32));
  off = static_cast<T>(static_cast<uint32_t>(P));
}

// ng does not divide nbins: the point lies at (ca + (2m+1) 2^-24) / ng on
// the axis, and Q = (ca 2^24 + 2m + 1) N is that position times N ng 2^24.
// The bin is floor(Q / (ng 2^24)) = floor(floor(Q / 2^24) / ng), where
// floor(Q / 2^24) < ng N fits 32 bits when ng N < 2^32, and the offset, in
// units of 2^-32 of the bin, is 2^8 (Q mod ng 2^24) / ng, formed from its
// two parts with the reciprocal of ng (the factors 2^8 and 2^32 are exact,
// so the result is 2^8 times the offset in units of 2^-24, bit for bit).
template <typename T>
__device__ __forceinline__ void bin_strat_gen(uint32_t word, uint32_t ca, const DivU32& ng, uint32_t nbins,
                                              T inv_ng, int& j, T& off) {
  const uint64_t Q = ((static_cast<uint64_t>(ca) << 24) + ((word >> 9) * 2u + 1u)) * nbins;
  const uint32_t hi = static_cast<uint32_t>(Q >> 24);
  const uint32_t q = divu32(hi, ng);
  j = static_cast<int>(q);
  const T rhi = static_cast<T>(hi - q * ng.d);                     // < ng
  const T rlo = static_cast<T>(static_cast<uint32_t>(Q) << 8);  // (Q mod 2^24) 2^8
  off = fma(rhi, inv_ng * static_cast<T>(4294967296.0), rlo * inv_ng);
}

// The same map when ng N >= 2^32 (one axis cut into more than 2^32 / N
// cubes): a 64-bit division and an FP64 quotient for the offset.
template <typename T>
__device__ __forceinline__ void bin_strat_wide(uint32_t word, uint32_t ca, uint32_t ng, uint32_t nbins, int& j,
                                               T& off) {
  const uint64_t Q = ((static_cast<uint64_t>(ca) << 24) + ((word >> 9) * 2u + 1u)) * nbins;
  const uint64_t Dn = static_cast<uint64_t>(ng) << 24;
  const uint64_t q = Q / Dn;
  j = static_cast<int>(q);
  off = static_cast<T>(static_cast<double>(Q - q * Dn) * 256.0 / static_cast<double>(ng));
}

// A grid's table holds per bin the lower edge and the width times
// kWidthScale = 2^-32, so that a sample's point is fma(off, width', edge) with
// the offset `off` of the bin helpers: the same value as edge + (off 2^-32)
// width, since both scalings are exact, one multiply fewer per axis.
constexpr double kWidthScale = 0x1p-32;

// Grid table entry: lower edge and scaled width of a bin.
template <typename T>
struct TabEntry;
template <>
struct TabEntry<float> {
  using type = float2;
};
template <>
struct TabEntry<double> {
  using type = double2;
};

// ---------------------------------------------------------------------------
// math overloads
// ---------------------------------------------------------------------------
// FP32 reciprocal: the hardware estimate (1 ulp) instead of an IEEE divide
// sequence; FP64 keeps the correctly rounded division.
__device__ __forceinline__ float vrcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double vrcp(double x) { return 1.0 / x; }
// Hardware exp2/log2 in FP32, the accurate library functions in FP64.  The
// FP32 forms scale the argument by log2 e (or the result by ln 2), so the
// relative error of exp is about |x| 1e-7 on top of the instruction's own
// ulp: the same order as the rounding of an FP32 argument of that size.
__device__ __forceinline__ float vexp_fast(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ double vexp_fast(double x) { return exp(x); }
__device__ __forceinline__ float vlog_fast(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }
__device__ __forceinline__ double vlog_fast(double x) { return log(x); }
__device__ __forceinline__ float vlog2_fast(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double vlog2_fast(double x) { return log2(x); }
__device__ __forceinline__ float vexp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double vexp2_fast(double x) { return exp2(x); }
// sin and cos of 2 pi x for x in [0, 1): the hardware takes its argument in
// revolutions (absolute error ~1e-7 in FP32).
__device__ __forceinline__ void vsincos2pi(float x, float& s, float& c) {
  s = __builtin_amdgcn_sinf(x);
  c = __builtin_amdgcn_cosf(x);
}
__device__ __forceinline__ void vsincos2pi(double x, double& s, double& c) { sincospi(2.0 * x, &s, &c); }
// e^x - 1 in FP32: for |x| < 0.35 the Taylor series to x^8 / 8! (truncation
// below 1e-9 relative), otherwise exp2(x log2 e) - 1, where e^x - 1 is at
// least 0.29 in magnitude so the subtraction loses under two bits; max
// relative error about 3e-7.  FP64 keeps the library function.
__device__ __forceinline__ float vexpm1_fast(float x) {
  float p = 1.0f / 40320.0f;
  p = fmaf(p, x, 1.0f / 5040.0f);
  p = fmaf(p, x, 1.0f / 720.0f);
  p = fmaf(p, x, 1.0f / 120.0f);
  p = fmaf(p, x, 1.0f / 24.0f);
  p = fmaf(p, x, 1.0f / 6.0f);
  p = fmaf(p, x, 0.5f);
  p = fmaf(p, x * x, x);
  const float e = __builtin_amdgcn_exp2f(x * 1.4426950408889634f) - 1.0f;
  return fabsf(x) < 0.35f ? p : e;
}
__device__ __forceinline__ double vexpm1_fast(double x) { return expm1(x); }
__device__ __forceinline__ float vlog(float x) { return logf(x); }
__device__ __forceinline__ double vlog(double x) { return log(x); }
__device__ __forceinline__ float vsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double vsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float vrsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double vrsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ bool vfinite(float x) { return isfinite(x); }
__device__ __forceinline__ bool vfinite(double x) { return isfinite(x); }

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// LDS maximum of a positive double: non-negative doubles order like their
// bit patterns read as unsigned 64-bit integers.  The slot starts at +0.
__device__ __forceinline__ void lds_max_pos(double* p, double v) {
  __hip_atomic_fetch_max(reinterpret_cast<unsigned long long*>(p),
                         static_cast<unsigned long long>(__double_as_longlong(v)), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void global_add(double* p, double v) { unsafeAtomicAdd(p, v); }

// Sum NV per-thread values over the block and add the totals to dst[idx[i]]
// with one global atomic each.  `red` is LDS scratch of 4*NV doubles.
template <int NV>
__device__ __forceinline__ void block_sum_to_global(const double (&v)[NV], double* red, double* dst,
                                                    const int (&idx)[NV]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double t = wave_sum(v[i]);
    if (lane == 0) red[wave * NV + i] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kBlock / kWave; ++w) t += red[w * NV + i];
      if (t != 0.0) global_add(dst + idx[i], t);
    }
  }
  __syncthreads();
}

}  // namespace vmc
