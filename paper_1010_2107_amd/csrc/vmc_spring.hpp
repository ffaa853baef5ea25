// vmc_spring.hpp -- SPRING: unweighted events from the result of the BASES
// integration phase (Kanzaki, arXiv:1010.2107, Sec. 3.1; Kawabata, CPC 41
// (1986) 127).
//
// The integration phase records the largest weight w = f J of every cube.
// The envelope is constant on a cube and held as an integer number q_c of
// quanta (q_c = ceil(wmax_c / gmax 2^20), one quantum = h gmax / 2^20 with
// a headroom h >= 1 over the recorded maxima), so that the running sums
// P_c = q_0 + ... + q_{c-1} and the choice of a cube are exact integer
// arithmetic.  A trial draws a 64-bit integer r64, takes
// r = floor(r64 T / 2^64) (T = P_M) and the cube c with P_c <= r < P_{c+1},
// places a point uniformly in the cube's y-range, maps it through the
// frozen grid and keeps it when u g_c < w (g_c = q_c quanta).  Kept points
// are distributed as f(x) dx wherever w <= g_c; a trial with w > g_c is kept
// and counted as an overflow.
//
// The cube search starts from a guide table: with K = 2^kbits >= M buckets
// of r64 (bucket b = r64 >> (64 - kbits)), guide[b] is the cube of the
// smallest r64 of bucket b, so the cube of any r64 in bucket b lies in
// [guide[b], guide[b+1]] and the binary search over P usually has nothing
// left to do.
#pragma once

#include "vmc_kernels.hpp"

namespace vmc {

// SPRING state: 8-byte slots; doubles at SP_UNIT, SP_GMAX, SP_ENV, unsigned
// 64-bit integers elsewhere.  Slots from SP_HDR on are scratch for the
// set-up's scan (one per scan block).
enum : int {
  SP_UNIT = 0,     // envelope value of one quantum, headroom x gmax / 2^20
  SP_GMAX = 1,     // largest cube maximum
  SP_TOTAL = 2,    // T = sum of q_c
  SP_ENV = 3,      // envelope integral T unit / M (the acceptance is about I / this)
  SP_KBITS = 4,    // guide buckets K = 2^kbits
  SP_NCUBES = 5,   // M
  SP_BADMAX = 6,   // cubes whose maximum is +Inf (set-up fails)
  SP_TRIALS = 8,   // trials run
  SP_KEPT = 9,     // trials kept (stored or not)
  SP_OVER = 10,    // kept trials whose weight exceeded the envelope
  SP_SLOT = 11,    // next event slot (events beyond the buffer are not stored)
  SP_HDR = 16
};

constexpr uint32_t kSpringTag = 2u << 8;  // counter word 1 = word group | tag
constexpr double kSpringQuanta = 1048576.0;

struct SpringArgs {
  SampleArgs A;  // grid table and edges, theta, key, it = pass, ng, per_cube, M, nbins
  const uint64_t* prefix;  // [M+1] running sums of q
  const uint32_t* guide;   // [K+1]
  uint64_t* state;
  uint64_t trial0, ntrials, max_events;
  void* events;            // [max_events][D] points x, float or double as the integrand
  uint64_t* event_trial;   // [max_events] trial number of each stored event, or NULL
};

// Kept events are staged in LDS and written out kStage at a time: one
// atomic reserves a block's run of consecutive slots, and the copy to the
// event buffer is contiguous.
constexpr int kStage = 512;

template <class F>
__global__ __launch_bounds__(kBlock) void k_spring(const SpringArgs P) {
  using T = typename F::T;
  constexpr int D = F::D;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[(kBlock / kWave) * 2];
  __shared__ uint64_t s_trial[kStage];
  __shared__ unsigned int s_n;
  __shared__ unsigned long long s_base;
  const SampleArgs& A = P.A;
  typename TabEntry<T>::type* tab;
  (void)setup_lds<F, 0>(A, smem, tab);
  // staged points after the grid table
  T* s_x = reinterpret_cast<T*>(smem + sizeof(typename TabEntry<T>::type) * D * A.nbins);
  const F fn = block_setup<F>(A.theta);
  if (threadIdx.x == 0) s_n = 0u;

  const uint64_t total = P.state[SP_TOTAL];
  const double unit = __longlong_as_double(static_cast<long long>(P.state[SP_UNIT]));
  const uint32_t kbits = static_cast<uint32_t>(P.state[SP_KBITS]);
  const uint32_t last = A.M - 1;
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long* slot_ctr = reinterpret_cast<unsigned long long*>(P.state + SP_SLOT);
  double n_kept = 0.0, n_over = 0.0;

  // copy the staged events out (whole block; s_n is block-uniform here)
  auto flush = [&]() {
    const unsigned int n = s_n;
    if (threadIdx.x == 0) s_base = atomicAdd(slot_ctr, static_cast<unsigned long long>(n));
    __syncthreads();
    const uint64_t base = s_base;
    const uint64_t room = base < P.max_events ? P.max_events - base : 0;
    const uint64_t m = min(static_cast<uint64_t>(n), room);
    T* ev = static_cast<T*>(P.events) + base * D;
    for (uint64_t k = threadIdx.x; k < m * D; k += kBlock) ev[k] = s_x[k];
    if (P.event_trial)
      for (uint64_t k = threadIdx.x; k < m; k += kBlock) P.event_trial[base + k] = s_trial[k];
    __syncthreads();
    if (threadIdx.x == 0) s_n = 0u;
    __syncthreads();
  };

  __syncthreads();
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kBlock;
  for (uint64_t base_i = static_cast<uint64_t>(blockIdx.x) * kBlock; base_i < P.ntrials; base_i += stride) {
    const uint64_t i = base_i + threadIdx.x;
    bool keep = false;
    T x[D];
    uint64_t t = 0;
    if (i < P.ntrials) {
      t = P.trial0 + i;
      // words 0..D-1: the point in the cube; D, D+1: the cube choice (low
      // and high half of r64); D+2: the acceptance uniform
      uint32_t w[D + 3];
      philox_words<D + 3>(static_cast<uint32_t>(t), kSpringTag, A.it, static_cast<uint32_t>(t >> 32), A.key, w);
      const uint64_t r64 = (static_cast<uint64_t>(w[D + 1]) << 32) | w[D];
      const uint64_t r = __umul64hi(r64, total);
      const uint64_t b = kbits ? (r64 >> (64 - kbits)) : 0;
      uint32_t lo = min(P.guide[b], last), hi = min(P.guide[b + 1], last);
      while (lo < hi) {  // last c in [lo, hi] with P_c <= r
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (P.prefix[mid] <= r)
          lo = mid;
        else
          hi = mid - 1;
      }
      const uint32_t c = lo;
      const double g = static_cast<double>(P.prefix[c + 1] - P.prefix[c]) * unit;
      uint32_t cc[D], wp[D];
      digits<D>(c, A.ngdiv, cc);
#pragma unroll
      for (int a = 0; a < D; ++a) wp[a] = w[a];
      int j[D];
      T jac;
      make_point<T, D, true>(A, tab, wp, cc, j, x, jac);
      T gr[F::NGRAD + 1];
      const T fv = fn.template eval<false>(x, gr);
      const double wd = static_cast<double>(fv * jac);
      const double u = static_cast<double>(((w[D + 2] >> 9) << 1) | 1u) * 5.9604644775390625e-08;
      keep = u * g < wd;
      n_kept += keep ? 1.0 : 0.0;
      n_over += (wd > g) ? 1.0 : 0.0;
    }
    // stage: one LDS atomic per wave, kept lanes take consecutive entries
    // (at most kBlock new entries: the stage was flushed below kStage - kBlock)
    const uint64_t mask = __ballot(keep);
    if (keep) {
      const int leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
      unsigned int wbase = 0;
      if (lane == leader) wbase = atomicAdd(&s_n, static_cast<unsigned int>(__popcll(mask)));
      wbase = __shfl(wbase, leader, kWave);
      const unsigned int e = wbase + static_cast<unsigned int>(__popcll(mask & __lanemask_lt()));
#pragma unroll
      for (int a = 0; a < D; ++a) s_x[e * D + a] = x[a];
      s_trial[e] = t;
    }
    __syncthreads();
    const unsigned int staged = s_n;
    __syncthreads();  // every thread has read the count before the next stage
    if (staged > static_cast<unsigned int>(kStage - kBlock)) flush();
  }
  __syncthreads();
  const unsigned int staged = s_n;
  __syncthreads();
  if (staged > 0u) flush();
  // counts (exact in FP64 below 2^53): one atomic per block and counter
  const double wk = wave_sum(n_kept), wo = wave_sum(n_over);
  if (lane == 0) {
    red[2 * (threadIdx.x / kWave)] = wk;
    red[2 * (threadIdx.x / kWave) + 1] = wo;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double k = 0.0, o = 0.0;
    for (int v = 0; v < kBlock / kWave; ++v) {
      k += red[2 * v];
      o += red[2 * v + 1];
    }
    if (k != 0.0) atomicAdd(reinterpret_cast<unsigned long long*>(P.state + SP_KEPT), static_cast<unsigned long long>(k));
    if (o != 0.0) atomicAdd(reinterpret_cast<unsigned long long*>(P.state + SP_OVER), static_cast<unsigned long long>(o));
    if (blockIdx.x == 0) atomicAdd(reinterpret_cast<unsigned long long*>(P.state + SP_TRIALS), P.ntrials);
  }
}

}  // namespace vmc
