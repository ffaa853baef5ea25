// vmc_kernels.hpp -- the sample-and-accumulate kernels (steps 2-4 of the
// six-step structure of Kanzaki, arXiv:1010.2107, Sec. 3.1).
//
// One sample per lane per loop trip: Philox words -> bin index -> grid map
// from the LDS table -> integrand -> w = f J.  Each block keeps a private
// FP64 histogram of sum w and sum w^2 per axis and bin in LDS (2 D LDS
// atomics per sample) and merges it with one global FP64 atomic per
// non-zero bin when it finishes; scalar sums are reduced over the wave with
// DPP shuffles and over the block through LDS, then added with one atomic
// per block.  Samples are never stored: the random stream is counter-based,
// so any pass can regenerate any sample.
#pragma once

#include <type_traits>

#include "vmc_device.hpp"

namespace vmc {

// Scalar block layout (doubles); mirrored in the public header.
enum : int {
  S_S1 = 0,
  S_S2 = 1,
  S_V = 2,
  S_NONFIN = 3,
  S_I = 4,
  S_VAR = 5,
  S_NEFF = 6,
  S_NZERO = 7,
  S_W = 8,
  S_MEAN = 9,
  S_M2 = 10,
  S_NITER = 11,
  S_NEXACT = 12,
  S_SUMEXACT = 13,
  S_IBAR = 14,
  S_SIGBAR = 15,
  S_CHI2 = 16,
  S_NTOTAL = 17,
  S_GRAD = 32,
  S_LEN = 128
};

// Block partial sums go to one of kStripes copies (block b to copy b mod
// kStripes) so that no address sees more than 1/kStripes of the blocks'
// atomics; the publish kernel adds the copies up.  A copy holds the 2 D N
// bin sums and then kStripeScal scalar slots: S1, S2, non-finite count,
// zero count, V, then per gradient parameter its sum, sum of squares and
// V_p.
constexpr int kStripes = 32;
constexpr int kStripeScal = 64;
enum : int { T_S1 = 0, T_S2 = 1, T_NONFIN = 2, T_NZERO = 3, T_V = 4, T_G = 5 };

// Pass kinds: forward sums, adjoint sums, both; KIND_CMAX (stratified
// forward only) also folds each cube's largest weight into cube_max.
enum : int { KIND_FWD = 1, KIND_ADJ = 2, KIND_FUSED = 3, KIND_CMAX = 4 };

// per-thread accumulator slots: S1, S2, non-finite count, zero count, then
// the gradient sums
constexpr int kA0 = 4;

struct SampleArgs {
  const float* table32;  // [d][N][2] (lo, width x 2^-24), FP32
  const double* edges;   // [d][N+1], FP64
  double* bins;          // [2][d][N] published bin sums
  double* stripes;       // kStripes copies of stripe_len doubles (block partial sums)
  double* scal;          // S_LEN doubles
  double* cube_max;      // [M] largest weight per cube (KIND_CMAX)
  const double* theta;   // device parameters
  Key key;
  uint32_t it, kid;
  uint32_t nbins;
  uint32_t ng;        // <= 1: plain
  uint32_t per_cube;  // nbins / ng when ng divides nbins, else 0
  DivU32 ngdiv;       // division by ng (stratified)
  double ng_inv;      // 1 / ng (stratified)
  uint32_t ng_wide;   // ng nbins >= 2^32 (stratified, ng not dividing nbins)
  uint32_t M;         // cubes
  uint32_t k;         // samples per cube
  uint32_t log2G;     // lanes per cube = 1 << log2G
  uint64_t ncall;     // plain: samples; stratified: k * M
  uint64_t block_items;  // samples (plain) or cube units (stratified) per tile
  uint64_t ntiles;       // tiles of the launch; block b takes tiles b, b + gridDim.x, ...
  uint32_t stripe_len;   // doubles per copy: 2 D N bins, then kStripeScal scalars (padded)
};

// Estimate of one iteration and its variance,
//   plain:      I = S1/n, var = (S2/n - I^2)/(n-1)
//   stratified: I = S1/(kM), var = sum_c (k S2_c - S1_c^2)/(k^2 (k-1) M^2),
// then the running combination with weights 1/var, updated with West's
// weighted incremental mean so that chi^2 needs no stored history.
// Iterations with var = 0 are exact; when any exist the combined value is
// their mean with zero error.
__device__ inline void finalize_one(double* scal, int strat, double n, double kd, double Md, int fwd, int ngrad) {
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

// Integrands that split their evaluation at the cuts (stage1: map, phase
// space, cuts; stage2: the matrix element) set kStaged; the plain kernel
// then queues the samples that pass in LDS, per wave, and runs stage 2 on
// full waves of queued samples.
template <class F, class = void>
struct StagedTraits {
  static constexpr bool value = false;
  static constexpr int words = 0;
};
template <class F>
struct StagedTraits<F, std::void_t<decltype(F::kStaged)>> {
  static constexpr bool value = F::kStaged;
  static constexpr int words = F::kStateWords;
};
constexpr int kQueueCap = kWave;  // entries per wave (at most 63 wait between runs)
// queue words per entry: the state, the Jacobian and the bin indices (4 per word)
template <class F>
constexpr int queue_words() {
  return StagedTraits<F>::words + 1 + (F::D + 3) / 4;
}
template <class F>
constexpr int queue_bytes() {
  return StagedTraits<F>::value ? (kBlock / kWave) * kQueueCap * queue_words<F>() * 4 : 0;
}
// The stratified kernels of the queued integrands queue the owner lane with
// each entry and keep, per wave, slots per cube the wave holds (sum w, sum
// w^2, largest w of the cube's chunks there, then sum and sum of squares of
// J df/dtheta_q per gradient) that lanes add the queued samples of other
// lanes into: 64 / G slots of each kind for G lanes per cube, one when a
// cube spans whole waves.  The queue's bytes per block (the slots, which
// depend on G and on the gradients, come on top).
template <class F>
constexpr int strat_queue_words() {
  return queue_words<F>() + 1;
}
template <class F>
constexpr int strat_queue_bytes() {
  return StagedTraits<F>::value ? (kBlock / kWave) * kQueueCap * strat_queue_words<F>() * 4 : 0;
}
__host__ __device__ constexpr uint32_t strat_slot_shift(uint32_t log2G) { return log2G < 6 ? log2G : 6; }
__host__ __device__ constexpr int strat_slot_kinds(int ngrad) { return 3 + 2 * ngrad; }
__host__ __device__ constexpr int strat_slot_bytes(uint32_t log2G, int ngrad) {
  return (kBlock / kWave) * strat_slot_kinds(ngrad) * 8 * (kWave >> strat_slot_shift(log2G));
}

// LDS layout: grid table first (16-byte entries for FP64), then the histogram
// [2][d][N] (adjacent bins 8 bytes apart, so a wave's random bins spread
// over the LDS banks).
template <typename T, int D>
__device__ __forceinline__ void load_table(const SampleArgs& A, typename TabEntry<T>::type* tab) {
  const int n = D * static_cast<int>(A.nbins);
  for (int i = threadIdx.x; i < n; i += kBlock) {
    if constexpr (sizeof(T) == 4) {
      tab[i] = reinterpret_cast<const float2*>(A.table32)[i];
    } else {
      const int a = i / A.nbins, j = i - a * A.nbins;
      const double* e = A.edges + static_cast<size_t>(a) * (A.nbins + 1);
      tab[i] = make_double2(e[j], (e[j + 1] - e[j]) * kWidthScale);
    }
  }
}

// Map the words of one sample to the point x and the Jacobian.
template <typename T, int D, bool STRAT>
__device__ __forceinline__ void make_point(const SampleArgs& A, const typename TabEntry<T>::type* tab,
                                           const uint32_t (&w)[D], const uint32_t (&cc)[D], int (&j)[D],
                                           T (&x)[D], T& jac) {
  const int N = static_cast<int>(A.nbins);
  const T Nk = static_cast<T>(N) * static_cast<T>(1.0 / kWidthScale);  // per-axis Jacobian factor, exact
  jac = T(1);
  // stratified: the bins of all axes first, with the (launch-uniform) choice
  // of bin map taken once, so that the table reads below form one
  // straight-line run
  T offs[D];
  if constexpr (STRAT) {
    if (A.per_cube) {
#pragma unroll
      for (int a = 0; a < D; ++a) bin_strat_div<T>(w[a], cc[a], A.per_cube, j[a], offs[a]);
    } else if (D > 1 || !A.ng_wide) {
      const T inv = static_cast<T>(A.ng_inv);
#pragma unroll
      for (int a = 0; a < D; ++a) bin_strat_gen<T>(w[a], cc[a], A.ngdiv, A.nbins, inv, j[a], offs[a]);
    } else if constexpr (D == 1) {
      // ng N >= 2^32 needs ng > 2^24, which ng^dim <= 2^31 allows on one axis only
      bin_strat_wide<T>(w[0], cc[0], A.ng, A.nbins, j[0], offs[0]);
    }
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    T off;
    if constexpr (!STRAT) {
      bin_plain<T>(w[a], A.nbins, j[a], off);
    } else {
      off = offs[a];
    }
    const auto e = tab[a * N + j[a]];
    x[a] = fma(off, e.y, e.x);
    jac *= e.y * Nk;  // J = prod N width; N width is exact from the scaled width
  }
}

template <class F, int KIND>
__device__ __forceinline__ void accumulate(const SampleArgs& A, double* hist, const int (&j)[F::D],
                                           typename F::T fv, typename F::T jac,
                                           const typename F::T (&g)[F::NGRAD + 1], double* acc,
                                           uint32_t* cnt) {
  constexpr int D = F::D;
  constexpr bool HIST = KIND & KIND_FWD, GRAD = KIND & KIND_ADJ;
  const int N = static_cast<int>(A.nbins);
  if (HIST) {
    const auto wv = fv * jac;  // w = f J in the integrand's precision
    const double wd = static_cast<double>(wv);
    acc[0] += wd;
    acc[1] += wd * wd;
    cnt[0] += vfinite(wv) ? 0u : 1u;
    cnt[1] += (wv == 0) ? 1u : 0u;
    const int dn = D * N;  // sum w^2 sits one axis set after sum w
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double* h = &hist[a * N + j[a]];
      lds_add(h, wd);
      lds_add(h + dn, wd * wd);
    }
  }
  if (GRAD) {
#pragma unroll
    for (int q = 0; q < F::NGRAD; ++q) {
      const double gq = static_cast<double>(g[q] * jac);
      acc[kA0 + q] += gq;
      acc[kA0 + F::NGRAD + q] += gq * gq;
    }
  }
}

// The block's copy of the partial sums.
__device__ __forceinline__ double* block_stripe(const SampleArgs& A) {
  return A.stripes + static_cast<size_t>(blockIdx.x % kStripes) * A.stripe_len;
}

// Add the block's histogram to its copy of the bin sums (non-zero bins).
template <int D>
__device__ __forceinline__ void flush_hist(const SampleArgs& A, const double* hist) {
  double* dst = block_stripe(A);
  const int n = 2 * D * static_cast<int>(A.nbins);
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const double v = hist[i];
    if (v != 0.0) global_add(&dst[i], v);
  }
}

// Add the block's accumulators and histogram to its copy.
template <class F, int KIND, int NACC>
__device__ __forceinline__ void flush_block(const SampleArgs& A, double* hist, const double (&acc)[NACC],
                                            double* red) {
  constexpr int D = F::D;
  constexpr bool HIST = KIND & KIND_FWD, GRAD = KIND & KIND_ADJ;
  constexpr int NG = GRAD ? F::NGRAD : 0;
  int idx[NACC];
  idx[0] = T_S1;
  idx[1] = T_S2;
  idx[2] = T_NONFIN;
  idx[3] = T_NZERO;
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    idx[kA0 + q] = T_G + q;
    idx[kA0 + NG + q] = T_G + NG + q;
  }
  block_sum_to_global<NACC>(acc, red, block_stripe(A) + 2 * D * A.nbins, idx);
  if (HIST) flush_hist<D>(A, hist);
}

template <class F, int KIND>
__device__ __forceinline__ double* setup_lds(const SampleArgs& A, unsigned char* smem,
                                             typename TabEntry<typename F::T>::type*& tab) {
  using TE = typename TabEntry<typename F::T>::type;
  constexpr int D = F::D;
  tab = reinterpret_cast<TE*>(smem);
  double* hist = reinterpret_cast<double*>(smem + sizeof(TE) * D * A.nbins);
  load_table<typename F::T, D>(A, tab);
  if (KIND & KIND_FWD) {
    const int n = 2 * D * static_cast<int>(A.nbins);
    for (int i = threadIdx.x; i < n; i += kBlock) hist[i] = 0.0;
  }
  __syncthreads();
  return hist;
}

// The integrand's per-parameter constants (normalisations, erf, logs in
// FP64) are computed once per block by thread 0 and broadcast through LDS.
template <class F>
__device__ __forceinline__ F block_setup(const double* theta) {
  __shared__ F shared_fn;
  if (threadIdx.x == 0) shared_fn.setup(theta);
  __syncthreads();
  return shared_fn;
}

// ---------------------------------------------------------------------------
// Plain (VEGAS) sampling: tile t is samples [t B, (t+1) B), the block's
// lanes stride through it; by default every block takes one tile and the
// hardware dispatcher balances the blocks over the CUs.
// ---------------------------------------------------------------------------
template <class F, int KIND>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(StagedTraits<F>::value ? 3 : 1)))
void k_plain(const SampleArgs A) {
  using T = typename F::T;
  constexpr int D = F::D;
  constexpr int NG = (KIND & KIND_ADJ) ? F::NGRAD : 0;
  constexpr int NACC = kA0 + 2 * NG;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[(kBlock / kWave) * NACC];
  typename TabEntry<T>::type* tab;
  double* hist = setup_lds<F, KIND>(A, smem, tab);

  const F fn = block_setup<F>(A.theta);
  double acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.0;
  uint32_t cnt[2] = {0u, 0u};  // non-finite and zero weights

  const uint32_t dummy_cc[D] = {};
  if constexpr (StagedTraits<F>::value) {
    // Per-wave LDS queue (structure of arrays) of samples that passed stage 1.
    // When the waiting and the newly passed samples make a full wave, every
    // lane runs stage 2 once: a lane that passed on its own sample, any other
    // lane on the newest queued one.  Otherwise the passed samples join the
    // queue, which therefore never holds more than 63.
    constexpr int NQ = queue_words<F>();
    constexpr int NS = StagedTraits<F>::words;
    constexpr int NPK = (D + 3) / 4;  // bin indices, four per word
    using State = typename F::State;
    const int lane = threadIdx.x & (kWave - 1);
    // after the histogram (forward passes) or right after the table
    float* q = reinterpret_cast<float*>(hist + ((KIND & KIND_FWD) ? 2 * D * A.nbins : 0)) +
               (threadIdx.x / kWave) * NQ * kQueueCap;
    uint32_t* qj = reinterpret_cast<uint32_t*>(q + (NS + 1) * kQueueCap);
    auto push = [&](int e, const State& st, T jac, const uint32_t (&pk)[NPK]) {
      F::store_state(st, q, kQueueCap, e);
      q[NS * kQueueCap + e] = static_cast<float>(jac);
#pragma unroll
      for (int w = 0; w < NPK; ++w) qj[w * kQueueCap + e] = pk[w];
    };
    auto pop = [&](int e, State& st, T& jac, uint32_t (&pk)[NPK]) {
      st = F::load_state(q, kQueueCap, e);
      jac = static_cast<T>(q[NS * kQueueCap + e]);
#pragma unroll
      for (int w = 0; w < NPK; ++w) pk[w] = qj[w * kQueueCap + e];
    };
    auto run = [&](const State& st, T jac, const uint32_t (&pk)[NPK]) {
      int j[D];
#pragma unroll
      for (int a = 0; a < D; ++a) j[a] = static_cast<int>((pk[a / 4] >> (8 * (a % 4))) & 0xFFu);
      T g[F::NGRAD + 1];
      const T fv = fn.template stage2<(KIND & KIND_ADJ) != 0>(st, g);
      accumulate<F, KIND>(A, hist, j, fv, jac, g, acc, cnt);
    };
    int qn = 0;  // entries waiting (wave-uniform)
    for (uint64_t t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
      const uint64_t b0 = t * A.block_items;
      const uint64_t b1 = min(b0 + A.block_items, A.ncall);
      for (uint64_t base = b0; base < b1; base += kBlock) {
        const uint64_t s = base + threadIdx.x;
        bool pass = false;
        State st;
        uint32_t pk[NPK] = {};
        T jac = T(0);
        if (s < b1) {
          uint32_t w[D];
          // The round keys are recomputed per sample in scalar registers
          // rather than held across the loop, where they crowd the scalar
          // register file into spills.
          Key key = A.key;
          asm volatile("" : "+s"(key.k0), "+s"(key.k1));
          sample_words<D>(static_cast<uint32_t>(s), A.it, A.kid, key, w);
          T x[D];
          int j[D];
          make_point<T, D, false>(A, tab, w, dummy_cc, j, x, jac);
#pragma unroll
          for (int a = 0; a < D; ++a) pk[a / 4] |= static_cast<uint32_t>(j[a]) << (8 * (a % 4));
          pass = fn.stage1(x, st);
          cnt[1] += pass ? 0u : 1u;  // f = 0 outside the cuts: nothing else to add
        }
        const uint64_t m = __ballot(pass);
        const int np = static_cast<int>(__popcll(m));
        if (qn + np >= kWave) {
          if (!pass) pop(qn - 1 - static_cast<int>(__popcll(~m & __lanemask_lt())), st, jac, pk);
          run(st, jac, pk);
          qn -= kWave - np;
        } else {
          if (pass) push(qn + static_cast<int>(__popcll(m & __lanemask_lt())), st, jac, pk);
          qn += np;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (lane < qn) {
      State st;
      T jac;
      uint32_t pk[NPK];
      pop(lane, st, jac, pk);
      run(st, jac, pk);
    }
  } else {
    for (uint64_t t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
      const uint64_t b0 = t * A.block_items;
      const uint64_t b1 = min(b0 + A.block_items, A.ncall);
      for (uint64_t s = b0 + threadIdx.x; s < b1; s += kBlock) {
        uint32_t w[D];
        sample_words<D>(static_cast<uint32_t>(s), A.it, A.kid, A.key, w);
        int j[D];
        T x[D], jac;
        make_point<T, D, false>(A, tab, w, dummy_cc, j, x, jac);
        T g[F::NGRAD + 1];
        const T fv = fn.template eval<(KIND & KIND_ADJ) != 0>(x, g);
        accumulate<F, KIND>(A, hist, j, fv, jac, g, acc, cnt);
      }
    }
  }
  acc[2] = static_cast<double>(cnt[0]);
  acc[3] = static_cast<double>(cnt[1]);
  __syncthreads();
  flush_block<F, KIND, NACC>(A, hist, acc, red);
}

// ---------------------------------------------------------------------------
// Stratified (BASES) sampling.  A unit is (cube c, chunk g); the 2^log2G
// chunks of one cube sit on adjacent lanes (up to 64 in a wave, up to 256
// across the waves of a block) and split the cube's k samples s = c + t M
// between them.  After the cube's samples the chunk sums are combined with
// lane shuffles (and through LDS across waves) and the first lane adds the
// cube's k S2_c - S1_c^2 (and its gradient analogue) to the variance sums.
// The passes of integrands that split at the cuts queue the samples that
// pass, as the plain kernel does; a queued sample's weight (and gradient)
// returns to the cube it belongs to through the wave's LDS slots.
// ---------------------------------------------------------------------------
// The queued forward and fused passes ask for at least 3 waves per SIMD,
// the occupancy of the plain kernel, which bounds their registers at 168:
// the fused W + 4 partons pass then spills 108 bytes per lane and runs
// 1.5 % slower than at 2 waves, the fused W + 2 partons pass 17 % faster.
template <class F, int KIND>
constexpr int strat_min_waves() {
  return (StagedTraits<F>::value && (KIND & KIND_FWD)) ? 3 : 1;
}

template <class F, int KIND>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(strat_min_waves<F, KIND>())))
void k_strat(const SampleArgs A) {
  using T = typename F::T;
  constexpr int D = F::D;
  constexpr bool FWD = KIND & KIND_FWD, GRAD = KIND & KIND_ADJ, CMAX = KIND & KIND_CMAX;
  constexpr int NG = GRAD ? F::NGRAD : 0;
  constexpr int NACC = kA0 + 2 * NG + 1 + NG;  // + V and V_p
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[(kBlock / kWave) * NACC];
  typename TabEntry<T>::type* tab;
  double* hist = setup_lds<F, KIND>(A, smem, tab);

  const F fn = block_setup<F>(A.theta);
  double acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.0;
  uint32_t cnt[2] = {0u, 0u};  // non-finite and zero weights

  const uint32_t G = 1u << A.log2G;
  const uint64_t units = static_cast<uint64_t>(A.M) << A.log2G;
  const double kd = static_cast<double>(A.k);
  for (uint64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const uint64_t u0 = tile * A.block_items;
    const uint64_t u1 = min(u0 + A.block_items, units);
    for (uint64_t base = u0; base < u1; base += kBlock) {
      const uint64_t u = base + threadIdx.x;
      const bool active = u < u1;
      const uint32_t c = static_cast<uint32_t>(u >> A.log2G);
      const uint32_t gidx = static_cast<uint32_t>(u) & (G - 1);
      // The unit's cube coordinates.  From dim 4 up (ng < 256, as
      // ng^dim <= 2^31) they are packed four to a word and taken apart again
      // for every sample behind an opaque copy: held whole, they and the
      // per-axis values derived from them would stay live across the
      // sample loop in dim registers each.
      constexpr bool PACK = D >= 4;
      uint32_t ccp[PACK ? (D + 3) / 4 : D];
      {
        uint32_t cc[D];
        digits<D>(c, A.ngdiv, cc);
        if constexpr (PACK) {
#pragma unroll
          for (int v = 0; v < (D + 3) / 4; ++v) ccp[v] = 0u;
#pragma unroll
          for (int a = 0; a < D; ++a) ccp[a / 4] |= cc[a] << (8 * (a % 4));
        } else {
#pragma unroll
          for (int a = 0; a < D; ++a) ccp[a] = cc[a];
        }
      }
      auto coords = [&](uint32_t (&cc)[D]) {
        if constexpr (PACK) {
#pragma unroll
          for (int v = 0; v < (D + 3) / 4; ++v) asm volatile("" : "+v"(ccp[v]));
#pragma unroll
          for (int a = 0; a < D; ++a) cc[a] = (ccp[a / 4] >> (8 * (a % 4))) & 0xFFu;
        } else {
#pragma unroll
          for (int a = 0; a < D; ++a) cc[a] = ccp[a];
        }
      };
      const uint32_t t0 = active ? static_cast<uint32_t>((static_cast<uint64_t>(gidx) * A.k) >> A.log2G) : 0u;
      const uint32_t t1 =
          active ? static_cast<uint32_t>((static_cast<uint64_t>(gidx + 1) * A.k) >> A.log2G) : 0u;
      double c1 = 0.0, c2 = 0.0, cm = 0.0;
      double cg1[NG + 1], cg2[NG + 1];
#pragma unroll
      for (int q = 0; q < NG; ++q) cg1[q] = cg2[q] = 0.0;
      if constexpr (StagedTraits<F>::value) {
        // Stage 1 for every sample of the chunk (the loop runs to the
        // longest chunk of the wave), stage 2 on full waves of queued samples.
        constexpr int NQ = strat_queue_words<F>();
        constexpr int NSL = strat_slot_kinds(NG);
        constexpr int NS = StagedTraits<F>::words;
        constexpr int NPK = (D + 3) / 4;
        using State = typename F::State;
        const int lane = threadIdx.x & (kWave - 1);
        // the wave's cubes: lane >> sh (sh = log2 G up to 6), S of them
        const uint32_t sh = strat_slot_shift(A.log2G);
        const int S = kWave >> sh;
        // after the histogram (forward passes) or right after the table
        double* const after = hist + (FWD ? 2 * D * A.nbins : 0);
        double* slot = after + (threadIdx.x / kWave) * NSL * S;  // [NSL][S]
        float* q = reinterpret_cast<float*>(after + (kBlock / kWave) * NSL * S) +
                   (threadIdx.x / kWave) * NQ * kQueueCap;
        uint32_t* qj = reinterpret_cast<uint32_t*>(q + (NS + 1) * kQueueCap);
        uint32_t* qo = qj + NPK * kQueueCap;  // owner lane
        if (lane < S) {
#pragma unroll
          for (int v = 0; v < NSL; ++v) slot[v * S + lane] = 0.0;
        }
        __builtin_amdgcn_wave_barrier();
        auto push = [&](int e, const State& st, T jc, const uint32_t (&pk)[NPK]) {
          F::store_state(st, q, kQueueCap, e);
          q[NS * kQueueCap + e] = static_cast<float>(jc);
#pragma unroll
          for (int v = 0; v < NPK; ++v) qj[v * kQueueCap + e] = pk[v];
          qo[e] = static_cast<uint32_t>(lane);
        };
        auto pop = [&](int e, State& st, T& jc, uint32_t (&pk)[NPK], int& owner) {
          st = F::load_state(q, kQueueCap, e);
          jc = static_cast<T>(q[NS * kQueueCap + e]);
#pragma unroll
          for (int v = 0; v < NPK; ++v) pk[v] = qj[v * kQueueCap + e];
          owner = static_cast<int>(qo[e]);
        };
        auto run = [&](const State& st, T jc, const uint32_t (&pk)[NPK], int owner) {
          int j[D];
#pragma unroll
          for (int a = 0; a < D; ++a) j[a] = static_cast<int>((pk[a / 4] >> (8 * (a % 4))) & 0xFFu);
          T g[F::NGRAD + 1];
          const T fv = fn.template stage2<GRAD>(st, g);
          accumulate<F, KIND>(A, hist, j, fv, jc, g, acc, cnt);
          const double wd = static_cast<double>(fv * jc);
          double gd[NG + 1];
#pragma unroll
          for (int v = 0; v < NG; ++v) gd[v] = static_cast<double>(g[v] * jc);
          if (owner == lane) {
            if (FWD) {
              c1 += wd;
              c2 += wd * wd;
              if (CMAX) cm = fmax(cm, wd);  // a NaN weight never becomes the maximum
            }
#pragma unroll
            for (int v = 0; v < NG; ++v) {
              cg1[v] += gd[v];
              cg2[v] += gd[v] * gd[v];
            }
          } else {
            const int oc = owner >> sh;  // the owner's cube in the wave
            if (FWD) {
              lds_add(&slot[oc], wd);
              lds_add(&slot[S + oc], wd * wd);
              if (CMAX && wd > 0.0) lds_max_pos(&slot[2 * S + oc], wd);
            }
#pragma unroll
            for (int v = 0; v < NG; ++v) {
              lds_add(&slot[(3 + 2 * v) * S + oc], gd[v]);
              lds_add(&slot[(4 + 2 * v) * S + oc], gd[v] * gd[v]);
            }
          }
        };
        const uint32_t nt = static_cast<uint32_t>((static_cast<uint64_t>(A.k) + G - 1) >> A.log2G);
        int qn = 0;  // entries waiting (wave-uniform)
        for (uint32_t i = 0; i < nt; ++i) {
          const uint32_t t = t0 + i;
          bool pass = false;
          State st;
          uint32_t pk[NPK] = {};
          T jc = T(0);
          if (t < t1) {  // t1 = 0 for inactive units
            uint32_t w[D];
            sample_words<D>(c + t * A.M, A.it, A.kid, A.key, w);
            T x[D];
            int j[D];
            uint32_t cc[D];
            coords(cc);
            make_point<T, D, true>(A, tab, w, cc, j, x, jc);
#pragma unroll
            for (int a = 0; a < D; ++a) pk[a / 4] |= static_cast<uint32_t>(j[a]) << (8 * (a % 4));
            pass = fn.stage1(x, st);
            cnt[1] += pass ? 0u : 1u;  // f = 0 outside the cuts
          }
          const uint64_t m = __ballot(pass);
          const int np = static_cast<int>(__popcll(m));
          if (qn + np >= kWave) {
            int owner = lane;
            if (!pass) pop(qn - 1 - static_cast<int>(__popcll(~m & __lanemask_lt())), st, jc, pk, owner);
            run(st, jc, pk, owner);
            qn -= kWave - np;
          } else {
            if (pass) push(qn + static_cast<int>(__popcll(m & __lanemask_lt())), st, jc, pk);
            qn += np;
          }
          __builtin_amdgcn_wave_barrier();
        }
        if (lane < qn) {
          State st;
          T jc;
          uint32_t pk[NPK];
          int owner;
          pop(lane, st, jc, pk, owner);
          run(st, jc, pk, owner);
        }
        __builtin_amdgcn_wave_barrier();
        if ((lane & ((1 << sh) - 1)) == 0) {  // the first lane of each cube in the wave
          const int oc = lane >> sh;
          if (FWD) {
            c1 += slot[oc];
            c2 += slot[S + oc];
            if (CMAX) cm = fmax(cm, slot[2 * S + oc]);
          }
#pragma unroll
          for (int v = 0; v < NG; ++v) {
            cg1[v] += slot[(3 + 2 * v) * S + oc];
            cg2[v] += slot[(4 + 2 * v) * S + oc];
          }
        }
        __builtin_amdgcn_wave_barrier();
      } else {
        for (uint32_t t = t0; t < t1; ++t) {
          const uint32_t s = c + t * A.M;
          uint32_t w[D];
          sample_words<D>(s, A.it, A.kid, A.key, w);
          int j[D];
          T x[D], jac;
          uint32_t cc[D];
          coords(cc);
          make_point<T, D, true>(A, tab, w, cc, j, x, jac);
          T g[F::NGRAD + 1];
          const T fv = fn.template eval<GRAD>(x, g);
          accumulate<F, KIND>(A, hist, j, fv, jac, g, acc, cnt);
          if (FWD) {
            const double wd = static_cast<double>(fv * jac);
            c1 += wd;
            c2 += wd * wd;
            if (CMAX) cm = fmax(cm, wd);  // a NaN weight never becomes the maximum
          }
#pragma unroll
          for (int q = 0; q < NG; ++q) {
            const double gq = static_cast<double>(g[q] * jac);
            cg1[q] += gq;
            cg2[q] += gq * gq;
          }
        }
      }
      const uint32_t Gw = G < kWave ? G : static_cast<uint32_t>(kWave);  // chunks of a cube in one wave
      for (uint32_t off = 1; off < Gw; off <<= 1) {
        if (FWD) {
          c1 += __shfl_xor(c1, off, kWave);
          c2 += __shfl_xor(c2, off, kWave);
        }
        if (CMAX) cm = fmax(cm, __shfl_xor(cm, off, kWave));
#pragma unroll
        for (int q = 0; q < NG; ++q) {
          cg1[q] += __shfl_xor(cg1[q], off, kWave);
          cg2[q] += __shfl_xor(cg2[q], off, kWave);
        }
      }
      if (G > static_cast<uint32_t>(kWave)) {
        // a cube spans G/64 waves of the block (units come in runs of
        // kBlock, a multiple of G): their partial sums meet in LDS
        __shared__ double xw[kBlock / kWave][3 + 2 * NG];
        const int wv = threadIdx.x / kWave;
        const bool head = (threadIdx.x & (kWave - 1)) == 0;
        if (head) {
          xw[wv][0] = c1;
          xw[wv][1] = c2;
          xw[wv][2] = cm;
#pragma unroll
          for (int q = 0; q < NG; ++q) {
            xw[wv][3 + 2 * q] = cg1[q];
            xw[wv][4 + 2 * q] = cg2[q];
          }
        }
        __syncthreads();
        const int per = static_cast<int>(G / kWave);
        if (head && wv % per == 0) {
          for (int o = 1; o < per; ++o) {
            c1 += xw[wv + o][0];
            c2 += xw[wv + o][1];
            cm = fmax(cm, xw[wv + o][2]);
#pragma unroll
            for (int q = 0; q < NG; ++q) {
              cg1[q] += xw[wv + o][3 + 2 * q];
              cg2[q] += xw[wv + o][4 + 2 * q];
            }
          }
        }
        __syncthreads();
      }
      if (active && gidx == 0) {
        if (FWD) acc[kA0 + 2 * NG] += kd * c2 - c1 * c1;
        if (CMAX && cm > A.cube_max[c]) A.cube_max[c] = cm;  // one writer per cube and launch
#pragma unroll
        for (int q = 0; q < NG; ++q) acc[kA0 + 1 + 2 * NG + q] += kd * cg2[q] - cg1[q] * cg1[q];
      }
    }
  }
  acc[2] = static_cast<double>(cnt[0]);
  acc[3] = static_cast<double>(cnt[1]);
  __syncthreads();
  // the V slots go through the same block reduction
  int idx[NACC];
  idx[0] = T_S1;
  idx[1] = T_S2;
  idx[2] = T_NONFIN;
  idx[3] = T_NZERO;
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    idx[kA0 + q] = T_G + q;
    idx[kA0 + NG + q] = T_G + NG + q;
    idx[kA0 + 1 + 2 * NG + q] = T_G + 2 * NG + q;
  }
  idx[kA0 + 2 * NG] = T_V;
  block_sum_to_global<NACC>(acc, red, block_stripe(A) + 2 * D * A.nbins, idx);
  if (FWD) flush_hist<D>(A, hist);
}

// ---------------------------------------------------------------------------
// Per-sample dump (tests): the same words, point and integrand as the
// accumulating kernels, for samples [s0, s0 + count).
// ---------------------------------------------------------------------------
struct DumpArgs {
  SampleArgs A;
  uint64_t s0, count;
  uint32_t* words;  // [count][D]
  uint8_t* bins;    // [count][D] bin index per axis
  void* w;
  void* f;
  void* jac;
  void* grad;  // [count][NGRAD] df/dtheta_p
};

// GRAD: also the per-sample gradients (a kernel of its own, so that the
// forward dump keeps the code, and the weights, of the accumulating kernels)
template <class F, bool GRAD>
__global__ __launch_bounds__(kBlock) void k_dump(const DumpArgs P) {
  using T = typename F::T;
  constexpr int D = F::D;
  extern __shared__ __align__(16) unsigned char smem[];
  const SampleArgs& A = P.A;
  typename TabEntry<T>::type* tab;
  (void)setup_lds<F, 0>(A, smem, tab);
  const F fn = block_setup<F>(A.theta);
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= P.count) return;
  const uint32_t s = static_cast<uint32_t>(P.s0 + i);
  uint32_t w[D];
  sample_words<D>(s, A.it, A.kid, A.key, w);
  uint32_t cc[D];
  int j[D];
  T x[D], jac;
  if (A.ng > 1) {
    uint32_t r = s % A.M;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      cc[a] = r % A.ng;
      r /= A.ng;
    }
    make_point<T, D, true>(A, tab, w, cc, j, x, jac);
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) cc[a] = 0;
    make_point<T, D, false>(A, tab, w, cc, j, x, jac);
  }
  T g[F::NGRAD + 1];
#pragma unroll
  for (int q = 0; q <= F::NGRAD; ++q) g[q] = T(0);
  T fv;
  if constexpr (StagedTraits<F>::value) {
    // The sample kernels hand the stage-1 state to stage 2 through LDS or a
    // register merge, where no multiply-add can fuse across the boundary;
    // the state goes through an opaque copy here as well, so the dump gives
    // the weights those kernels add up, bit for bit.
    typename F::State st;
    const bool pass = fn.stage1(x, st);
    float sw[StagedTraits<F>::words];
    F::store_state(st, sw, 1, 0);
#pragma unroll
    for (int i = 0; i < StagedTraits<F>::words; ++i) asm volatile("" : "+v"(sw[i]));
    fv = pass ? fn.template stage2<GRAD>(F::load_state(sw, 1, 0), g) : T(0);
  } else {
    fv = fn.template eval<GRAD>(x, g);
  }
  if (P.words) {
#pragma unroll
    for (int a = 0; a < D; ++a) P.words[i * D + a] = w[a];
  }
  if (P.bins) {
#pragma unroll
    for (int a = 0; a < D; ++a) P.bins[i * D + a] = static_cast<uint8_t>(j[a]);
  }
  if (P.w) static_cast<T*>(P.w)[i] = fv * jac;
  if (P.f) static_cast<T*>(P.f)[i] = fv;
  if (P.jac) static_cast<T*>(P.jac)[i] = jac;
  if constexpr (GRAD) {
#pragma unroll
    for (int q = 0; q < F::NGRAD; ++q) static_cast<T*>(P.grad)[i * F::NGRAD + q] = g[q];
  }
}

}  // namespace vmc
