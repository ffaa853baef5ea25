// vmc_batch.hip -- many independent integrals of uneven dimension and call
// count in one persistent launch (the batched form of the per-iteration
// sample-and-accumulate pass, steps 2-4 of the six-step structure of
// Kanzaki, arXiv:1010.2107, Sec. 3.1), plus the batched estimate and grid
// refinement.
//
// Work list: tiles (integral k, contiguous sample range), largest integrals
// first.  Persistent blocks take tiles from a device counter.  A block keeps
// its LDS table and histogram while consecutive tiles belong to the same
// integral and merges them (one global atomic per non-zero bin, one per
// scalar) only when the integral changes and at the end.  The dimension of
// the current integral selects a dimension-specialised tile body, so every
// per-axis array stays in registers.  The random words of sample s of
// integral k use the counter (s, word group, it, k), so results do not
// depend on the schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "vmc.h"
#include "vmc_error.hpp"
#include "vmc_gauss.hpp"
#include "vmc_small.hpp"

using namespace vmc;

namespace {

constexpr int kDmax = 12;

struct BatchDesc {
  uint64_t ncall;
  uint32_t d, kid;
  uint32_t off_edges, off_table, off_bins, off_theta, off_scal;
  uint32_t pad;
};
static_assert(sizeof(BatchDesc) == 40, "descriptor layout");

struct BatchTile {
  uint32_t k, s0, s1, pad;
};

struct AxisRef {
  uint32_t k, a;
};

struct BatchArgs {
  const BatchDesc* desc;
  const BatchTile* tiles;
  uint32_t* counter;
  double* edges;
  float* table;
  double* bins;
  double* scal;
  const double* theta;
  Key key;
  uint32_t it;
  uint32_t ntiles;
  uint32_t nbins;
};

template <int NG>
constexpr int batch_nacc() {
  return kA0 + 2 * NG;
}

// Merge a block's accumulators for integral k into its scalar block and bins.
template <int NGMAX, int NACC>
__device__ __forceinline__ void batch_flush(const BatchArgs& B, int k, int d, double* hist, double (&acc)[NACC],
                                            uint32_t (&cnt)[2], double* red, bool fwd) {
  const BatchDesc& ds = B.desc[k];
  acc[2] = static_cast<double>(cnt[0]);
  acc[3] = static_cast<double>(cnt[1]);
  int idx[NACC];
  idx[0] = S_S1;
  idx[1] = S_S2;
  idx[2] = S_NONFIN;
  idx[3] = S_NZERO;
#pragma unroll
  for (int q = 0; q < NGMAX; ++q) {
    idx[kA0 + q] = S_GRAD + 5 * q;
    idx[kA0 + NGMAX + q] = S_GRAD + 5 * q + 1;
  }
  __syncthreads();
  block_sum_to_global<NACC>(acc, red, B.scal + ds.off_scal, idx);
  if (fwd) {
    const int n = 2 * d * static_cast<int>(B.nbins);
    double* gb = B.bins + ds.off_bins;
    for (int i = threadIdx.x; i < n; i += kBlock) {
      const double v = hist[i];
      if (v != 0.0) global_add(&gb[i], v);
    }
  }
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.0;
  cnt[0] = cnt[1] = 0u;
  __syncthreads();
}

template <typename T, int D, int KIND, int NGMAX, int NACC>
__device__ __forceinline__ void batch_tile(const BatchArgs& B, const BatchDesc& ds, const BatchTile& tl,
                                           const typename TabEntry<T>::type* tab, double* hist,
                                           double (&acc)[NACC], uint32_t (&cnt)[2]) {
  constexpr bool FWD = KIND & KIND_FWD, GRAD = KIND & KIND_ADJ;
  const int N = static_cast<int>(B.nbins);
  const T Nk = static_cast<T>(N) * static_cast<T>(1.0 / kWidthScale);
  const GaussAxesF<T, D> fn = block_setup<GaussAxesF<T, D>>(B.theta + ds.off_theta);
  for (uint32_t s = tl.s0 + threadIdx.x; s < tl.s1; s += kBlock) {
    uint32_t w[D];
    sample_words<D>(s, B.it, ds.kid, B.key, w);
    int j[D];
    T x[D];
    T jac = T(1);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T off;
      bin_plain<T>(w[a], B.nbins, j[a], off);
      const auto e = tab[a * N + j[a]];
      x[a] = fma(off, e.y, e.x);
      jac *= e.y * Nk;
    }
    T g[D + 2];
    const T fv = fn.template eval<GRAD>(x, g);
    if (FWD) {
      const T wv = fv * jac;
      const double wd = static_cast<double>(wv);
      acc[0] += wd;
      acc[1] += wd * wd;
      cnt[0] += vfinite(wv) ? 0u : 1u;
      cnt[1] += (wv == 0) ? 1u : 0u;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        lds_add(&hist[a * N + j[a]], wd);
        lds_add(&hist[(D + a) * N + j[a]], wd * wd);
      }
    }
    if (GRAD) {
#pragma unroll
      for (int q = 0; q < D + 1; ++q) {
        const double gq = static_cast<double>(g[q] * jac);
        acc[kA0 + q] += gq;
        acc[kA0 + NGMAX + q] += gq * gq;
      }
    }
  }
}

template <typename T, int KIND>
__global__ __launch_bounds__(kBlock) void k_batched(const BatchArgs B) {
  constexpr bool FWD = KIND & KIND_FWD, GRAD = KIND & KIND_ADJ;
  constexpr int NGMAX = GRAD ? kDmax + 1 : 0;
  constexpr int NACC = batch_nacc<NGMAX>();
  using TE = typename TabEntry<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[(kBlock / kWave) * NACC];
  __shared__ uint32_t s_tile;
  const int N = static_cast<int>(B.nbins);
  TE* tab = reinterpret_cast<TE*>(smem);
  double* hist = reinterpret_cast<double*>(smem + sizeof(TE) * kDmax * N);
  double acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.0;
  uint32_t cnt[2] = {0u, 0u};
  int cur = -1, cur_d = 0;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(B.counter, 1u);
    __syncthreads();
    const uint32_t t = s_tile;
    if (t >= B.ntiles) break;  // same t in every thread: the whole block leaves
    const BatchTile tl = B.tiles[t];
    if (static_cast<int>(tl.k) != cur) {
      if (cur >= 0) batch_flush<NGMAX, NACC>(B, cur, cur_d, hist, acc, cnt, red, FWD);
      cur = static_cast<int>(tl.k);
      const BatchDesc& ds = B.desc[cur];
      cur_d = static_cast<int>(ds.d);
      const int n = cur_d * N;
      for (int i = threadIdx.x; i < n; i += kBlock) {
        if constexpr (sizeof(T) == 4) {
          tab[i] = reinterpret_cast<const float2*>(B.table + ds.off_table)[i];
        } else {
          const int a = i / N, jb = i - a * N;
          const double* e = B.edges + ds.off_edges + static_cast<size_t>(a) * (N + 1);
          tab[i] = make_double2(e[jb], (e[jb + 1] - e[jb]) * kWidthScale);
        }
      }
      if (FWD)
        for (int i = threadIdx.x; i < 2 * n; i += kBlock) hist[i] = 0.0;
    }
    __syncthreads();  // table ready, and every thread has read s_tile
    const BatchDesc& ds = B.desc[cur];
    switch (cur_d) {
#define VMC_CASE(DD)                                                                 \
  case DD:                                                                           \
    batch_tile<T, DD, KIND, NGMAX, NACC>(B, ds, tl, tab, hist, acc, cnt); \
    break;
      VMC_CASE(1)
      VMC_CASE(2)
      VMC_CASE(3)
      VMC_CASE(4)
      VMC_CASE(5)
      VMC_CASE(6)
      VMC_CASE(7)
      VMC_CASE(8)
      VMC_CASE(9)
      VMC_CASE(10)
      VMC_CASE(11)
      VMC_CASE(12)
#undef VMC_CASE
      default:
        break;
    }
  }
  if (cur >= 0) batch_flush<NGMAX, NACC>(B, cur, cur_d, hist, acc, cnt, red, FWD);
}

// Clears the work counter and, per integral, the forward sums (slots 0..7
// and the bins) and/or the gradient sums.
__global__ __launch_bounds__(kBlock) void k_batch_clear(double* bins, uint32_t nbins_total, double* scal,
                                                        uint32_t n, int fwd, int grad, uint32_t* counter) {
  const uint32_t tid = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t stride = gridDim.x * kBlock;
  if (fwd)
    for (uint32_t i = tid; i < nbins_total; i += stride) bins[i] = 0.0;
  const uint32_t nf = fwd ? 8u : 0u, ng = grad ? 5u * (kDmax + 1) : 0u;
  const uint32_t per = nf + ng;
  for (uint32_t i = tid; i < n * per; i += stride) {
    const uint32_t k = i / per, r = i - k * per;
    const uint32_t slot = r < nf ? r : S_GRAD + (r - nf);
    scal[static_cast<size_t>(k) * S_LEN + slot] = 0.0;
  }
  if (tid == 0) *counter = 0u;
}

__global__ void k_batch_combine_reset(double* scal, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t per = S_NTOTAL - S_W + 1;
  if (i >= n * per) return;
  const uint32_t k = i / per;
  scal[static_cast<size_t>(k) * S_LEN + S_W + (i - k * per)] = 0.0;
}

__global__ void k_batch_finalize(const BatchDesc* desc, double* scal, uint32_t n, int fwd, int grad) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const BatchDesc ds = desc[k];
  finalize_one(scal + ds.off_scal, 0, static_cast<double>(ds.ncall), 0.0, 0.0, fwd, grad ? ds.d + 1 : 0);
}

__global__ __launch_bounds__(kBlock) void k_batch_refine(const BatchDesc* desc, const AxisRef* axes, double* edges,
                                                         float* table, const double* bins, int N, double alpha) {
  const AxisRef ar = axes[blockIdx.x];
  const BatchDesc ds = desc[ar.k];
  refine_axis(edges + ds.off_edges + static_cast<size_t>(ar.a) * (N + 1),
              table + ds.off_table + static_cast<size_t>(2) * ar.a * N,
              bins + ds.off_bins + static_cast<size_t>(ds.d + ar.a) * N, N, alpha);
}

__global__ __launch_bounds__(kBlock) void k_batch_reset(const BatchDesc* desc, uint32_t n, double* edges,
                                                        float* table, double* bins, double* scal, int N) {
  const BatchDesc ds = desc[blockIdx.x];
  const int d = static_cast<int>(ds.d);
  for (int i = threadIdx.x; i < d * (N + 1); i += kBlock)
    edges[ds.off_edges + i] = static_cast<double>(i % (N + 1)) / static_cast<double>(N);
  for (int i = threadIdx.x; i < d * N; i += kBlock) {
    const int j = i % N;
    const double lo = static_cast<double>(j) / N, hi = static_cast<double>(j + 1) / N;
    table[ds.off_table + 2 * i] = static_cast<float>(lo);
    table[ds.off_table + 2 * i + 1] = static_cast<float>((hi - lo) * kWidthScale);
  }
  for (int i = threadIdx.x; i < 2 * d * N; i += kBlock) bins[ds.off_bins + i] = 0.0;
  for (int i = threadIdx.x; i < S_LEN; i += kBlock) scal[ds.off_scal + i] = 0.0;
}

}  // namespace

#define fail vmc::set_error

struct vmc_batch_s {
  int n = 0, N = 0, integrand = 0;
  std::vector<BatchDesc> desc;
  std::vector<AxisRef> axes;
  std::vector<BatchTile> tiles;
  size_t sz[6] = {};
  double* edges = nullptr;
  float* table = nullptr;
  double* bins = nullptr;
  double* scal = nullptr;
  const double* theta = nullptr;
  unsigned char* meta = nullptr;
  size_t meta_cap = 0;  // bytes of the bound meta buffer
  int spt = 0, blocks = 0;
  bool dirty = true;  // device copy of the work list is stale
  size_t meta_used = 0;
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t events_used = 0;
  // grid-state version (bind, reset, refine) and the one of the last
  // forward pass: an adjoint-only pass needs the two to agree
  uint64_t version = 1;
  uint64_t fwd_version = 0;
  ~vmc_batch_s() {
    for (auto& e : events) {
      hipEventDestroy(e.first);
      hipEventDestroy(e.second);
    }
  }
  // byte offsets inside meta
  size_t off_desc() const { return 256; }
  size_t off_axes() const { return off_desc() + ((sizeof(BatchDesc) * n + 255) / 256) * 256; }
  size_t off_tiles() const { return off_axes() + ((sizeof(AxisRef) * axes.size() + 255) / 256) * 256; }
  uint64_t total_calls() const {
    uint64_t t = 0;
    for (auto& d : desc) t += d.ncall;
    return t;
  }
  int effective_spt() const {
    if (spt) return spt;
    return 16;
  }
  int effective_blocks() const { return blocks ? blocks : 1024; }
  void build_tiles() {
    tiles.clear();
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return desc[a].ncall * desc[a].d > desc[b].ncall * desc[b].d;
    });
    const uint64_t tile = static_cast<uint64_t>(kBlock) * effective_spt();
    for (int k : order) {
      for (uint64_t s0 = 0; s0 < desc[k].ncall; s0 += tile) {
        const uint64_t s1 = std::min<uint64_t>(s0 + tile, desc[k].ncall);
        tiles.push_back(BatchTile{static_cast<uint32_t>(k), static_cast<uint32_t>(s0), static_cast<uint32_t>(s1), 0});
      }
    }
    dirty = true;
  }
};

namespace {

int hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(VMC_E_HIP, "%s: %s", what, hipGetErrorString(e));
  return VMC_OK;
}

#define HIP_TRY(expr, what)              \
  do {                                   \
    int rc__ = hip_ok((expr), (what));   \
    if (rc__ != VMC_OK) return rc__;     \
  } while (0)

int need_bound(vmc_batch_t b) {
  if (!b) return fail(VMC_E_INVALID, "batch handle is NULL");
  if (!b->edges || !b->table || !b->bins || !b->scal || !b->theta || !b->meta)
    return fail(VMC_E_UNBOUND, "batch buffers not bound (vmc_batch_bind)");
  return VMC_OK;
}

size_t meta_bytes(const vmc_batch_s* b, size_t ntiles) {
  return b->off_tiles() + sizeof(BatchTile) * ntiles;
}

// Copy descriptors, axis list and tiles to the device (waits for the copy:
// the host vectors may change right after).
int upload(vmc_batch_t b, hipStream_t st) {
  if (!b->dirty) return VMC_OK;
  const size_t need = meta_bytes(b, b->tiles.size());
  if (need > b->meta_cap)
    return fail(VMC_E_SCHEDULE, "work list needs %zu bytes of meta buffer, %zu bound (query the sizes after "
                "vmc_batch_set_schedule)", need, b->meta_cap);
  std::vector<unsigned char> host(need, 0);
  std::memcpy(host.data() + b->off_desc(), b->desc.data(), sizeof(BatchDesc) * b->n);
  std::memcpy(host.data() + b->off_axes(), b->axes.data(), sizeof(AxisRef) * b->axes.size());
  std::memcpy(host.data() + b->off_tiles(), b->tiles.data(), sizeof(BatchTile) * b->tiles.size());
  HIP_TRY(hipMemcpyAsync(b->meta, host.data(), need, hipMemcpyHostToDevice, st), "batch meta H2D");
  HIP_TRY(hipStreamSynchronize(st), "stream synchronize");
  b->dirty = false;
  return VMC_OK;
}

template <int KIND>
const void* batched_kernel(bool fp64) {
  return fp64 ? reinterpret_cast<const void*>(&k_batched<double, KIND>)
              : reinterpret_cast<const void*>(&k_batched<float, KIND>);
}

}  // namespace

extern "C" {

int vmc_batch_create(int n, const int* dims, int nbins, int integrand, const int64_t* ncall, vmc_batch_t* out) {
  if (!out || !dims || !ncall) return fail(VMC_E_INVALID, "NULL argument");
  if (n < 1 || n > 65536) return fail(VMC_E_INVALID, "batch size %d outside [1, 65536]", n);
  if (integrand != VMC_GAUSS_AXES)
    return fail(VMC_E_INTEGRAND, "the batched launch is built for VMC_GAUSS_AXES only (got %d)", integrand);
  if (nbins < 2 || nbins > 256) return fail(VMC_E_NBINS, "nbins %d outside [2,256]", nbins);
  auto* b = new vmc_batch_s;
  b->n = n;
  b->N = nbins;
  b->integrand = integrand;
  b->desc.resize(n);
  uint64_t oe = 0, ot = 0, ob = 0, oth = 0;
  for (int k = 0; k < n; ++k) {
    if (dims[k] < 1 || dims[k] > kDmax) {
      delete b;
      return fail(VMC_E_DIM, "integral %d: dim %d outside [1,%d]", k, dims[k], kDmax);
    }
    if (ncall[k] < 2 || ncall[k] > 4294967295LL) {
      delete b;
      return fail(VMC_E_NCALLS, "integral %d: ncall %lld outside [2, 2^32)", k, (long long)ncall[k]);
    }
    BatchDesc& d = b->desc[k];
    d.ncall = static_cast<uint64_t>(ncall[k]);
    d.d = static_cast<uint32_t>(dims[k]);
    d.kid = static_cast<uint32_t>(k);
    d.off_edges = static_cast<uint32_t>(oe);
    d.off_table = static_cast<uint32_t>(ot);
    d.off_bins = static_cast<uint32_t>(ob);
    d.off_theta = static_cast<uint32_t>(oth);
    d.off_scal = static_cast<uint32_t>(static_cast<uint64_t>(k) * S_LEN);
    oe += static_cast<uint64_t>(dims[k]) * (nbins + 1);
    ot += static_cast<uint64_t>(dims[k]) * nbins * 2;
    ob += static_cast<uint64_t>(dims[k]) * nbins * 2;
    oth += dims[k] + 1;
    for (int a = 0; a < dims[k]; ++a) b->axes.push_back(AxisRef{static_cast<uint32_t>(k), static_cast<uint32_t>(a)});
  }
  b->sz[0] = sizeof(double) * oe;
  b->sz[1] = sizeof(float) * ot;
  b->sz[2] = sizeof(double) * ob;
  b->sz[3] = sizeof(double) * S_LEN * static_cast<size_t>(n);
  b->sz[4] = sizeof(double) * oth;
  b->build_tiles();
  b->sz[5] = meta_bytes(b, b->tiles.size());
  *out = b;
  return VMC_OK;
}

int vmc_batch_destroy(vmc_batch_t b) {
  delete b;
  return VMC_OK;
}

int vmc_batch_workspace_sizes(vmc_batch_t b, size_t out[6]) {
  if (!b || !out) return fail(VMC_E_INVALID, "NULL argument");
  b->sz[5] = meta_bytes(b, b->tiles.size());
  for (int i = 0; i < 6; ++i) out[i] = b->sz[i];
  return VMC_OK;
}

int vmc_batch_bind(vmc_batch_t b, double* edges, float* table, double* bins, double* scal, const double* theta,
                   void* meta, size_t meta_bytes_bound) {
  if (!b) return fail(VMC_E_INVALID, "batch handle is NULL");
  if (!edges || !table || !bins || !scal || !theta || !meta) return fail(VMC_E_INVALID, "a device buffer is NULL");
  b->edges = edges;
  b->table = table;
  b->bins = bins;
  b->scal = scal;
  b->theta = theta;
  b->meta = static_cast<unsigned char*>(meta);
  b->meta_cap = meta_bytes_bound;
  b->dirty = true;
  ++b->version;
  return VMC_OK;
}

int vmc_batch_set_schedule(vmc_batch_t b, int samples_per_thread, int blocks) {
  if (!b) return fail(VMC_E_INVALID, "batch handle is NULL");
  if (samples_per_thread < 0 || samples_per_thread > 4096)
    return fail(VMC_E_SCHEDULE, "samples_per_thread %d outside [0, 4096]", samples_per_thread);
  if (blocks < 0 || blocks > 65536) return fail(VMC_E_SCHEDULE, "blocks %d outside [0, 65536]", blocks);
  b->spt = samples_per_thread;
  b->blocks = blocks;
  b->build_tiles();
  return VMC_OK;
}

int vmc_batch_reset(vmc_batch_t b, void* stream) {
  int rc = need_bound(b);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = upload(b, st);
  if (rc) return rc;
  const BatchDesc* d = reinterpret_cast<const BatchDesc*>(b->meta + b->off_desc());
  hipLaunchKernelGGL(k_batch_reset, dim3(b->n), dim3(kBlock), 0, st, d, static_cast<uint32_t>(b->n), b->edges,
                     b->table, b->bins, b->scal, b->N);
  ++b->version;
  HIP_TRY(hipGetLastError(), "k_batch_reset launch");
  return VMC_OK;
}

int vmc_iterate_batched(vmc_batch_t b, uint64_t seed, uint32_t it, int kind, uint32_t flags, void* stream) {
  int rc = need_bound(b);
  if (rc) return rc;
  if (kind < 1 || kind > 3) return fail(VMC_E_INVALID, "kind %d: 1 forward, 2 adjoint, 3 both", kind);
  if (kind == KIND_ADJ && b->fwd_version != b->version)
    return fail(VMC_E_GRID, "no forward pass on the grids' present state (reset or refine since)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = upload(b, st);
  if (rc) return rc;
  const bool fp64 = flags & VMC_FLAG_FP64;
  const bool fwd = kind & KIND_FWD, grad = kind & KIND_ADJ;
  BatchArgs A{};
  A.desc = reinterpret_cast<const BatchDesc*>(b->meta + b->off_desc());
  A.tiles = reinterpret_cast<const BatchTile*>(b->meta + b->off_tiles());
  A.counter = reinterpret_cast<uint32_t*>(b->meta);
  A.edges = b->edges;
  A.table = b->table;
  A.bins = b->bins;
  A.scal = b->scal;
  A.theta = b->theta;
  A.key = Key{static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)};
  A.it = it;
  A.ntiles = static_cast<uint32_t>(b->tiles.size());
  A.nbins = static_cast<uint32_t>(b->N);
  const uint32_t nb_total = static_cast<uint32_t>(b->sz[2] / sizeof(double));
  hipLaunchKernelGGL(k_batch_clear, dim3(std::max<uint32_t>(1, std::min<uint32_t>(1024, (nb_total + kBlock - 1) / kBlock))),
                     dim3(kBlock), 0, st, b->bins, nb_total, b->scal, static_cast<uint32_t>(b->n), fwd ? 1 : 0,
                     grad ? 1 : 0, A.counter);
  HIP_TRY(hipGetLastError(), "k_batch_clear launch");
  const void* fn = kind == KIND_FWD ? batched_kernel<KIND_FWD>(fp64)
                   : kind == KIND_ADJ ? batched_kernel<KIND_ADJ>(fp64)
                                      : batched_kernel<KIND_FUSED>(fp64);
  const size_t tab_bytes = (fp64 ? sizeof(double2) : sizeof(float2)) * kDmax * b->N;
  const size_t lds = tab_bytes + (fwd ? sizeof(double) * 2 * kDmax * b->N : 0);
  if (lds > 65536) {
    HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)),
            "LDS size attribute");
  }
  const int grid = std::min<int>(b->effective_blocks(), static_cast<int>(b->tiles.size()));
  void* args[] = {&A};
  std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
  if (b->timing) {
    if (b->events_used == b->events.size()) {
      std::pair<hipEvent_t, hipEvent_t> e;
      HIP_TRY(hipEventCreate(&e.first), "hipEventCreate");
      HIP_TRY(hipEventCreate(&e.second), "hipEventCreate");
      b->events.push_back(e);
    }
    ev = &b->events[b->events_used++];
    HIP_TRY(hipEventRecord(ev->first, st), "hipEventRecord");
  }
  HIP_TRY(hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, lds, st), "batched kernel launch");
  if (ev) HIP_TRY(hipEventRecord(ev->second, st), "hipEventRecord");
  hipLaunchKernelGGL(k_batch_finalize, dim3((b->n + 63) / 64), dim3(64), 0, st, A.desc, b->scal,
                     static_cast<uint32_t>(b->n), fwd ? 1 : 0, grad ? 1 : 0);
  HIP_TRY(hipGetLastError(), "k_batch_finalize launch");
  if (fwd) b->fwd_version = b->version;
  return VMC_OK;
}

int vmc_refine_batched(vmc_batch_t b, double alpha, void* stream) {
  int rc = need_bound(b);
  if (rc) return rc;
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(VMC_E_INVALID, "alpha %g must be finite and >= 0", alpha);
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = upload(b, st);
  if (rc) return rc;
  const BatchDesc* d = reinterpret_cast<const BatchDesc*>(b->meta + b->off_desc());
  const AxisRef* ax = reinterpret_cast<const AxisRef*>(b->meta + b->off_axes());
  hipLaunchKernelGGL(k_batch_refine, dim3(static_cast<unsigned>(b->axes.size())), dim3(kBlock), 0, st, d, ax, b->edges,
                     b->table, b->bins, b->N, alpha);
  ++b->version;
  HIP_TRY(hipGetLastError(), "k_batch_refine launch");
  return VMC_OK;
}

int vmc_batch_set_edges(vmc_batch_t b, int k, const double* host_edges, void* stream) {
  int rc = need_bound(b);
  if (rc) return rc;
  if (k < 0 || k >= b->n) return fail(VMC_E_INVALID, "integral %d outside [0, %d)", k, b->n);
  if (!host_edges) return fail(VMC_E_INVALID, "host_edges is NULL");
  const BatchDesc& ds = b->desc[k];
  const int d = static_cast<int>(ds.d), N = b->N;
  for (int a = 0; a < d; ++a) {
    const double* e = host_edges + static_cast<size_t>(a) * (N + 1);
    if (e[0] != 0.0 || e[N] != 1.0)
      return fail(VMC_E_GRID, "integral %d axis %d: edges must run from 0 to 1 (got %g .. %g)", k, a, e[0], e[N]);
    for (int j = 0; j < N; ++j)
      if (!(e[j + 1] > e[j]))
        return fail(VMC_E_GRID, "integral %d axis %d: edges not strictly increasing at bin %d", k, a, j);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  ++b->version;
  HIP_TRY(hipMemcpyAsync(b->edges + ds.off_edges, host_edges, sizeof(double) * d * (N + 1), hipMemcpyHostToDevice, st),
          "edges H2D");
  hipLaunchKernelGGL(k_table, dim3((d * N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, b->edges + ds.off_edges,
                     b->table + ds.off_table, d, N);
  HIP_TRY(hipGetLastError(), "k_table launch");
  HIP_TRY(hipStreamSynchronize(st), "stream synchronize");
  return VMC_OK;
}

int vmc_batch_combine_reset(vmc_batch_t b, void* stream) {
  int rc = need_bound(b);
  if (rc) return rc;
  const uint32_t total = static_cast<uint32_t>(b->n) * (S_NTOTAL - S_W + 1);
  hipLaunchKernelGGL(k_batch_combine_reset, dim3((total + kBlock - 1) / kBlock), dim3(kBlock), 0,
                     static_cast<hipStream_t>(stream), b->scal, static_cast<uint32_t>(b->n));
  HIP_TRY(hipGetLastError(), "k_batch_combine_reset launch");
  return VMC_OK;
}

int vmc_batch_timing(vmc_batch_t b, int enable, double* total_ms, int64_t* launches) {
  if (!b) return fail(VMC_E_INVALID, "batch handle is NULL");
  double tot = 0.0;
  for (size_t i = 0; i < b->events_used; ++i) {
    HIP_TRY(hipEventSynchronize(b->events[i].second), "hipEventSynchronize");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, b->events[i].first, b->events[i].second), "hipEventElapsedTime");
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = static_cast<int64_t>(b->events_used);
  b->events_used = 0;
  b->timing = enable != 0;
  return VMC_OK;
}

}  // extern "C"
