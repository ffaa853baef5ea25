// vmc_capi.hip -- the extern "C" boundary declared in include/vmc.h:
// argument validation, launch shapes, and the stream-ordered sequence of
// kernels that makes up one iteration (steps 2-5 of the six-step program
// structure of Kanzaki, arXiv:1010.2107, Sec. 3.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "vmc.h"
#include "vmc_error.hpp"
#include "vmc_registry.hpp"
#include "vmc_small.hpp"
#include "vmc_spring_setup.hpp"

using namespace vmc;

static thread_local std::string g_last_error;

namespace vmc {
int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}
}  // namespace vmc

#define fail vmc::set_error

static int hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(VMC_E_HIP, "%s: %s", what, hipGetErrorString(e));
  return VMC_OK;
}

#define HIP_TRY(expr, what)                       \
  do {                                            \
    int rc__ = hip_check((expr), (what));         \
    if (rc__ != VMC_OK) return rc__;              \
  } while (0)

struct vmc_grid_s {
  int d = 0, N = 0;
  int ng = 1;
  double* edges = nullptr;
  float* table = nullptr;
  double* bins = nullptr;
  double* scal = nullptr;
  int block_items = 0;  // 0: built-in
  int chunks = 0;       // 0: built-in
  // The partial-sum copies and the work counter behind the bin sums may be
  // non-zero (buffers bound and not reset yet): cleared before a pass.
  bool acc_dirty = true;
  // per-cube maxima of stratified forward passes (SPRING input), or NULL
  double* cube_max = nullptr;
  int64_t cube_max_n = 0;
  // buffers of the last successful spring_setup and the stratification they hold
  const uint64_t* sp_prefix = nullptr;
  const uint32_t* sp_guide = nullptr;
  const uint64_t* sp_state = nullptr;
  int sp_ng = 0;
  bool timing = false;  // record events around every sample-kernel launch
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t events_used = 0;
  // Grid-state version: advanced by every call that can change where the
  // samples land (bind, reset, stratify, refine, set_edges).  A forward pass
  // records it; an adjoint pass needs the version of the forward pass it
  // differentiates.
  uint64_t version = 1;
  uint64_t fwd_version = 0;  // 0: no forward pass on this state
  bool bound() const { return edges && table && bins && scal; }
  ~vmc_grid_s() {
    for (auto& e : events) {
      hipEventDestroy(e.first);
      hipEventDestroy(e.second);
    }
  }
};

// The bins buffer: the published [2][d][N] sums, then kStripes copies of
// the block partial sums (2 d N bins and kStripeScal scalars each, padded
// to 128 bytes).
static size_t stripe_len(int d, int N) { return (static_cast<size_t>(2) * d * N + kStripeScal + 15) / 16 * 16; }
static size_t bins_total(int d, int N) { return static_cast<size_t>(2) * d * N + kStripes * stripe_len(d, N); }

// The blocks' partial sums of vmc_iterate_static live in this array instead
// of the tail of the bound bins buffer: room for the largest grid (16 axes
// of 256 bins), 32 copies of 2 d N bins and the scalar slots, 2.02 MiB per
// GPU for the life of the process.  In host code `scratch` is only a
// handle: its device address comes from hipGetSymbolAddress, per device.
constexpr size_t kStaticScratch = static_cast<size_t>(kStripes) * ((2 * 16 * 256 + kStripeScal + 15) / 16 * 16);
static __device__ __align__(256) double scratch[kStaticScratch];

extern "C" {

const char* vmc_last_error(void) { return g_last_error.c_str(); }

int vmc_version(void) { return 300; }

int vmc_workspace_sizes(int dim, int nbins, size_t out[4]) {
  if (!out) return fail(VMC_E_INVALID, "out is NULL");
  if (dim < 1 || dim > 16) return fail(VMC_E_DIM, "dim %d outside [1,16]", dim);
  if (nbins < 2 || nbins > 256) return fail(VMC_E_NBINS, "nbins %d outside [2,256]", nbins);
  out[0] = sizeof(double) * static_cast<size_t>(dim) * (nbins + 1);
  out[1] = sizeof(float) * 2 * static_cast<size_t>(dim) * nbins;
  out[2] = sizeof(double) * bins_total(dim, nbins);
  out[3] = sizeof(double) * S_LEN;
  return VMC_OK;
}

int vmc_create(int dim, int nbins, vmc_grid_t* out) {
  size_t sz[4];
  if (!out) return fail(VMC_E_INVALID, "out is NULL");
  int rc = vmc_workspace_sizes(dim, nbins, sz);
  if (rc) return rc;
  vmc_grid_s* g = new vmc_grid_s;
  g->d = dim;
  g->N = nbins;
  *out = g;
  return VMC_OK;
}

int vmc_destroy(vmc_grid_t g) {
  delete g;
  return VMC_OK;
}

int vmc_bind(vmc_grid_t g, double* edges, float* table, double* bins, double* scal) {
  if (!g) return fail(VMC_E_INVALID, "grid handle is NULL");
  if (!edges || !table || !bins || !scal) return fail(VMC_E_INVALID, "a device buffer is NULL");
  g->edges = edges;
  g->table = table;
  g->bins = bins;
  g->scal = scal;
  g->acc_dirty = true;
  ++g->version;
  return VMC_OK;
}

static int need_bound(vmc_grid_t g) {
  if (!g) return fail(VMC_E_INVALID, "grid handle is NULL");
  if (!g->bound()) return fail(VMC_E_UNBOUND, "device buffers not bound (vmc_bind)");
  return VMC_OK;
}

int vmc_reset(vmc_grid_t g, void* stream) {
  int rc = need_bound(g);
  if (rc) return rc;
  // the published sums only: the private tail is cleared before the next
  // pass that uses it (vmc_iterate_static callers may bind just the sums)
  hipLaunchKernelGGL(k_reset, dim3(16), dim3(kBlock), 0, static_cast<hipStream_t>(stream), g->edges, g->table,
                     g->bins, 2 * g->d * g->N, g->scal, g->d, g->N);
  HIP_TRY(hipGetLastError(), "k_reset launch");
  g->acc_dirty = true;
  ++g->version;
  return VMC_OK;
}

int bases_stratify(vmc_grid_t g, int ng) {
  if (!g) return fail(VMC_E_INVALID, "grid handle is NULL");
  if (ng <= 1) {
    g->ng = 1;
    ++g->version;
    return VMC_OK;
  }
  double cubes = std::pow(static_cast<double>(ng), g->d);
  if (cubes > 1099511627776.0) return fail(VMC_E_STRAT, "ng^dim = %.3g exceeds 2^40", cubes);
  g->ng = ng;
  ++g->version;
  return VMC_OK;
}

int bases_cube_max(vmc_grid_t g, double* cube_max, int64_t ncubes) {
  if (!g) return fail(VMC_E_INVALID, "grid handle is NULL");
  if (cube_max && ncubes < 1) return fail(VMC_E_INVALID, "ncubes %lld < 1", (long long)ncubes);
  g->cube_max = cube_max;
  g->cube_max_n = cube_max ? ncubes : 0;
  return VMC_OK;
}

int vmc_set_schedule(vmc_grid_t g, int block_samples, int chunks_per_cube) {
  if (!g) return fail(VMC_E_INVALID, "grid handle is NULL");
  if (block_samples != 0 && (block_samples < kBlock || block_samples > (1 << 24) || block_samples % kBlock))
    return fail(VMC_E_SCHEDULE, "block_samples %d: need 0 or a multiple of %d in [%d, 2^24]", block_samples,
                kBlock, kBlock);
  if (chunks_per_cube != 0 &&
      (chunks_per_cube < 1 || chunks_per_cube > kBlock || (chunks_per_cube & (chunks_per_cube - 1))))
    return fail(VMC_E_SCHEDULE, "chunks_per_cube %d: need 0 or a power of two in [1, %d]", chunks_per_cube, kBlock);
  g->block_items = block_samples;
  g->chunks = chunks_per_cube;
  return VMC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Launch planning shared by iterate / adjoint / dump.
// ---------------------------------------------------------------------------
namespace {

struct Plan {
  const KernelSet* ks = nullptr;
  SampleArgs A{};
  bool strat = false;
  uint64_t items = 0;  // samples or cube units
  size_t lds = 0;
  int d = 0;
  double n_eff = 0;
};

int plan_launch(vmc_grid_t g, int integrand, const double* theta, int ntheta, int64_t ncall, uint64_t seed,
                uint32_t it, uint32_t flags, Plan& P) {
  int rc = need_bound(g);
  if (rc) return rc;
  if (integrand < VMC_CONST || integrand > VMC_WHEL)
    return fail(VMC_E_INTEGRAND, "unknown integrand id %d", integrand);
  const bool fp64 = flags & VMC_FLAG_FP64;
  P.ks = lookup_kernels(integrand, g->d, fp64);
  if (!P.ks)
    return fail(VMC_E_DIM, "integrand %d is not compiled for dim %d (%s)", integrand, g->d, fp64 ? "fp64" : "fp32");
  if (ntheta != P.ks->ntheta)
    return fail(VMC_E_PARAMS, "integrand %d in dim %d takes %d parameters, got %d", integrand, g->d, P.ks->ntheta,
                ntheta);
  if (ntheta > 0 && !theta) return fail(VMC_E_INVALID, "theta is NULL");
  if (ncall < 2 || ncall > 4294967296LL) return fail(VMC_E_NCALLS, "ncall %lld outside [2, 2^32]", (long long)ncall);
  SampleArgs& A = P.A;
  A.table32 = g->table;
  A.edges = g->edges;
  A.bins = g->bins;
  A.stripes = g->bins + static_cast<size_t>(2) * g->d * g->N;
  A.stripe_len = static_cast<uint32_t>(stripe_len(g->d, g->N));
  A.scal = g->scal;
  A.theta = theta;
  A.key = Key{static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)};
  A.it = it;
  A.kid = 0;
  A.nbins = static_cast<uint32_t>(g->N);
  P.strat = g->ng > 1;
  if (!P.strat) {
    A.ng = 1;
    A.ncall = static_cast<uint64_t>(ncall);
    P.items = A.ncall;
    P.n_eff = static_cast<double>(ncall);
    A.block_items = g->block_items;  // 0: chosen at launch
  } else {
    uint64_t M = 1;
    for (int a = 0; a < g->d; ++a) M *= static_cast<uint64_t>(g->ng);
    const uint64_t k = static_cast<uint64_t>(ncall) / M;
    if (k < 2)
      return fail(VMC_E_NCALLS, "ncall %lld gives %llu samples per cube for %llu cubes; need >= 2", (long long)ncall,
                  (unsigned long long)k, (unsigned long long)M);
    A.ng = static_cast<uint32_t>(g->ng);
    A.per_cube = (g->N % g->ng == 0) ? static_cast<uint32_t>(g->N / g->ng) : 0u;
    A.ngdiv = make_divu32(A.ng);
    A.ng_inv = 1.0 / static_cast<double>(A.ng);
    A.ng_wide = static_cast<uint64_t>(A.ng) * A.nbins >= (1ull << 32) ? 1u : 0u;
    A.M = static_cast<uint32_t>(M);
    A.k = static_cast<uint32_t>(k);
    A.ncall = k * M;
    P.n_eff = static_cast<double>(k * M);
    // built-in lanes per cube (at most one block per cube): first enough
    // cube units (M G, one per lane) to fill the chip (2^18), down to one or
    // two samples per unit; then, for the integrands that queue stage 2,
    // up to 2^19 units while units keep at least 8 samples
    uint32_t G = static_cast<uint32_t>(g->chunks);
    if (!G) {
      G = 1;
      while (G < kBlock && 2 * static_cast<uint64_t>(G) <= k && M * G < (1ull << 18)) G <<= 1;
      if (P.ks->strat_queue_bytes)
        while (G < kBlock && 16 * static_cast<uint64_t>(G) <= k && M * G < (1ull << 19)) G <<= 1;
    }
    uint32_t lg = 0;
    while ((1u << lg) < G) ++lg;
    A.log2G = lg;
    P.items = M << lg;
    A.block_items = g->block_items;  // 0: chosen at launch
  }
  P.d = g->d;
  P.lds = static_cast<size_t>(P.ks->tab_entry_bytes) * g->d * g->N;
  return VMC_OK;
}

// Blocks of one kernel that fit on the current device at once (cached per
// device, kernel and LDS size).
struct OccEntry {
  int dev;
  const void* fn;
  size_t lds;
  int blocks;
};
std::mutex g_occ_mu;
std::vector<OccEntry> g_occ;

int resident_blocks(const void* fn, size_t lds, int* out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  {
    std::lock_guard<std::mutex> lk(g_occ_mu);
    for (const auto& e : g_occ)
      if (e.dev == dev && e.fn == fn && e.lds == lds) {
        *out = e.blocks;
        return VMC_OK;
      }
  }
  int per_cu = 0, cus = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, lds), "occupancy query");
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count query");
  const int blocks = std::max(1, per_cu) * std::max(1, cus);
  std::lock_guard<std::mutex> lk(g_occ_mu);
  g_occ.push_back(OccEntry{dev, fn, lds, blocks});
  *out = blocks;
  return VMC_OK;
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and cleared there once; every pass's
// publish kernel leaves the copies it used at zero again.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(hipStream_t stream, double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(VMC_E_INVALID, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    const int n = static_cast<int>(kStaticScratch);
    hipLaunchKernelGGL(k_clear, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, static_cast<double*>(ptr),
                       n, nullptr, 0, 0);
    HIP_TRY(hipGetLastError(), "k_clear launch");
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return VMC_OK;
}

// One sample pass: blocks add their partial sums into kStripes copies; the
// publish kernel then adds the copies up and forms the estimate.  The
// copies are zero between passes (cleared here after a bind).  With
// static_copies the copies are the library's own device array, not the
// tail of the bound bins buffer.
int launch_sample(vmc_grid_t g, Plan& P, int kind, hipStream_t stream, bool static_copies = false) {
  if (static_copies) {
    if (static_cast<size_t>(kStripes) * P.A.stripe_len > kStaticScratch)
      return fail(VMC_E_NBINS, "dim x nbins needs %zu doubles of partial sums, the static array holds %zu",
                  static_cast<size_t>(kStripes) * P.A.stripe_len, kStaticScratch);
    int rc = static_scratch(stream, &P.A.stripes);
    if (rc) return rc;
  }
  const void* fn = P.strat ? P.ks->strat[kind] : P.ks->plain[kind];
  if (!fn) return fail(VMC_E_INTEGRAND, "integrand has no parameters to differentiate");
  size_t lds = P.lds;
  if (kind & KIND_FWD) lds += sizeof(double) * 2 * static_cast<size_t>(P.d) * P.A.nbins;
  if (!P.strat) {
    lds += static_cast<size_t>(P.ks->queue_bytes);
  } else if (P.ks->strat_queue_bytes) {
    const int ng = (kind & KIND_ADJ) ? P.ks->ngrad : 0;
    lds += static_cast<size_t>(P.ks->strat_queue_bytes) + static_cast<size_t>(strat_slot_bytes(P.A.log2G, ng));
  }
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return fail(VMC_E_NBINS, "dim x nbins needs %zu bytes of LDS per block: %s", lds,
                                     hipGetErrorString(e));
  }
  SampleArgs A = P.A;
  if (!A.block_items) {
    // built-in: one tile per block; plain: at least 1024 blocks, at most
    // 8192 samples per block (short blocks even out the cut-dependent cost
    // and the tail of the last wave); stratified: one cube unit per lane,
    // or two or four when units are short, toward 4096 samples per block
    // (8192 for the queued integrands, whose waves drain their queue at
    // every unit's end; the table load and the bin flush are per block),
    // but at least about 512 blocks
    uint64_t b = (P.items + 1023) / 1024;
    if (P.strat) {
      const double per_unit = static_cast<double>(A.k) / static_cast<double>(1u << A.log2G);
      const double toward = P.ks->strat_queue_bytes ? 8192.0 : 4096.0;
      uint64_t r = 1;
      while (r < 4 && 2.0 * static_cast<double>(r * kBlock) * per_unit <= toward) r <<= 1;
      b = std::min<uint64_t>(r * kBlock, (P.items + 511) / 512);
    }
    b = ((b + kBlock - 1) / kBlock) * kBlock;
    b = std::max<uint64_t>(b, kBlock);
    if (!P.strat) b = std::min<uint64_t>(b, 8192);
    if (!P.strat && P.ks->queue_bytes) {
      // queued integrands (cut-dependent cost per tile): at least two tiles
      // per block the device holds at once, so that the dispatcher can even
      // out slow tiles, but tiles of at least 1024 samples
      int resident = 0;
      int rc = resident_blocks(fn, lds, &resident);
      if (rc) return rc;
      const uint64_t want = 2 * static_cast<uint64_t>(resident);
      uint64_t br = (P.items + want - 1) / want;
      br = ((br + kBlock - 1) / kBlock) * kBlock;
      b = std::min<uint64_t>(b, std::max<uint64_t>(br, 1024));
    }
    A.block_items = b;
  }
  A.ntiles = (P.items + A.block_items - 1) / A.block_items;
  if (A.ntiles > 0x7fffffffULL) return fail(VMC_E_SCHEDULE, "%llu tiles: too many", (unsigned long long)A.ntiles);
  const uint64_t grid = A.ntiles;
  const int nb = 2 * g->d * g->N;
  if (g->acc_dirty && !static_copies) {
    const int n = static_cast<int>(bins_total(g->d, g->N)) - nb;
    hipLaunchKernelGGL(k_clear, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, P.A.stripes, n, g->scal,
                       0, 0);
    HIP_TRY(hipGetLastError(), "k_clear launch");
    g->acc_dirty = false;
  }
  void* args[] = {&A};
  std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
  if (g->timing) {
    if (g->events_used == g->events.size()) {
      std::pair<hipEvent_t, hipEvent_t> e;
      HIP_TRY(hipEventCreate(&e.first), "hipEventCreate");
      HIP_TRY(hipEventCreate(&e.second), "hipEventCreate");
      g->events.push_back(e);
    }
    ev = &g->events[g->events_used++];
    HIP_TRY(hipEventRecord(ev->first, stream), "hipEventRecord");
  }
  HIP_TRY(hipLaunchKernel(fn, dim3(static_cast<unsigned>(grid)), dim3(kBlock), args, lds, stream),
          "sample kernel launch");
  if (ev) HIP_TRY(hipEventRecord(ev->second, stream), "hipEventRecord");
  const int pub_blocks = std::max(1, (nb + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_publish, dim3(pub_blocks), dim3(kBlock), 0, stream, g->bins, P.A.stripes,
                     static_cast<int>(P.A.stripe_len), nb, g->scal, (kind & KIND_FWD) ? 1 : 0,
                     P.strat ? 1 : 0, (kind & KIND_ADJ) ? P.ks->ngrad : 0, P.n_eff, static_cast<double>(P.A.k),
                     static_cast<double>(P.A.M));
  HIP_TRY(hipGetLastError(), "k_publish launch");
  return VMC_OK;
}

}  // namespace

extern "C" {

int vmc_iterate(vmc_grid_t g, int integrand, const double* theta, int ntheta, int64_t ncall, uint64_t seed,
                uint32_t it, uint32_t flags, void* stream) {
  Plan P;
  int rc = plan_launch(g, integrand, theta, ntheta, ncall, seed, it, flags, P);
  if (rc) return rc;
  int kind = KIND_FWD;
  if (P.strat && g->cube_max) {
    if (static_cast<uint64_t>(g->cube_max_n) < P.A.M)
      return fail(VMC_E_INVALID, "cube-maximum buffer holds %lld cubes, the stratification has %u",
                  (long long)g->cube_max_n, P.A.M);
    P.A.cube_max = g->cube_max;
    kind |= KIND_CMAX;
  }
  rc = launch_sample(g, P, kind, static_cast<hipStream_t>(stream));
  if (rc == VMC_OK) g->fwd_version = g->version;
  return rc;
}

int vmc_iterate_static(vmc_grid_t g, int integrand, const double* theta, int ntheta, int64_t ncall, uint64_t seed,
                       uint32_t it, uint32_t flags, void* stream) {
  Plan P;
  int rc = plan_launch(g, integrand, theta, ntheta, ncall, seed, it, flags, P);
  if (rc) return rc;
  int kind = KIND_FWD;
  if (P.strat && g->cube_max) {
    if (static_cast<uint64_t>(g->cube_max_n) < P.A.M)
      return fail(VMC_E_INVALID, "cube-maximum buffer holds %lld cubes, the stratification has %u",
                  (long long)g->cube_max_n, P.A.M);
    P.A.cube_max = g->cube_max;
    kind |= KIND_CMAX;
  }
  rc = launch_sample(g, P, kind, static_cast<hipStream_t>(stream), true);
  if (rc == VMC_OK) g->fwd_version = g->version;
  return rc;
}

int vmc_iterate_adjoint(vmc_grid_t g, int integrand, const double* theta, int ntheta, int64_t ncall,
                        uint64_t seed, uint32_t it, uint32_t flags, void* stream) {
  Plan P;
  int rc = plan_launch(g, integrand, theta, ntheta, ncall, seed, it, flags, P);
  if (rc) return rc;
  if (P.ks->ngrad <= 0) return fail(VMC_E_INTEGRAND, "integrand %d has no parameters to differentiate", integrand);
  if (g->fwd_version != g->version)
    return fail(VMC_E_GRID, g->fwd_version == 0
                                ? "no forward pass on this grid state: run vmc_iterate first"
                                : "the grid changed (refine, set_edges, reset, stratify or bind) since the "
                                  "forward pass this adjoint pass would differentiate");
  return launch_sample(g, P, KIND_ADJ, static_cast<hipStream_t>(stream));
}

int vmc_iterate_fused(vmc_grid_t g, int integrand, const double* theta, int ntheta, int64_t ncall, uint64_t seed,
                      uint32_t it, uint32_t flags, void* stream) {
  Plan P;
  int rc = plan_launch(g, integrand, theta, ntheta, ncall, seed, it, flags, P);
  if (rc) return rc;
  if (P.ks->ngrad <= 0) return fail(VMC_E_INTEGRAND, "integrand %d has no parameters to differentiate", integrand);
  rc = launch_sample(g, P, KIND_FUSED, static_cast<hipStream_t>(stream));
  if (rc == VMC_OK) g->fwd_version = g->version;
  return rc;
}

int vmc_grid_version(vmc_grid_t g, uint64_t* version) {
  if (!g || !version) return fail(VMC_E_INVALID, "NULL argument");
  *version = g->version;
  return VMC_OK;
}

int vmc_integrand_info(int integrand, int dim, uint32_t flags, int* ntheta, int* ngrad) {
  if (integrand < VMC_CONST || integrand > VMC_WHEL) return fail(VMC_E_INTEGRAND, "unknown integrand id %d", integrand);
  const bool fp64 = flags & VMC_FLAG_FP64;
  const KernelSet* ks = lookup_kernels(integrand, dim, fp64);
  if (!ks)
    return fail(VMC_E_DIM, "integrand %d is not compiled for dim %d (%s)", integrand, dim, fp64 ? "fp64" : "fp32");
  if (ntheta) *ntheta = ks->ntheta;
  if (ngrad) *ngrad = ks->ngrad;
  return VMC_OK;
}

int vmc_timing(vmc_grid_t g, int enable, double* total_ms, int64_t* launches) {
  if (!g) return fail(VMC_E_INVALID, "grid handle is NULL");
  double tot = 0.0;
  for (size_t i = 0; i < g->events_used; ++i) {
    auto& e = g->events[i];
    HIP_TRY(hipEventSynchronize(e.second), "hipEventSynchronize");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second), "hipEventElapsedTime");
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = static_cast<int64_t>(g->events_used);
  g->events_used = 0;
  g->timing = enable != 0;
  return VMC_OK;
}

int vmc_refine(vmc_grid_t g, double alpha, void* stream) {
  int rc = need_bound(g);
  if (rc) return rc;
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(VMC_E_INVALID, "alpha %g must be finite and >= 0", alpha);
  hipLaunchKernelGGL(k_refine, dim3(g->d), dim3(kBlock), 0, static_cast<hipStream_t>(stream), g->edges, g->table,
                     g->bins, g->d, g->N, alpha);
  ++g->version;
  HIP_TRY(hipGetLastError(), "k_refine launch");
  return VMC_OK;
}

int vmc_combine_reset(vmc_grid_t g, void* stream) {
  int rc = need_bound(g);
  if (rc) return rc;
  hipLaunchKernelGGL(k_combine_reset, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), g->scal);
  HIP_TRY(hipGetLastError(), "k_combine_reset launch");
  return VMC_OK;
}

int vmc_get_edges(vmc_grid_t g, double* host_edges, void* stream) {
  int rc = need_bound(g);
  if (rc) return rc;
  if (!host_edges) return fail(VMC_E_INVALID, "host_edges is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(host_edges, g->edges, sizeof(double) * g->d * (g->N + 1), hipMemcpyDeviceToHost, st),
          "edges D2H");
  HIP_TRY(hipStreamSynchronize(st), "stream synchronize");
  return VMC_OK;
}

int vmc_set_edges(vmc_grid_t g, const double* host_edges, void* stream) {
  int rc = need_bound(g);
  if (rc) return rc;
  if (!host_edges) return fail(VMC_E_INVALID, "host_edges is NULL");
  for (int a = 0; a < g->d; ++a) {
    const double* e = host_edges + static_cast<size_t>(a) * (g->N + 1);
    if (e[0] != 0.0 || e[g->N] != 1.0)
      return fail(VMC_E_GRID, "axis %d: edges must run from 0 to 1 (got %g .. %g)", a, e[0], e[g->N]);
    for (int j = 0; j < g->N; ++j)
      if (!(e[j + 1] > e[j])) return fail(VMC_E_GRID, "axis %d: edges not strictly increasing at bin %d", a, j);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  ++g->version;
  HIP_TRY(hipMemcpyAsync(g->edges, host_edges, sizeof(double) * g->d * (g->N + 1), hipMemcpyHostToDevice, st),
          "edges H2D");
  const int n = g->d * g->N;
  hipLaunchKernelGGL(k_table, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, g->edges, g->table, g->d, g->N);
  HIP_TRY(hipGetLastError(), "k_table launch");
  HIP_TRY(hipStreamSynchronize(st), "stream synchronize");
  return VMC_OK;
}

int vmc_dump_samples(vmc_grid_t g, int integrand, const double* theta, int ntheta, int64_t ncall, uint64_t seed,
                     uint32_t it, uint32_t flags, int64_t s0, int64_t count, uint32_t* words, uint8_t* bins, void* w,
                     void* f, void* jac, void* grad, void* stream) {
  Plan P;
  int rc = plan_launch(g, integrand, theta, ntheta, ncall, seed, it, flags, P);
  if (rc) return rc;
  if (s0 < 0 || count < 0 || static_cast<uint64_t>(s0 + count) > P.A.ncall)
    return fail(VMC_E_INVALID, "sample range [%lld, %lld) outside [0, %llu)", (long long)s0, (long long)(s0 + count),
                (unsigned long long)P.A.ncall);
  if (grad && P.ks->ngrad <= 0)
    return fail(VMC_E_INTEGRAND, "integrand %d has no parameters to differentiate", integrand);
  if (count == 0) return VMC_OK;
  DumpArgs D{};
  D.A = P.A;
  D.s0 = static_cast<uint64_t>(s0);
  D.count = static_cast<uint64_t>(count);
  D.words = words;
  D.bins = bins;
  D.w = w;
  D.f = f;
  D.jac = jac;
  D.grad = grad;
  void* args[] = {&D};
  const uint64_t grid = (D.count + kBlock - 1) / kBlock;
  HIP_TRY(hipLaunchKernel(grad ? P.ks->dump_grad : P.ks->dump, dim3(static_cast<unsigned>(grid)), dim3(kBlock), args,
                          P.lds,
                          static_cast<hipStream_t>(stream)),
          "dump kernel launch");
  return VMC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// SPRING
// ---------------------------------------------------------------------------
namespace {

struct SpringShape {
  uint64_t M = 0, K = 0, nblk = 0;
  uint32_t kbits = 0;
};

int spring_shape(vmc_grid_t g, SpringShape& S) {
  if (!g) return fail(VMC_E_INVALID, "grid handle is NULL");
  if (g->ng <= 1) return fail(VMC_E_STRAT, "SPRING needs a stratified grid (bases_stratify with ng >= 2)");
  uint64_t M = 1;
  for (int a = 0; a < g->d; ++a) {
    M *= static_cast<uint64_t>(g->ng);
    if (M > (1ull << 28)) return fail(VMC_E_STRAT, "ng^dim exceeds 2^28 cubes for SPRING");
  }
  S.M = M;
  while ((1ull << S.kbits) < M) ++S.kbits;
  S.K = 1ull << S.kbits;
  S.nblk = (M + kScanChunk - 1) / kScanChunk;
  return VMC_OK;
}

}  // namespace

extern "C" {

int spring_workspace_sizes(vmc_grid_t g, size_t out[3]) {
  if (!out) return fail(VMC_E_INVALID, "out is NULL");
  SpringShape S;
  int rc = spring_shape(g, S);
  if (rc) return rc;
  out[0] = sizeof(uint64_t) * (S.M + 1);
  out[1] = sizeof(uint32_t) * (S.K + 1);
  out[2] = sizeof(uint64_t) * (SP_HDR + S.nblk);
  return VMC_OK;
}

int spring_setup(vmc_grid_t g, const double* cube_max, double headroom, uint64_t* prefix, uint32_t* guide,
                 uint64_t* state, void* stream) {
  SpringShape S;
  int rc = spring_shape(g, S);
  if (rc) return rc;
  if (!cube_max || !prefix || !guide || !state) return fail(VMC_E_INVALID, "a device buffer is NULL");
  if (!(headroom >= 1.0) || !std::isfinite(headroom))
    return fail(VMC_E_INVALID, "headroom %g must be finite and >= 1", headroom);
  g->sp_prefix = nullptr;
  g->sp_guide = nullptr;
  g->sp_state = nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned gblocks = static_cast<unsigned>(std::min<uint64_t>((S.M + kBlock - 1) / kBlock, 2048));
  hipLaunchKernelGGL(k_sp_init, dim3(1), dim3(64), 0, st, state, S.M, S.kbits);
  hipLaunchKernelGGL(k_sp_gmax, dim3(gblocks), dim3(kBlock), 0, st, cube_max, S.M, state);
  hipLaunchKernelGGL(k_sp_blocksum, dim3(static_cast<unsigned>(S.nblk)), dim3(kBlock), 0, st, cube_max, S.M, state);
  hipLaunchKernelGGL(k_sp_scan_blocks, dim3(1), dim3(kBlock), 0, st, state, S.nblk, headroom);
  hipLaunchKernelGGL(k_sp_scan, dim3(static_cast<unsigned>(S.nblk)), dim3(kBlock), 0, st, cube_max, S.M, state,
                     prefix);
  const unsigned kblocks = static_cast<unsigned>(std::min<uint64_t>((S.K + kBlock) / kBlock, 4096));
  hipLaunchKernelGGL(k_sp_guide, dim3(kblocks), dim3(kBlock), 0, st, prefix, S.M, state, guide);
  HIP_TRY(hipGetLastError(), "SPRING set-up launch");
  uint64_t hdr[SP_HDR];
  HIP_TRY(hipMemcpyAsync(hdr, state, sizeof hdr, hipMemcpyDeviceToHost, st), "SPRING state D2H");
  HIP_TRY(hipStreamSynchronize(st), "stream synchronize");
  if (hdr[SP_BADMAX]) return fail(VMC_E_SPRING, "%llu cube maxima are +Inf", (unsigned long long)hdr[SP_BADMAX]);
  if (hdr[SP_TOTAL] == 0) return fail(VMC_E_SPRING, "no cube has a positive finite maximum weight");
  g->sp_prefix = prefix;
  g->sp_guide = guide;
  g->sp_state = state;
  g->sp_ng = g->ng;
  return VMC_OK;
}

int spring_clear_counts(uint64_t* state, void* stream) {
  if (!state) return fail(VMC_E_INVALID, "state is NULL");
  hipLaunchKernelGGL(k_sp_clear_counts, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), state);
  HIP_TRY(hipGetLastError(), "k_sp_clear_counts launch");
  return VMC_OK;
}

int spring_generate(vmc_grid_t g, int integrand, const double* theta, int ntheta, const uint64_t* prefix,
                    const uint32_t* guide, uint64_t* state, uint64_t seed, uint32_t pass, int64_t trial0,
                    int64_t ntrials, int64_t max_events, void* events, uint64_t* event_trial, uint32_t flags,
                    void* stream) {
  int rc = need_bound(g);
  if (rc) return rc;
  SpringShape S;
  rc = spring_shape(g, S);
  if (rc) return rc;
  if (!prefix || prefix != g->sp_prefix || guide != g->sp_guide || state != g->sp_state || g->sp_ng != g->ng)
    return fail(VMC_E_SPRING, "these buffers have not been set up by spring_setup for this stratification");
  if (integrand < VMC_CONST || integrand > VMC_WHEL) return fail(VMC_E_INTEGRAND, "unknown integrand id %d", integrand);
  const bool fp64 = flags & VMC_FLAG_FP64;
  const KernelSet* ks = lookup_kernels(integrand, g->d, fp64);
  if (!ks)
    return fail(VMC_E_DIM, "integrand %d is not compiled for dim %d (%s)", integrand, g->d, fp64 ? "fp64" : "fp32");
  if (ntheta != ks->ntheta)
    return fail(VMC_E_PARAMS, "integrand %d in dim %d takes %d parameters, got %d", integrand, g->d, ks->ntheta,
                ntheta);
  if (ntheta > 0 && !theta) return fail(VMC_E_INVALID, "theta is NULL");
  if (trial0 < 0 || ntrials < 0 || ntrials > (1ll << 40) || trial0 > (1ll << 62))
    return fail(VMC_E_INVALID, "trials [%lld, +%lld): need trial0 in [0, 2^62] and ntrials in [0, 2^40]",
                (long long)trial0, (long long)ntrials);
  if (max_events < 0 || (max_events > 0 && !events))
    return fail(VMC_E_INVALID, "max_events %lld needs an event buffer", (long long)max_events);
  if (ntrials == 0) return VMC_OK;
  SpringArgs SP{};
  SampleArgs& A = SP.A;
  A.table32 = g->table;
  A.edges = g->edges;
  A.bins = g->bins;
  A.scal = g->scal;
  A.theta = theta;
  A.key = Key{static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)};
  A.it = pass;
  A.nbins = static_cast<uint32_t>(g->N);
  A.ng = static_cast<uint32_t>(g->ng);
  A.per_cube = (g->N % g->ng == 0) ? static_cast<uint32_t>(g->N / g->ng) : 0u;
  A.ngdiv = make_divu32(A.ng);
  A.ng_inv = 1.0 / static_cast<double>(A.ng);
  A.ng_wide = static_cast<uint64_t>(A.ng) * A.nbins >= (1ull << 32) ? 1u : 0u;
  A.M = static_cast<uint32_t>(S.M);
  SP.prefix = prefix;
  SP.guide = guide;
  SP.state = state;
  SP.trial0 = static_cast<uint64_t>(trial0);
  SP.ntrials = static_cast<uint64_t>(ntrials);
  SP.max_events = static_cast<uint64_t>(max_events);
  SP.events = events;
  SP.event_trial = event_trial;
  // grid table, then the staged points
  const size_t lds = static_cast<size_t>(ks->tab_entry_bytes) * g->d * g->N +
                     static_cast<size_t>(kStage) * g->d * (fp64 ? sizeof(double) : sizeof(float));
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(ks->spring, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return fail(VMC_E_NBINS, "dim x nbins needs %zu bytes of LDS per block: %s", lds,
                                     hipGetErrorString(e));
  }
  int resident = 0;
  rc = resident_blocks(ks->spring, lds, &resident);
  if (rc) return rc;
  const uint64_t grid = std::min<uint64_t>((SP.ntrials + kBlock - 1) / kBlock, static_cast<uint64_t>(resident));
  void* args[] = {&SP};
  HIP_TRY(hipLaunchKernel(ks->spring, dim3(static_cast<unsigned>(grid)), dim3(kBlock), args, lds,
                          static_cast<hipStream_t>(stream)),
          "SPRING kernel launch");
  return VMC_OK;
}

}  // extern "C"
