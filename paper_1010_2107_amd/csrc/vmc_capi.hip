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
#include <string>
#include <vector>

#include "vmc.h"
#include "vmc_error.hpp"
#include "vmc_registry.hpp"
#include "vmc_small.hpp"

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
  bool timing = false;  // record events around every sample-kernel launch
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t events_used = 0;
  bool bound() const { return edges && table && bins && scal; }
  ~vmc_grid_s() {
    for (auto& e : events) {
      hipEventDestroy(e.first);
      hipEventDestroy(e.second);
    }
  }
};

extern "C" {

const char* vmc_last_error(void) { return g_last_error.c_str(); }

int vmc_version(void) { return 100; }

int vmc_workspace_sizes(int dim, int nbins, size_t out[4]) {
  if (!out) return fail(VMC_E_INVALID, "out is NULL");
  if (dim < 1 || dim > 16) return fail(VMC_E_DIM, "dim %d outside [1,16]", dim);
  if (nbins < 2 || nbins > 256) return fail(VMC_E_NBINS, "nbins %d outside [2,256]", nbins);
  out[0] = sizeof(double) * static_cast<size_t>(dim) * (nbins + 1);
  out[1] = sizeof(float) * 2 * static_cast<size_t>(dim) * nbins;
  out[2] = sizeof(double) * 2 * static_cast<size_t>(dim) * nbins;
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
  hipLaunchKernelGGL(k_reset, dim3(16), dim3(kBlock), 0, static_cast<hipStream_t>(stream), g->edges, g->table,
                     g->bins, g->scal, g->d, g->N);
  HIP_TRY(hipGetLastError(), "k_reset launch");
  return VMC_OK;
}

int bases_stratify(vmc_grid_t g, int ng) {
  if (!g) return fail(VMC_E_INVALID, "grid handle is NULL");
  if (ng <= 1) {
    g->ng = 1;
    return VMC_OK;
  }
  double cubes = std::pow(static_cast<double>(ng), g->d);
  if (cubes > 1099511627776.0) return fail(VMC_E_STRAT, "ng^dim = %.3g exceeds 2^40", cubes);
  g->ng = ng;
  return VMC_OK;
}

int vmc_set_schedule(vmc_grid_t g, int block_samples, int chunks_per_cube) {
  if (!g) return fail(VMC_E_INVALID, "grid handle is NULL");
  if (block_samples != 0 && (block_samples < kBlock || block_samples > (1 << 24) || block_samples % kBlock))
    return fail(VMC_E_SCHEDULE, "block_samples %d: need 0 or a multiple of %d in [%d, 2^24]", block_samples,
                kBlock, kBlock);
  if (chunks_per_cube != 0 &&
      (chunks_per_cube < 1 || chunks_per_cube > 64 || (chunks_per_cube & (chunks_per_cube - 1))))
    return fail(VMC_E_SCHEDULE, "chunks_per_cube %d: need 0 or a power of two in [1, 64]", chunks_per_cube);
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
  uint64_t grid = 0;
  size_t lds = 0;
  int d = 0;
  double n_eff = 0;
};

int plan_launch(vmc_grid_t g, int integrand, const double* theta, int ntheta, int64_t ncall, uint64_t seed,
                uint32_t it, uint32_t flags, Plan& P) {
  int rc = need_bound(g);
  if (rc) return rc;
  if (integrand < VMC_CONST || integrand > VMC_PSVOL)
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
    // built-in: at least 1024 blocks, at most 8192 samples per block (many
    // short blocks even out the per-block variation of cut-dependent work
    // and the tail of the last wave of blocks)
    uint64_t b = g->block_items;
    if (!b) {
      b = (A.ncall + 1023) / 1024;
      b = ((b + kBlock - 1) / kBlock) * kBlock;
      b = std::min<uint64_t>(std::max<uint64_t>(b, kBlock), 8192);
    }
    A.block_items = b;
  } else {
    uint64_t M = 1;
    for (int a = 0; a < g->d; ++a) M *= static_cast<uint64_t>(g->ng);
    const uint64_t k = static_cast<uint64_t>(ncall) / M;
    if (k < 2)
      return fail(VMC_E_NCALLS, "ncall %lld gives %llu samples per cube for %llu cubes; need >= 2", (long long)ncall,
                  (unsigned long long)k, (unsigned long long)M);
    A.ng = static_cast<uint32_t>(g->ng);
    A.per_cube = (g->N % g->ng == 0) ? static_cast<uint32_t>(g->N / g->ng) : 0u;
    A.M = static_cast<uint32_t>(M);
    A.k = static_cast<uint32_t>(k);
    A.ncall = k * M;
    P.n_eff = static_cast<double>(k * M);
    // built-in: about 32 samples per lane, and about 512 blocks
    uint32_t G = static_cast<uint32_t>(g->chunks);
    if (!G) {
      uint64_t want = k / 32;
      G = 1;
      while (G < 64 && 2 * G <= want) G <<= 1;
    }
    uint32_t lg = 0;
    while ((1u << lg) < G) ++lg;
    A.log2G = lg;
    P.items = M << lg;
    uint64_t b = g->block_items;
    if (!b) {
      b = (P.items + 511) / 512;
      b = ((b + kBlock - 1) / kBlock) * kBlock;
      if (b < kBlock) b = kBlock;
    }
    A.block_items = b;
  }
  P.grid = (P.items + A.block_items - 1) / A.block_items;
  if (P.grid > 0x7fffffffULL) return fail(VMC_E_SCHEDULE, "grid of %llu blocks too large", (unsigned long long)P.grid);
  P.d = g->d;
  P.lds = static_cast<size_t>(P.ks->tab_entry_bytes) * g->d * g->N;
  return VMC_OK;
}

int launch_sample(vmc_grid_t g, const Plan& P, int kind, hipStream_t stream) {
  const void* fn = P.strat ? P.ks->strat[kind] : P.ks->plain[kind];
  if (!fn) return fail(VMC_E_INTEGRAND, "integrand has no parameters to differentiate");
  size_t lds = P.lds;
  if (kind & KIND_FWD) lds += sizeof(double) * 2 * static_cast<size_t>(P.d) * P.A.nbins;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return fail(VMC_E_NBINS, "dim x nbins needs %zu bytes of LDS per block: %s", lds,
                                     hipGetErrorString(e));
  }
  SampleArgs A = P.A;
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
  HIP_TRY(hipLaunchKernel(fn, dim3(static_cast<unsigned>(P.grid)), dim3(kBlock), args, lds, stream),
          "sample kernel launch");
  if (ev) HIP_TRY(hipEventRecord(ev->second, stream), "hipEventRecord");
  return VMC_OK;
}

}  // namespace

extern "C" {

int vmc_iterate(vmc_grid_t g, int integrand, const double* theta, int ntheta, int64_t ncall, uint64_t seed,
                uint32_t it, uint32_t flags, void* stream) {
  Plan P;
  int rc = plan_launch(g, integrand, theta, ntheta, ncall, seed, it, flags, P);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nb = 2 * g->d * g->N;
  hipLaunchKernelGGL(k_clear, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, st, g->bins, nb, g->scal, 0,
                     S_NZERO + 1);
  HIP_TRY(hipGetLastError(), "k_clear launch");
  rc = launch_sample(g, P, KIND_FWD, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, g->scal, P.strat ? 1 : 0, P.n_eff,
                     static_cast<double>(P.A.k), static_cast<double>(P.A.M), 1, 0);
  HIP_TRY(hipGetLastError(), "k_finalize launch");
  return VMC_OK;
}

int vmc_iterate_adjoint(vmc_grid_t g, int integrand, const double* theta, int ntheta, int64_t ncall,
                        uint64_t seed, uint32_t it, uint32_t flags, void* stream) {
  Plan P;
  int rc = plan_launch(g, integrand, theta, ntheta, ncall, seed, it, flags, P);
  if (rc) return rc;
  if (P.ks->ngrad <= 0) return fail(VMC_E_INTEGRAND, "integrand %d has no parameters to differentiate", integrand);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_clear, dim3(1), dim3(kBlock), 0, st, g->bins, 0, g->scal, S_GRAD,
                     S_GRAD + 5 * P.ks->ngrad);
  HIP_TRY(hipGetLastError(), "k_clear launch");
  rc = launch_sample(g, P, KIND_ADJ, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, g->scal, P.strat ? 1 : 0, P.n_eff,
                     static_cast<double>(P.A.k), static_cast<double>(P.A.M), 0, P.ks->ngrad);
  HIP_TRY(hipGetLastError(), "k_finalize launch");
  return VMC_OK;
}

int vmc_iterate_fused(vmc_grid_t g, int integrand, const double* theta, int ntheta, int64_t ncall, uint64_t seed,
                      uint32_t it, uint32_t flags, void* stream) {
  Plan P;
  int rc = plan_launch(g, integrand, theta, ntheta, ncall, seed, it, flags, P);
  if (rc) return rc;
  if (P.ks->ngrad <= 0) return fail(VMC_E_INTEGRAND, "integrand %d has no parameters to differentiate", integrand);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nb = 2 * g->d * g->N;
  hipLaunchKernelGGL(k_clear, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, st, g->bins, nb, g->scal, 0,
                     S_NZERO + 1);
  HIP_TRY(hipGetLastError(), "k_clear launch");
  hipLaunchKernelGGL(k_clear, dim3(1), dim3(kBlock), 0, st, g->bins, 0, g->scal, S_GRAD,
                     S_GRAD + 5 * P.ks->ngrad);
  HIP_TRY(hipGetLastError(), "k_clear launch");
  rc = launch_sample(g, P, KIND_FUSED, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, g->scal, P.strat ? 1 : 0, P.n_eff,
                     static_cast<double>(P.A.k), static_cast<double>(P.A.M), 1, P.ks->ngrad);
  HIP_TRY(hipGetLastError(), "k_finalize launch");
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
  HIP_TRY(hipMemcpyAsync(g->edges, host_edges, sizeof(double) * g->d * (g->N + 1), hipMemcpyHostToDevice, st),
          "edges H2D");
  const int n = g->d * g->N;
  hipLaunchKernelGGL(k_table, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, g->edges, g->table, g->d, g->N);
  HIP_TRY(hipGetLastError(), "k_table launch");
  HIP_TRY(hipStreamSynchronize(st), "stream synchronize");
  return VMC_OK;
}

int vmc_dump_samples(vmc_grid_t g, int integrand, const double* theta, int ntheta, int64_t ncall, uint64_t seed,
                     uint32_t it, uint32_t flags, int64_t s0, int64_t count, uint32_t* words, void* w, void* f,
                     void* jac, void* stream) {
  Plan P;
  int rc = plan_launch(g, integrand, theta, ntheta, ncall, seed, it, flags, P);
  if (rc) return rc;
  if (s0 < 0 || count < 0 || static_cast<uint64_t>(s0 + count) > P.A.ncall)
    return fail(VMC_E_INVALID, "sample range [%lld, %lld) outside [0, %llu)", (long long)s0, (long long)(s0 + count),
                (unsigned long long)P.A.ncall);
  if (count == 0) return VMC_OK;
  DumpArgs D{};
  D.A = P.A;
  D.s0 = static_cast<uint64_t>(s0);
  D.count = static_cast<uint64_t>(count);
  D.words = words;
  D.w = w;
  D.f = f;
  D.jac = jac;
  void* args[] = {&D};
  const uint64_t grid = (D.count + kBlock - 1) / kBlock;
  HIP_TRY(hipLaunchKernel(P.ks->dump, dim3(static_cast<unsigned>(grid)), dim3(kBlock), args, P.lds,
                          static_cast<hipStream_t>(stream)),
          "dump kernel launch");
  return VMC_OK;
}

}  // extern "C"
