// vmc_registry.hpp -- lookup of the compiled integrand instantiations.
// Each instantiation unit compiles one family for a fixed list of
// dimensions and precisions; the C ABI asks here for the kernels of an
// (integrand, dim, precision) triple and gets NULL when it is not built.
#pragma once

#include "vmc_kernels.hpp"
#include "vmc_spring.hpp"

namespace vmc {

// Kernel entry points of one integrand instantiation.
struct KernelSet {
  const void* plain[4];  // indexed by KIND (1 fwd, 2 adj, 3 fused)
  const void* strat[8];  // and KIND_FWD | KIND_CMAX
  const void* dump;
  const void* dump_grad;  // the dump with per-sample gradients (NULL without parameters)
  const void* spring;
  int queue_bytes;        // LDS of the plain kernels' stage-2 queue (0: unstaged)
  int strat_queue_bytes;  // LDS of the stratified forward kernels' queue (0: unstaged); their slots come on top
  int ngrad;
  int ntheta;
  int tab_entry_bytes;
};

template <class F>
KernelSet make_kernel_set() {
  KernelSet s{};
  s.plain[KIND_FWD] = reinterpret_cast<const void*>(&k_plain<F, KIND_FWD>);
  s.strat[KIND_FWD] = reinterpret_cast<const void*>(&k_strat<F, KIND_FWD>);
  s.strat[KIND_FWD | KIND_CMAX] = reinterpret_cast<const void*>(&k_strat<F, KIND_FWD | KIND_CMAX>);
  if constexpr (F::NGRAD > 0) {
    s.plain[KIND_ADJ] = reinterpret_cast<const void*>(&k_plain<F, KIND_ADJ>);
    s.strat[KIND_ADJ] = reinterpret_cast<const void*>(&k_strat<F, KIND_ADJ>);
    s.plain[KIND_FUSED] = reinterpret_cast<const void*>(&k_plain<F, KIND_FUSED>);
    s.strat[KIND_FUSED] = reinterpret_cast<const void*>(&k_strat<F, KIND_FUSED>);
    s.dump_grad = reinterpret_cast<const void*>(&k_dump<F, true>);
  }
  s.dump = reinterpret_cast<const void*>(&k_dump<F, false>);
  s.spring = reinterpret_cast<const void*>(&k_spring<F>);
  s.queue_bytes = queue_bytes<F>();
  s.strat_queue_bytes = strat_queue_bytes<F>();
  s.ngrad = F::NGRAD;
  s.ntheta = F::NTHETA;
  s.tab_entry_bytes = static_cast<int>(sizeof(typename TabEntry<typename F::T>::type));
  return s;
}

const KernelSet* lookup_gauss_f32(int id, int d);
const KernelSet* lookup_axes_f32(int id, int d);
const KernelSet* lookup_gauss_f64(int id, int d);
const KernelSet* lookup_phys_f32(int id, int d);
const KernelSet* lookup_phys_f64(int id, int d);
const KernelSet* lookup_whel_f32(int d);
const KernelSet* lookup_whel_f64(int d);

inline const KernelSet* lookup_kernels(int id, int d, bool fp64) {
  if (id == 7) return fp64 ? lookup_whel_f64(d) : lookup_whel_f32(d);
  if (fp64) {
    if (id == 5 || id == 6) return lookup_phys_f64(id, d);
    return lookup_gauss_f64(id, d);
  }
  if (id == 4) return lookup_axes_f32(id, d);
  if (id == 5 || id == 6) return lookup_phys_f32(id, d);
  return lookup_gauss_f32(id, d);
}

// One static KernelSet per instantiation.
template <class F>
const KernelSet* kernel_set() {
  static const KernelSet s = make_kernel_set<F>();
  return &s;
}

}  // namespace vmc
