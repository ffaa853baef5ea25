// vmc_registry.hpp -- lookup of the compiled integrand instantiations.
// Each instantiation unit compiles one family for a fixed list of
// dimensions and precisions; the C ABI asks here for the kernels of an
// (integrand, dim, precision) triple and gets NULL when it is not built.
#pragma once

#include "vmc_kernels.hpp"

namespace vmc {

const KernelSet* lookup_gauss_f32(int id, int d);
const KernelSet* lookup_axes_f32(int id, int d);
const KernelSet* lookup_gauss_f64(int id, int d);
const KernelSet* lookup_phys_f32(int id, int d);
const KernelSet* lookup_phys_f64(int id, int d);

inline const KernelSet* lookup_kernels(int id, int d, bool fp64) {
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
