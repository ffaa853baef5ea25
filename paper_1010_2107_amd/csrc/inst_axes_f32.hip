// FP32 instantiations of the per-axis Gaussian product (the batched
// configuration draws its dimensions from 2..12).
#include "vmc_gauss.hpp"
#include "vmc_registry.hpp"

namespace vmc {

const KernelSet* lookup_axes_f32(int id, int d) {
  if (id != 4) return nullptr;
  switch (d) {
    case 1: return kernel_set<GaussAxesF<float, 1>>();
    case 2: return kernel_set<GaussAxesF<float, 2>>();
    case 3: return kernel_set<GaussAxesF<float, 3>>();
    case 4: return kernel_set<GaussAxesF<float, 4>>();
    case 5: return kernel_set<GaussAxesF<float, 5>>();
    case 6: return kernel_set<GaussAxesF<float, 6>>();
    case 7: return kernel_set<GaussAxesF<float, 7>>();
    case 8: return kernel_set<GaussAxesF<float, 8>>();
    case 9: return kernel_set<GaussAxesF<float, 9>>();
    case 10: return kernel_set<GaussAxesF<float, 10>>();
    case 11: return kernel_set<GaussAxesF<float, 11>>();
    case 12: return kernel_set<GaussAxesF<float, 12>>();
    default: return nullptr;
  }
}

}  // namespace vmc
