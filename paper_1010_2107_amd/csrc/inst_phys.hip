// Instantiations of the W + partons integrand (VMC_WJETS) and of its
// flux x phase-space part (VMC_PSVOL) for 1..4 partons (dim 7, 10, 13, 16),
// in FP32 (production) and FP64 (round-off-level checks).
#include "vmc_phys.hpp"
#include "vmc_registry.hpp"

namespace vmc {

template <typename T>
static const KernelSet* phys(int id, int d) {
  if (id == 5) {
    switch (d) {
      case 7: return kernel_set<WJets<T, 7>>();
      case 10: return kernel_set<WJets<T, 10>>();
      case 13: return kernel_set<WJets<T, 13>>();
      case 16: return kernel_set<WJets<T, 16>>();
      default: return nullptr;
    }
  }
  if (id == 6) {
    switch (d) {
      case 7: return kernel_set<PsVol<T, 7>>();
      case 10: return kernel_set<PsVol<T, 10>>();
      case 13: return kernel_set<PsVol<T, 13>>();
      case 16: return kernel_set<PsVol<T, 16>>();
      default: return nullptr;
    }
  }
  return nullptr;
}

const KernelSet* lookup_phys_f32(int id, int d) { return phys<float>(id, d); }
const KernelSet* lookup_phys_f64(int id, int d) { return phys<double>(id, d); }

}  // namespace vmc
