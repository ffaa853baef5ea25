// Instantiations of the helicity-amplitude integrand u dbar -> W+(-> mu+ nu)
// + n gluons (VMC_WHEL) for n = 0, 1, 2 (dim 5, 8, 11), in FP32
// (production) and FP64 (round-off-level checks).
#include "vmc_registry.hpp"
#include "vmc_whel.hpp"

namespace vmc {

template <typename T>
static const KernelSet* whel(int d) {
  switch (d) {
    case 5: return kernel_set<WHel<T, 5>>();
    case 8: return kernel_set<WHel<T, 8>>();
    case 11: return kernel_set<WHel<T, 11>>();
    default: return nullptr;
  }
}

const KernelSet* lookup_whel_f32(int d) { return whel<float>(d); }
const KernelSet* lookup_whel_f64(int d) { return whel<double>(d); }

}  // namespace vmc
