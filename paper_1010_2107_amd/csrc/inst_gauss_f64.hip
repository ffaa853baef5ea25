// FP64 instantiations (map and integrand in double precision) of the
// Gaussian-family integrands, used to check the full pipeline against the
// double-precision reference at round-off level.
#include "vmc_gauss.hpp"
#include "vmc_registry.hpp"

namespace vmc {

#define VMC_DIMS(F, T)                   \
  switch (d) {                           \
    case 1: return kernel_set<F<T, 1>>(); \
    case 2: return kernel_set<F<T, 2>>(); \
    case 3: return kernel_set<F<T, 3>>(); \
    case 4: return kernel_set<F<T, 4>>(); \
    case 8: return kernel_set<F<T, 8>>(); \
    default: return nullptr;             \
  }

const KernelSet* lookup_gauss_f64(int id, int d) {
  switch (id) {
    case 0: VMC_DIMS(ConstF, double)
    case 1: VMC_DIMS(LinearF, double)
    case 2: VMC_DIMS(GaussF, double)
    case 3: VMC_DIMS(DGaussF, double)
    case 4:
      switch (d) {
        case 2: return kernel_set<GaussAxesF<double, 2>>();
        case 3: return kernel_set<GaussAxesF<double, 3>>();
        default: return nullptr;
      }
    default: return nullptr;
  }
}

}  // namespace vmc
