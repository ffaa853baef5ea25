// FP32 instantiations of the constant, linear, single- and double-Gaussian
// integrands for the dimensions the configurations and tests use.
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

const KernelSet* lookup_gauss_f32(int id, int d) {
  switch (id) {
    case 0: VMC_DIMS(ConstF, float)
    case 1: VMC_DIMS(LinearF, float)
    case 2: VMC_DIMS(GaussF, float)
    case 3: VMC_DIMS(DGaussF, float)
    default: return nullptr;
  }
}

}  // namespace vmc
