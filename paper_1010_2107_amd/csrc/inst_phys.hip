// Physics-shaped integrand instantiations (filled in with the W + partons
// toy); until then no dimension is compiled.
#include "vmc_registry.hpp"

namespace vmc {
const KernelSet* lookup_phys_f32(int, int) { return nullptr; }
const KernelSet* lookup_phys_f64(int, int) { return nullptr; }
}  // namespace vmc
