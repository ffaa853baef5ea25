"""MI355X (gfx950) VEGAS/BASES hot path of Kanzaki, "Monte Carlo integration
on GPU" (arXiv:1010.2107): HIP kernels behind the C ABI in include/vmc.h,
with this thin Python binding (ctypes + torch device memory and streams).

The HIP library is loaded on first use; if it is missing or cannot be
loaded every call raises VmcNotBuilt -- there is no CPU fallback.
"""
from ._lib import (CONST, DGAUSS, FLAG_FP64, GAUSS, GAUSS_AXES, LINEAR, PSVOL, WHEL, WJETS, VmcError,
                   VmcNotBuilt, header_functions, lib)

__all__ = ["CONST", "LINEAR", "GAUSS", "DGAUSS", "GAUSS_AXES", "WJETS", "PSVOL", "WHEL", "FLAG_FP64", "VmcError",
           "VmcNotBuilt", "lib", "header_functions", "Grid", "integrate", "GraphedLoop", "Batch", "autotune",
           "VegasIntegral", "vegas_integral", "Spring"]

# the rest of the surface, imported on first use (torch is loaded then)
_LAZY = {"Grid": "grid", "integrate": "driver", "GraphedLoop": "driver", "Batch": "batch", "autotune": "autotune",
         "VegasIntegral": "autograd", "vegas_integral": "autograd", "Spring": "spring"}


def __getattr__(name):
    mod = _LAZY.get(name)
    if mod is None:
        raise AttributeError(name)
    import importlib
    return getattr(importlib.import_module(f".{mod}", __name__), name)
