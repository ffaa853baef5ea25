"""ctypes loader for libvmc.so (the HIP library declared in include/vmc.h).

Argument marshalling only.  There is no fallback: if the library is missing
or cannot be loaded, every call raises VmcNotBuilt.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvmc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vmc.h")

# integrand ids and flags (include/vmc.h)
CONST, LINEAR, GAUSS, DGAUSS, GAUSS_AXES, WJETS, PSVOL, WHEL = range(8)
FLAG_FP64 = 1

S_S1, S_S2, S_V, S_NONFINITE, S_I, S_VAR, S_NEFF, S_NZERO = 0, 1, 2, 3, 4, 5, 6, 7
S_NITER, S_IBAR, S_SIGBAR, S_CHI2, S_GRAD, SCAL_LEN = 11, 14, 15, 16, 32, 128
SP_UNIT, SP_GMAX, SP_TOTAL, SP_ENV, SP_KBITS, SP_NCUBES = 0, 1, 2, 3, 4, 5
SP_TRIALS, SP_KEPT, SP_OVER, SP_SLOT = 8, 9, 10, 11

ERRORS = {
    -1: "VMC_E_INVALID", -2: "VMC_E_DIM", -3: "VMC_E_NBINS", -4: "VMC_E_NCALLS", -5: "VMC_E_INTEGRAND",
    -6: "VMC_E_PARAMS", -7: "VMC_E_STRAT", -8: "VMC_E_GRID", -9: "VMC_E_HIP", -10: "VMC_E_UNBOUND",
    -11: "VMC_E_SCHEDULE", -12: "VMC_E_SPRING",
}


class VmcNotBuilt(ImportError):
    pass


class VmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


_lib = None

_c = ctypes
_vp = _c.c_void_p
_SIGS = {
    "vmc_last_error": (_c.c_char_p, []),
    "vmc_version": (_c.c_int, []),
    "vmc_workspace_sizes": (_c.c_int, [_c.c_int, _c.c_int, _c.POINTER(_c.c_size_t)]),
    "vmc_create": (_c.c_int, [_c.c_int, _c.c_int, _c.POINTER(_vp)]),
    "vmc_destroy": (_c.c_int, [_vp]),
    "vmc_bind": (_c.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "vmc_reset": (_c.c_int, [_vp, _vp]),
    "bases_stratify": (_c.c_int, [_vp, _c.c_int]),
    "vmc_iterate": (_c.c_int, [_vp, _c.c_int, _vp, _c.c_int, _c.c_int64, _c.c_uint64, _c.c_uint32, _c.c_uint32, _vp]),
    "vmc_iterate_static": (_c.c_int, [_vp, _c.c_int, _vp, _c.c_int, _c.c_int64, _c.c_uint64, _c.c_uint32, _c.c_uint32,
                                      _vp]),
    "vmc_iterate_adjoint": (_c.c_int, [_vp, _c.c_int, _vp, _c.c_int, _c.c_int64, _c.c_uint64, _c.c_uint32,
                                       _c.c_uint32, _vp]),
    "vmc_iterate_fused": (_c.c_int, [_vp, _c.c_int, _vp, _c.c_int, _c.c_int64, _c.c_uint64, _c.c_uint32,
                                     _c.c_uint32, _vp]),
    "vmc_refine": (_c.c_int, [_vp, _c.c_double, _vp]),
    "vmc_combine_reset": (_c.c_int, [_vp, _vp]),
    "vmc_get_edges": (_c.c_int, [_vp, _vp, _vp]),
    "vmc_set_edges": (_c.c_int, [_vp, _vp, _vp]),
    "vmc_dump_samples": (_c.c_int, [_vp, _c.c_int, _vp, _c.c_int, _c.c_int64, _c.c_uint64, _c.c_uint32, _c.c_uint32,
                                    _c.c_int64, _c.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "vmc_grid_version": (_c.c_int, [_vp, _c.POINTER(_c.c_uint64)]),
    "vmc_integrand_info": (_c.c_int, [_c.c_int, _c.c_int, _c.c_uint32, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int)]),
    "vmc_set_schedule": (_c.c_int, [_vp, _c.c_int, _c.c_int]),
    "vmc_timing": (_c.c_int, [_vp, _c.c_int, _c.POINTER(_c.c_double), _c.POINTER(_c.c_int64)]),
    "vmc_batch_create": (_c.c_int, [_c.c_int, _c.POINTER(_c.c_int), _c.c_int, _c.c_int, _c.POINTER(_c.c_int64),
                                    _c.POINTER(_vp)]),
    "vmc_batch_destroy": (_c.c_int, [_vp]),
    "vmc_batch_workspace_sizes": (_c.c_int, [_vp, _c.POINTER(_c.c_size_t)]),
    "vmc_batch_bind": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _c.c_size_t]),
    "vmc_batch_set_schedule": (_c.c_int, [_vp, _c.c_int, _c.c_int]),
    "vmc_batch_reset": (_c.c_int, [_vp, _vp]),
    "vmc_iterate_batched": (_c.c_int, [_vp, _c.c_uint64, _c.c_uint32, _c.c_int, _c.c_uint32, _vp]),
    "vmc_refine_batched": (_c.c_int, [_vp, _c.c_double, _vp]),
    "vmc_batch_combine_reset": (_c.c_int, [_vp, _vp]),
    "vmc_batch_set_edges": (_c.c_int, [_vp, _c.c_int, _vp, _vp]),
    "vmc_batch_timing": (_c.c_int, [_vp, _c.c_int, _c.POINTER(_c.c_double), _c.POINTER(_c.c_int64)]),
    "vmc_probe_lds_atomics": (_c.c_int, [_c.c_int, _c.c_int, _c.POINTER(_c.c_double), _vp]),
    "vmc_probe_fp32_fma": (_c.c_int, [_c.c_int, _c.c_int, _c.POINTER(_c.c_double), _vp]),
    "bases_cube_max": (_c.c_int, [_vp, _vp, _c.c_int64]),
    "spring_workspace_sizes": (_c.c_int, [_vp, _c.POINTER(_c.c_size_t)]),
    "spring_setup": (_c.c_int, [_vp, _vp, _c.c_double, _vp, _vp, _vp, _vp]),
    "spring_clear_counts": (_c.c_int, [_vp, _vp]),
    "spring_generate": (_c.c_int, [_vp, _c.c_int, _vp, _c.c_int, _vp, _vp, _vp, _c.c_uint64, _c.c_uint32,
                                   _c.c_int64, _c.c_int64, _c.c_int64, _vp, _vp, _c.c_uint32, _vp]),
}


def header_functions(path: str = HEADER) -> list[str]:
    """Names of the functions declared in include/vmc.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)


def lib():
    """The loaded library; raises VmcNotBuilt when it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise VmcNotBuilt(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    try:
        L = ctypes.CDLL(LIB_PATH)
    except OSError as e:
        raise VmcNotBuilt(f"cannot load {LIB_PATH}: {e}") from e
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def integrand_info(integrand: int, dim: int, fp64: bool = False) -> tuple[int, int]:
    """(ntheta, ngrad) of a compiled integrand: theta takes ntheta values, the
    adjoint pass differentiates the first ngrad of them."""
    nt, ng = ctypes.c_int(), ctypes.c_int()
    call("vmc_integrand_info", int(integrand), int(dim), FLAG_FP64 if fp64 else 0, ctypes.byref(nt), ctypes.byref(ng))
    return nt.value, ng.value


def check(rc: int) -> None:
    if rc != 0:
        msg = lib().vmc_last_error().decode(errors="replace")
        raise VmcError(rc, msg)


# ctypes wraps an out-of-range Python int silently; the integer arguments
# are checked against their C type first
_INT_RANGE = {ctypes.c_int: (-2**31, 2**31), ctypes.c_uint32: (0, 2**32), ctypes.c_int64: (-2**63, 2**63),
              ctypes.c_uint64: (0, 2**64)}


def call(name: str, *args) -> None:
    fn = getattr(lib(), name)
    for i, (a, t) in enumerate(zip(args, fn.argtypes or ())):
        lim = _INT_RANGE.get(t)
        if lim is not None and isinstance(a, int) and not lim[0] <= a < lim[1]:
            raise ValueError(f"{name}: argument {i} = {a} does not fit {t.__name__}")
    check(fn(*args))
