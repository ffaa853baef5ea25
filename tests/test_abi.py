"""The C ABI library builds, loads and exports every function declared in
include/vmc.h; host-side argument validation (no GPU needed)."""
import ctypes

import pytest

import paper_1010_2107_amd as V
from paper_1010_2107_amd import _lib as L


def test_every_declared_function_is_exported():
    names = V.header_functions()
    assert len(names) >= 17
    lib = V.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(L._SIGS), set(names) ^ set(L._SIGS)


def test_workspace_sizes_and_create_validation():
    sz = (ctypes.c_size_t * 4)()
    L.call("vmc_workspace_sizes", 8, 128, sz)
    assert list(sz) == [8 * 8 * 129, 4 * 2 * 8 * 128, 8 * 2 * 8 * 128, 8 * 128]
    for d, n, code in ((0, 10, "VMC_E_DIM"), (17, 10, "VMC_E_DIM"), (4, 1, "VMC_E_NBINS"), (4, 257, "VMC_E_NBINS")):
        h = ctypes.c_void_p()
        with pytest.raises(V.VmcError) as e:
            L.call("vmc_create", d, n, ctypes.byref(h))
        assert e.value.name == code


def test_host_side_errors_without_gpu():
    h = ctypes.c_void_p()
    L.call("vmc_create", 4, 50, ctypes.byref(h))
    try:
        with pytest.raises(V.VmcError) as e:
            L.call("vmc_iterate", h, V.GAUSS, None, 0, 1000, 1, 0, 0, None)
        assert e.value.name == "VMC_E_UNBOUND"
        with pytest.raises(V.VmcError) as e:
            L.call("vmc_set_schedule", h, 100, 0)
        assert e.value.name == "VMC_E_SCHEDULE"
        with pytest.raises(V.VmcError) as e:
            L.call("vmc_set_schedule", h, 0, 3)
        assert e.value.name == "VMC_E_SCHEDULE"
        L.call("vmc_set_schedule", h, 512, 8)
        with pytest.raises(V.VmcError) as e:
            L.call("bases_stratify", h, 1 << 11)  # (2^11)^4 = 2^44 cubes
        assert e.value.name == "VMC_E_STRAT"
        L.call("bases_stratify", h, 4)
        with pytest.raises(V.VmcError) as e:
            L.call("vmc_bind", h, None, None, None, None)
        assert e.value.name == "VMC_E_INVALID"
    finally:
        L.call("vmc_destroy", h)
    L.call("vmc_destroy", None)
    assert V.lib().vmc_version() >= 100
