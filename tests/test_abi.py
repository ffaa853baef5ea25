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
    stripe = (2 * 8 * 128 + 64 + 15) // 16 * 16  # one copy of the block partial sums
    assert list(sz) == [8 * 8 * 129, 4 * 2 * 8 * 128, 8 * (2 * 8 * 128 + 32 * stripe), 8 * 128]
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
        with pytest.raises(V.VmcError) as e:
            L.call("vmc_set_schedule", h, 0, 512)
        assert e.value.name == "VMC_E_SCHEDULE"
        L.call("vmc_set_schedule", h, 0, 256)
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


def test_batch_create_validation():
    def create(dims, ncalls, integrand=V.GAUSS_AXES, nbins=64):
        h = ctypes.c_void_p()
        d = (ctypes.c_int * len(dims))(*dims)
        n = (ctypes.c_int64 * len(ncalls))(*ncalls)
        L.call("vmc_batch_create", len(dims), d, nbins, integrand, n, ctypes.byref(h))
        return h
    for args, code in ((([13], [100]), "VMC_E_DIM"), (([3], [1]), "VMC_E_NCALLS"),
                       (([3], [100], V.GAUSS), "VMC_E_INTEGRAND"), (([3], [100], V.GAUSS_AXES, 1), "VMC_E_NBINS")):
        with pytest.raises(V.VmcError) as e:
            create(*args)
        assert e.value.name == code
    h = create([2, 12, 5], [10_000, 1_000_000, 257])
    sz = (ctypes.c_size_t * 6)()
    L.call("vmc_batch_workspace_sizes", h, sz)
    assert sz[0] == 8 * 19 * 65 and sz[1] == 4 * 2 * 19 * 64 and sz[2] == 8 * 2 * 19 * 64
    assert sz[3] == 8 * 128 * 3 and sz[4] == 8 * (3 + 19)
    with pytest.raises(V.VmcError) as e:
        L.call("vmc_batch_set_schedule", h, -1, 0)
    assert e.value.name == "VMC_E_SCHEDULE"
    with pytest.raises(V.VmcError) as e:
        L.call("vmc_iterate_batched", h, 1, 0, 1, 0, None)
    assert e.value.name == "VMC_E_UNBOUND"
    L.call("vmc_batch_destroy", h)


def test_integer_arguments_are_range_checked():
    """ctypes would wrap 2^31 into a negative int (ng = 2^31 would silently
    mean plain sampling); the binding refuses values that do not fit."""
    sizes = (ctypes.c_size_t * 4)()
    with pytest.raises(ValueError):
        L.call("vmc_workspace_sizes", 2**31, 64, sizes)
    with pytest.raises(ValueError):
        L.call("vmc_workspace_sizes", 4, -2**31 - 1, sizes)
    L.call("vmc_workspace_sizes", 4, 64, sizes)
    assert sizes[0] == 8 * 4 * 65


def test_build_flags():
    """Every unit is built for gfx950 with packed FP32 off and multiply-add
    fusion only within one source expression (so that every kernel inlining
    the same integrand code rounds it alike)."""
    from paper_1010_2107_amd import build as B
    f = " ".join(B.FLAGS)
    assert "--offload-arch=gfx950" in f or B.ARCH != "gfx950"
    assert "-Xclang -target-feature -Xclang -packed-fp32-ops" in f
    assert "-ffp-contract=on" in B.FLAGS
