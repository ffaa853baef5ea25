"""GPU parity of the batched persistent launch: each integral of a batch
against the FP64 oracle with integral id k (Philox counter word 3 = k).
Tolerances as for one grid: 1e-12 for the FP64 instantiation, 1e-5 relative
(norm-wise for bins) for the FP32 integrand; after each refinement both
sides continue from the oracle's grid (vmc_batch_set_edges); schedules
agree to FP64 summation order (1e-12); the batched configuration meets its
closed forms."""
import math

import numpy as np
import pytest
from scipy import special

import oracle as O
from paper_1010_2107_amd import workloads as W
from paper_1010_2107_amd.batch import Batch
from tests.gpu_util import announce, normwise, rel, require_gpu

pytestmark = pytest.mark.gpu

DIMS = [1, 2, 5, 12, 3, 7]
NCALLS = [2, 3001, 40_000, 65_537, 7, 100_003]


def _thetas(dims, seed=3):
    rng = np.random.default_rng(seed)
    return [tuple(0.2 + 0.6 * rng.random(d)) + (0.05 * 4 ** rng.random(),) for d in dims]


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("nbins", [16, 64])
@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_batched_matches_oracle_per_integral(fp64, nbins):
    """nbins = 64 is the batched configuration's grid."""
    announce(f"batched vs oracle fp64={fp64} nbins={nbins}")
    th = _thetas(DIMS)
    b = Batch(DIMS, NCALLS, th, nbins=nbins)
    edges = [O.uniform_edges(d, nbins) for d in DIMS]
    tol = 1e-12 if fp64 else 1e-5
    for it in range(3):
        b.iterate(1234, it, kind=3, fp64=fp64)
        r = b.results()
        gr = b.grads()
        for k, d in enumerate(DIMS):
            ref = O.iterate(W.GAUSS_AXES, edges[k], th[k], NCALLS[k], 1234, it, kid=k, want_grad=True)
            assert rel(r["S1"][k], ref["S1"]) <= tol, (k, it)
            assert rel(r["S2"][k], ref["S2"]) <= 2 * tol, (k, it)
            assert normwise(b.bins_of(k)[0], ref["bins"][0]) <= tol
            assert normwise(b.bins_of(k)[1], ref["bins"][1]) <= 2 * tol
            scale = np.abs(ref["gsum"]) + np.sqrt(ref["gsumsq"] * ref["n_eff"])
            assert np.all(np.abs(gr[k]["gsum"] - ref["gsum"]) <= max(tol, 1e-12) * scale), (k, it)
            if fp64:
                assert rel(r["var"][k], ref["var"]) <= 1e-9
        b.refine(1.5)
        for k in range(len(DIMS)):
            ref = O.iterate(W.GAUSS_AXES, edges[k], th[k], NCALLS[k], 1234, it, kid=k)
            new = O.refine(edges[k], ref["bins"][1], 1.5)
            if fp64:
                assert np.max(np.abs(b.edges_of(k) - new)) <= 1e-12
            # both sides go on from the oracle's grid: edges that differ by
            # rounding would move steep integrands' weights by more than 1e-12
            b.set_edges(k, new)
            edges[k] = new


def test_batched_schedule_invariance():
    announce("batched schedule invariance")
    th = _thetas(DIMS, 5)
    out = []
    for spt, blocks in ((0, 0), (1, 64), (4, 4096), (128, 16), (2, 1)):
        b = Batch(DIMS, NCALLS, th, nbins=64)
        b.set_schedule(spt, blocks)
        b.reset()
        b.iterate(77, 2, kind=3)
        out.append((b.results(), [b.bins_of(k) for k in range(len(DIMS))], b.grads()))
    r0, b0, g0 = out[0]
    for r, bb, gg in out[1:]:
        assert np.all(np.abs(r["S1"] - r0["S1"]) <= 1e-12 * np.abs(r0["S1"]))
        for k in range(len(DIMS)):
            assert normwise(bb[k], b0[k]) <= 1e-12
            assert np.all(np.abs(gg[k]["gsum"] - g0[k]["gsum"]) <= 1e-12 * (np.abs(g0[k]["gsum"]) + 1e-300))


def _closed(c, s):
    c = np.asarray(c)
    h = 0.5 * (special.erf((1 - c) / s) + special.erf(c / s))
    I = np.prod(h)
    dh_dc = (np.exp(-c**2 / s**2) - np.exp(-(1 - c)**2 / s**2)) / (s * math.sqrt(math.pi))
    dh_ds = (-(1 - c) * np.exp(-(1 - c)**2 / s**2) - c * np.exp(-c**2 / s**2)) / (s * s * math.sqrt(math.pi))
    return I, np.concatenate([I * dh_dc / h, [I * np.sum(dh_ds / h)]])


def test_batched_configuration_closed_forms():
    """64 integrals, d in [2,12], calls 1e4..1e7, 10 VEGAS iterations with
    the first 5 left out of the combination: every integral and every
    gradient component within 4.5 standard deviations of its closed form."""
    spec = W.batched_config()
    announce("batched configuration (64 integrals)")
    th = [spec.theta(k) for k in range(spec.n)]
    b = Batch(spec.dims, spec.ncalls, th, nbins=spec.nbins)
    r = b.run(spec.seed, spec.itmx, spec.itmx2, kind=3, freeze=spec.freeze)
    g = b.grads()
    zmax, gzmax = 0.0, 0.0
    for k in range(spec.n):
        I, G = _closed(spec.centres[k], spec.sigmas[k])
        z = abs(r["Ibar"][k] - I) / r["sigbar"][k]
        zmax = max(zmax, z)
        gz = np.abs(g[k]["grad"] - G) / np.sqrt(g[k]["grad_var"])
        gzmax = max(gzmax, gz.max())
    print(f"max |z| integrals {zmax:.2f}, gradients (last iteration) {gzmax:.2f}")
    assert zmax < 4.5 and gzmax < 4.5


def test_batched_set_edges():
    """A grid set from the host is the grid the integral samples (its FP32
    table rebuilt: the next iteration equals the oracle's on those edges),
    and malformed calls are refused without touching the grids."""
    import ctypes

    from paper_1010_2107_amd import _lib as L
    from paper_1010_2107_amd._lib import VmcError
    announce("batched set_edges")
    dims, ncalls = [3, 5], [20_001, 30_003]
    th = _thetas(dims, 9)
    b = Batch(dims, ncalls, th, nbins=32)
    rng = np.random.default_rng(11)
    edges = []
    for d in dims:
        w = rng.gamma(2.0, size=(d, 32)) + 0.05
        e = np.concatenate([np.zeros((d, 1)), np.cumsum(w, axis=1)], axis=1)
        e /= e[:, -1:]
        e[:, -1] = 1.0
        edges.append(e)
        b.set_edges(len(edges) - 1, e)
    for k in range(len(dims)):
        assert np.array_equal(b.edges_of(k), edges[k])
    b.iterate(5, 1, kind=1, fp64=True)
    r = b.results()
    for k, d in enumerate(dims):
        ref = O.iterate(W.GAUSS_AXES, edges[k], th[k], ncalls[k], 5, 1, kid=k)
        assert rel(r["S1"][k], ref["S1"]) <= 1e-12 and normwise(b.bins_of(k), ref["bins"]) <= 1e-12
    bad = edges[0].copy()
    bad[1, 5] = bad[1, 4]  # not strictly increasing
    for k, e, name in ((2, edges[0], "VMC_E_INVALID"), (-1, edges[0], "VMC_E_INVALID"), (0, bad, "VMC_E_GRID")):
        with pytest.raises(VmcError) as ex:
            # through the C ABI: the binding's shape check would stop k out of range first
            L.call("vmc_batch_set_edges", b._h, k, e.ctypes.data_as(ctypes.c_void_p), None)
        assert ex.value.name == name
    assert np.array_equal(b.edges_of(0), edges[0])
