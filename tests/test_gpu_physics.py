"""GPU parity of the W + partons toy integrand (d = 3 n_p + 4) and of its
flux x phase-space part against the FP64 oracle.

Tolerances:
  * FP64 instantiation, per sample: 1e-10 relative.  The oracle forms
    m_enu^2 = 2 p_e.p_nu from boosted momenta, which loses up to
    (E/m)^2 ~ 2e3 ulps; the Breit-Wigner slope m^2/(M Gamma) ~ 40 carries that
    into f at a few 1e-12 -- 1e-10 leaves margin.  Cut decisions must agree
    except for events within 1e-9 (relative) of a threshold.
  * FP32 integrand, against the oracle evaluated at the same point (the
    point as the FP32 grid map forms it, oracle.point32): per-sample median
    1e-5, 99th percentile 2e-4, contribution-weighted 1e-5; iteration sums
    S1 1e-5, S2 2e-5, bin planes 1e-5 and 2e-5 norm-wise (squaring doubles
    the relative error).  The distance to the oracle at the FP64 point is
    printed too; it adds the rounding of the point itself, amplified by the
    Breit-Wigner slope.  Cut decisions may differ only within 1e-4 of a
    threshold.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1010_2107_amd import workloads as W
from paper_1010_2107_amd.driver import integrate
from paper_1010_2107_amd.grid import Grid
from tests.gpu_util import announce, normwise, rel, require_gpu
from tests.phys_util import cut_margin

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TH = W.WJETS_THETA


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _grid(d, N, seed):
    rng = np.random.default_rng(seed)
    w = rng.gamma(2.0, size=(d, N)) + 0.05
    e = np.concatenate([np.zeros((d, 1)), np.cumsum(w, axis=1)], axis=1)
    e /= e[:, -1:]
    e[:, -1] = 1.0
    return e


@pytest.mark.parametrize("d", [7, 10, 13, 16])
def test_fp64_per_sample(d):
    announce(f"wjets fp64 per-sample d={d}")
    N, ncall, count = 64, 10_000_000, 20_000
    e = _grid(d, N, d)
    g = Grid(d, N)
    g.set_edges(e)
    s0 = 123_456
    got = g.dump(W.WJETS, TH, ncall, 1234, 3, s0, count, fp64=True)
    ref = O.eval_samples(W.WJETS, e, TH, ncall, 1234, 3, s0, count)
    assert np.array_equal(got["words"], ref["words"])
    assert np.allclose(got["jac"], ref["jac"], rtol=1e-13, atol=0)
    both = (got["f"] != 0) & (ref["f"] != 0)
    assert both.sum() > count // 50
    r = np.abs(got["f"][both] - ref["f"][both]) / np.abs(ref["f"][both])
    assert r.max() <= 1e-10, r.max()
    for i in np.nonzero((got["f"] != 0) != (ref["f"] != 0))[0]:
        assert cut_margin(ref["x"][i], TH) < 1e-9, i
    # phase-space part: no cuts, smooth.  The oracle forms (1 - x_a)^3 from
    # x_a = exp(...), whose relative error is eps / (1 - x_a); the tolerance
    # carries that conditioning (the GPU uses expm1 and is the sharper one).
    got = g.dump(W.PSVOL, TH[3:5], ncall, 1234, 3, s0, count, fp64=True)
    ref = O.eval_samples(W.PSVOL, e, TH[3:5], ncall, 1234, 3, s0, count)
    cond = np.array([1 / (1 - ev["x1"]) + 1 / (1 - ev["x2"])
                     for ev in (O.wjets_event(x, TH[3:5]) for x in ref["x"][:2000])])
    tol = 1e-12 + 8 * 2.2e-16 * 3 * cond
    r = np.abs(got["f"][:2000] - ref["f"][:2000]) / np.abs(ref["f"][:2000])
    assert np.all(r <= tol), (r / tol).max()


@pytest.mark.parametrize("d", [10, 16])
def test_fp32_per_sample(d):
    announce(f"wjets fp32 per-sample d={d}")
    N, ncall, count = 64, 50_000_000, 50_000
    e = _grid(d, N, 100 + d)
    g = Grid(d, N)
    g.set_edges(e)
    got = g.dump(W.WJETS, TH, ncall, 1234, 7, 1_000_000, count)
    ref = O.eval_samples(W.WJETS, e, TH, ncall, 1234, 7, 1_000_000, count, fp32_point=True)
    both = (got["f"] != 0) & (ref["f"] != 0)
    r = np.abs(got["f"][both] - ref["f"][both]) / np.abs(ref["f"][both])
    print(f"d={d} pass={both.mean():.3f} rel err median {np.median(r):.2e} p99 {np.quantile(r, .99):.2e} "
          f"max {r.max():.2e}")
    assert np.median(r) <= 1e-5
    assert np.quantile(r, 0.99) <= 2e-4
    flips = np.nonzero((got["f"] != 0) != (ref["f"] != 0))[0]
    for i in flips:
        assert cut_margin(ref["x"][i], TH) < 1e-4, i
    # weighted: the contribution-weighted error is what the sums see
    wsum = np.sum(np.abs(got["w"][both] - ref["w"][both])) / np.sum(np.abs(ref["w"]))
    print(f"d={d} contribution-weighted error {wsum:.2e}")
    assert wsum <= 1e-5, wsum


@pytest.mark.parametrize("d,ncall", [(10, 1_000_003), (16, 500_001)])
def test_fp32_iteration_sums_same_grid(d, ncall):
    announce(f"wjets fp32 sums d={d}")
    N = 64
    e = O.integrate(W.WJETS, d, N, TH, 100_000, 3, 77).edges
    g = Grid(d, N)
    g.set_edges(e)
    g.iterate(W.WJETS, TH, ncall, 1234, 9)
    r = g.result()
    ref = O.iterate(W.WJETS, e, TH, ncall, 1234, 9, fp32_point=True)
    r64 = O.iterate(W.WJETS, e, TH, ncall, 1234, 9)
    b = g.bins.cpu().numpy()
    for name, o in (("fp32 point", ref), ("fp64 point", r64)):
        print(f"d={d} vs oracle at the {name}: S1 {rel(r['S1'], o['S1']):.2e} S2 {rel(r['S2'], o['S2']):.2e} "
              f"plane 0 {normwise(b[0], o['bins'][0]):.2e} plane 1 {normwise(b[1], o['bins'][1]):.2e}")
    assert rel(r["S1"], ref["S1"]) <= 1e-5
    assert rel(r["S2"], ref["S2"]) <= 2e-5
    assert normwise(b[0], ref["bins"][0]) <= 1e-5
    assert normwise(b[1], ref["bins"][1]) <= 2e-5
    assert r["nonfinite"] == 0


def test_fp64_iteration_sums_same_grid():
    announce("wjets fp64 sums d=10 plain and stratified")
    d, N = 10, 64
    e = O.integrate(W.WJETS, d, N, TH, 50_000, 2, 78).edges
    for ng, ncall in ((1, 200_003), (2, 2**10 * 100 + 7)):
        g = Grid(d, N)
        g.stratify(ng)
        g.set_edges(e)
        g.iterate(W.WJETS, TH, ncall, 1234, 4, fp64=True)
        r = g.result()
        ref = O.iterate(W.WJETS, e, TH, ncall, 1234, 4, ng=ng)
        assert rel(r["S1"], ref["S1"]) <= 1e-10 and rel(r["S2"], ref["S2"]) <= 1e-10
        assert normwise(g.bins.cpu().numpy(), ref["bins"]) <= 1e-10
        g.adjoint(W.WJETS, TH, ncall, 1234, 4, fp64=True)
        gr = g.grad_result(3)
        rg = O.iterate(W.WJETS, e, TH, ncall, 1234, 4, ng=ng, want_grad=True)
        assert np.all(np.abs(gr["grad"] - rg["grad"]) <= 1e-10 * np.abs(rg["grad"]) + 1e-300)


def test_adjoint_coupling_identity_and_fd():
    """g dI/dg = 2 n_p I exactly per sample (coupling scaling), and central
    differences in (M, Gamma) with common random numbers (FP64, h = 1e-4 |theta|)."""
    announce("wjets adjoint identities d=10")
    d, N, ncall = 10, 64, 400_000
    e = O.integrate(W.WJETS, d, N, TH, 50_000, 2, 79).edges
    g = Grid(d, N)
    g.set_edges(e)
    g.fused(W.WJETS, TH, ncall, 1234, 2, fp64=True)
    r = g.result()
    G = g.grad_result(3)["grad"]
    assert rel(TH[2] * G[2], 4 * r["I"]) <= 1e-12
    for p in (0, 1):
        h = 1e-4 * TH[p]
        tp, tm = list(TH), list(TH)
        tp[p] += h
        tm[p] -= h
        g.iterate(W.WJETS, tp, ncall, 1234, 2, fp64=True)
        Ip = g.result()["I"]
        g.iterate(W.WJETS, tm, ncall, 1234, 2, fp64=True)
        Im = g.result()["I"]
        fd = (Ip - Im) / (2 * h)
        assert abs(fd - G[p]) <= 1e-5 * abs(r["I"]) / TH[p] + 1e-4 * abs(G[p]), (p, fd, G[p])


@pytest.mark.parametrize("w", [W.C3, W.C4], ids=lambda w: w.name)
def test_configuration_against_oracle_reference(w):
    path = os.path.join(HERE, "golden", "wjets_reference.json")
    if not os.path.exists(path):
        pytest.skip("reference integrals not generated (tests/golden/make_wjets_reference.py)")
    allref = json.load(open(path))
    if str(w.dim) not in allref:
        pytest.skip(f"no reference for d={w.dim} yet")
    ref = allref[str(w.dim)]
    announce(f"end-to-end {w.name}")
    r = integrate(w.integrand, w.dim, w.nbins, w.theta, w.ncall, w.itmx, w.seed, alpha=w.alpha)
    z = abs(r.Ibar - ref["Ibar"]) / np.hypot(r.sigbar, ref["sigbar"])
    print(f"{w.name}: GPU {r.Ibar:.6g} +- {r.sigbar:.3g}, oracle {ref['Ibar']:.6g} +- {ref['sigbar']:.3g}, z={z:.2f}")
    assert z < 3
