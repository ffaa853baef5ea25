"""End-to-end GPU runs of the configurations (statistical acceptance
|Ibar - I_ref| / sigbar < 3, the paper's "agree within statistical errors",
Sec. 6.2) and the adjoint: GPU adjoint vs oracle adjoint on the same samples,
vs central finite differences with common random numbers, and vs closed
forms."""
import math

import numpy as np
import pytest
from scipy import special

import oracle as O
from paper_1010_2107_amd import workloads as W
from paper_1010_2107_amd.driver import integrate
from paper_1010_2107_amd.grid import Grid
from tests.gpu_util import announce, rel, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("w", [W.C1, W.C2, W.C2_PLAIN], ids=lambda w: w.name)
def test_configuration_within_three_sigma(w):
    announce(f"end-to-end {w.name}")
    r = integrate(w.integrand, w.dim, w.nbins, w.theta, w.ncall, w.itmx, w.seed, alpha=w.alpha, ng=w.ng,
                  itmx2=w.itmx2)
    z = abs(r.Ibar - w.I_ref) / r.sigbar
    assert z < 3, (r.Ibar, r.sigbar)
    assert r.chi2dof < 5
    # the grid adapted: later iterations are more precise than the first
    assert r.var[-1] < r.var[0]


@pytest.mark.parametrize("ng", [1, 4])
def test_bases_two_phase_driver_matches_oracle(ng):
    """The driver's two phases (paper Sec. 3.1 and 6.1: ITMX1 iterations that
    re-optimise the grid, then ITMX2 iterations on the frozen grid whose
    results alone are combined), FP64 instantiation, against the oracle's
    driver.  Before each sample pass the GPU grid is set to the edges the
    oracle sampled on, so both sides see the same samples: every I_k and
    var_k, the final Ibar, sigbar and chi^2/dof agree to summation order,
    the grid stays frozen in phase 2, and the phase-1 estimates are shown
    to be left out of the combination."""
    announce(f"bases two-phase driver ng={ng}")
    d, N, theta, seed, itmx1, itmx2 = 8, 128, (1 / 3, 2 / 3, 0.1), 4321, 3, 3
    ncall = 4**8 * 4 + 9 if ng > 1 else 200_003
    ref = O.integrate(W.DGAUSS, d, N, theta, ncall, itmx1, seed, ng=ng, itmx2=itmx2)
    assert len(ref.edges_seq) == itmx1 + itmx2
    # phase 2 samples one frozen grid: the grid of the last refinement
    for k in range(itmx1 + 1, itmx1 + itmx2):
        assert np.array_equal(ref.edges_seq[k], ref.edges_seq[itmx1])
    seen = []

    def sync(grid, k):
        if k <= itmx1:  # phase 2 must not move the grid: no sync there
            grid.set_edges(ref.edges_seq[k])
        seen.append(grid.get_edges())

    r = integrate(W.DGAUSS, d, N, theta, ncall, itmx1, seed, ng=ng, itmx2=itmx2, fp64=True, callback=sync)
    for k in range(itmx1 + 1, itmx1 + itmx2):  # the GPU grid stayed frozen in phase 2
        assert np.array_equal(seen[k], seen[itmx1])
    assert np.max(np.abs(r.grid.get_edges() - ref.edges)) <= 1e-12
    for k in range(itmx1 + itmx2):
        assert rel(r.I[k], ref.I_all[k]) <= 1e-12, k
        assert rel(r.var[k], ref.var_all[k]) <= 1e-10, k
    assert rel(r.Ibar, ref.Ibar) <= 1e-12
    assert rel(r.sigbar, ref.sigbar) <= 1e-10
    assert abs(r.chi2dof - ref.chi2dof) <= 1e-9
    assert r.niter == itmx2
    assert r.n_eff == (itmx1 + itmx2) * (ncall - ncall % 4**8 if ng > 1 else ncall)
    # combining all iterations instead gives a different answer at this precision
    Iall, sall, _ = O.combine(ref.I_all, ref.var_all)
    assert abs(Iall - r.Ibar) > 1e3 * 1e-12 * abs(r.Ibar) or abs(sall - r.sigbar) > 1e3 * 1e-10 * r.sigbar


ADJ_CASES = [
    ("gauss_d4", W.GAUSS, 4, 50, (0.45, 0.12), 200_003, 1),
    ("dgauss_d8_bases", W.DGAUSS, 8, 128, (1 / 3, 2 / 3, 0.1), 4**8 * 4 + 9, 4),
    ("axes_d3_plain", W.GAUSS_AXES, 3, 64, (0.3, 0.5, 0.7, 0.15), 150_001, 1),
    ("axes_d2_bases", W.GAUSS_AXES, 2, 64, (0.35, 0.6, 0.1), 8 * 8 * 50 + 3, 8),
]


def _adapted(iid, d, N, theta, ncall, ng):
    return O.integrate(iid, d, N, theta, min(ncall, 50_000) if ng == 1 else ncall, 3, 17, ng=ng).edges


@pytest.mark.parametrize("case", ADJ_CASES, ids=lambda c: c[0])
def test_adjoint_fp64_matches_oracle(case):
    name, iid, d, N, theta, ncall, ng = case
    announce(f"adjoint fp64 {name}")
    edges = _adapted(iid, d, N, theta, ncall, ng)
    g = Grid(d, N)
    g.stratify(ng)
    g.set_edges(edges)
    P = len(theta) if iid != W.GAUSS_AXES else d + 1
    g.iterate(iid, theta, ncall, 31, 4, fp64=True)  # the forward pass the adjoint differentiates
    g.adjoint(iid, theta, ncall, 31, 4, fp64=True)
    got = g.grad_result(P)
    ref = O.iterate(iid, edges, theta, ncall, 31, 4, ng=ng, want_grad=True)
    scale = np.abs(ref["gsum"]) + np.sqrt(ref["gsumsq"] * ref["n_eff"])
    assert np.all(np.abs(got["gsum"] - ref["gsum"]) <= 1e-12 * scale)
    assert np.all(np.abs(got["gsumsq"] - ref["gsumsq"]) <= 1e-12 * ref["gsumsq"])
    assert np.all(np.abs(got["grad_var"] - ref["grad_var"]) <= 1e-9 * ref["grad_var"])
    # fused pass gives the same gradient and the same forward sums
    g.fused(iid, theta, ncall, 31, 4, fp64=True)
    fz = g.grad_result(P)
    assert np.all(np.abs(fz["gsum"] - ref["gsum"]) <= 1e-12 * scale)
    r = g.result()
    assert rel(r["S1"], ref["S1"]) <= 1e-12


@pytest.mark.parametrize("case", ADJ_CASES, ids=lambda c: c[0])
def test_adjoint_fp32_matches_oracle(case):
    """FP32 integrand: |G_gpu - G_oracle| <= 1e-5 x (1/N) sum |J df/dtheta|."""
    name, iid, d, N, theta, ncall, ng = case
    announce(f"adjoint fp32 {name}")
    edges = _adapted(iid, d, N, theta, ncall, ng)
    g = Grid(d, N)
    g.stratify(ng)
    g.set_edges(edges)
    P = len(theta) if iid != W.GAUSS_AXES else d + 1
    g.iterate(iid, theta, ncall, 31, 4)
    g.adjoint(iid, theta, ncall, 31, 4)
    got = g.grad_result(P)
    ref = O.iterate(iid, edges, theta, ncall, 31, 4, ng=ng, want_grad=True)
    smp = O.eval_samples(iid, edges, theta, ncall, 31, 4, 0, ref["n_eff"], ng=ng)
    l1 = np.mean(np.abs(smp["jac"][:, None] * smp["grad"]), axis=0)
    assert np.all(np.abs(got["grad"] - ref["grad"]) <= 1e-5 * l1), (got["grad"], ref["grad"], l1)


def test_adjoint_vs_central_differences_common_random_numbers():
    """d=8 double Gaussian, h = 1e-4: FD of the GPU's own forward estimate on
    the same samples and frozen grid.  FP64 instantiation: FD truncation
    O(h^2 f'''), bound 1e-4 of the L1 scale."""
    w = W.C2
    announce("adjoint vs FD d8")
    ncall = 4**8 * 8
    edges = _adapted(w.integrand, w.dim, w.nbins, w.theta, ncall, w.ng)
    g = Grid(w.dim, w.nbins)
    g.stratify(w.ng)
    g.set_edges(edges)
    g.iterate(w.integrand, w.theta, ncall, 5, 3, fp64=True)
    g.adjoint(w.integrand, w.theta, ncall, 5, 3, fp64=True)
    G = g.grad_result(3)["grad"]
    smp = O.eval_samples(w.integrand, edges, w.theta, ncall, 5, 3, 0, 4**8 * 8, ng=w.ng)
    l1 = np.mean(np.abs(smp["jac"][:, None] * smp["grad"]), axis=0)
    h = w.fd_h
    for p in range(3):
        tp, tm = list(w.theta), list(w.theta)
        tp[p] += h
        tm[p] -= h
        g.iterate(w.integrand, tp, ncall, 5, 3, fp64=True)
        Ip = g.result()["I"]
        g.iterate(w.integrand, tm, ncall, 5, 3, fp64=True)
        Im = g.result()["I"]
        fd = (Ip - Im) / (2 * h)
        assert abs(fd - G[p]) <= 1e-4 * l1[p], (p, fd, G[p], l1[p])


def test_adjoint_statistics_against_closed_forms():
    announce("adjoint closed forms")
    # double Gaussian normalised on the cube: grad I = 0
    w = W.C2
    g = Grid(w.dim, w.nbins)
    g.stratify(w.ng)
    for it in range(6):
        g.iterate(w.integrand, w.theta, 1_000_000, 77, it)
        g.refine(1.5)
    g.iterate(w.integrand, w.theta, 4**8 * 60, 77, 6)
    g.adjoint(w.integrand, w.theta, 4**8 * 60, 77, 6)
    r = g.grad_result(3)
    z = np.abs(r["grad"]) / np.sqrt(r["grad_var"])
    assert np.all(z < 4), z
    # per-axis Gaussian product: closed-form gradient
    c, s = np.array([0.3, 0.5, 0.7, 0.4, 0.6]), 0.12
    th = tuple(c) + (s,)
    g = Grid(5, 64)
    for it in range(6):
        g.iterate(W.GAUSS_AXES, th, 500_000, 3, it)
        g.refine(1.5)
    g.iterate(W.GAUSS_AXES, th, 4_000_000, 3, 6)
    g.adjoint(W.GAUSS_AXES, th, 4_000_000, 3, 6)
    r = g.grad_result(6)
    hh = 0.5 * (special.erf((1 - c) / s) + special.erf(c / s))
    I = np.prod(hh)
    dh_dc = (np.exp(-c**2 / s**2) - np.exp(-(1 - c)**2 / s**2)) / (s * math.sqrt(math.pi))
    dh_ds = (-(1 - c) * np.exp(-(1 - c)**2 / s**2) - c * np.exp(-c**2 / s**2)) / (s * s * math.sqrt(math.pi))
    exact = np.concatenate([I * dh_dc / hh, [I * np.sum(dh_ds / hh)]])
    z = np.abs(r["grad"] - exact) / np.sqrt(r["grad_var"])
    assert np.all(z < 4), z
