"""The adjoint behind torch.autograd: backward() of the single-iteration
estimate equals the adjoint pass, the fused pass, the oracle's gradient on
the same samples, central differences with common random numbers, and (for
the physics integrands) the exact coupling identity g dI/dg = 2 n I; the
differentiable input is exactly the parameters the adjoint differentiates,
and a backward pass after the grid moved is refused."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1010_2107_amd import _lib as L
from paper_1010_2107_amd import workloads as W
from paper_1010_2107_amd._lib import VmcError
from paper_1010_2107_amd.autograd import vegas_integral
from paper_1010_2107_amd.grid import Grid
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("fused", [False, True])
def test_backward_matches_adjoint_and_fd(fused):
    announce(f"autograd d8 fused={fused}")
    w = W.C2
    g = Grid(w.dim, w.nbins)
    g.stratify(w.ng)
    for it in range(3):
        g.iterate(w.integrand, w.theta, 400_000, 11, it)
        g.refine(1.5)
    theta = torch.tensor(w.theta, dtype=torch.float64, device="cuda", requires_grad=True)
    ncall = 4**8 * 10
    I = vegas_integral(theta, g, w.integrand, ncall, 11, 3, fused=fused)
    (2.5 * I).backward()
    G = theta.grad.cpu().numpy() / 2.5
    g.adjoint(w.integrand, w.theta, ncall, 11, 3)
    ref = g.grad_result(3)["grad"]
    assert np.allclose(G, ref, rtol=1e-12, atol=1e-15)
    # central differences of the same estimator (same samples, same grid)
    h = 1e-3
    for p in range(3):
        tp = theta.detach().clone()
        tm = theta.detach().clone()
        tp[p] += h
        tm[p] -= h
        Ip = vegas_integral(tp, g, w.integrand, ncall, 11, 3).item()
        Im = vegas_integral(tm, g, w.integrand, ncall, 11, 3).item()
        fd = (Ip - Im) / (2 * h)
        # FP32 integrand: FD error ~ eps32 I / h plus O(h^2) truncation
        assert abs(fd - G[p]) <= 2e-3 * (1 + abs(G[p])), (p, fd, G[p])


def test_backward_physics_coupling_identity():
    announce("autograd wjets d10")
    w = W.C3
    g = Grid(w.dim, w.nbins)
    for it in range(3):
        g.iterate(w.integrand, w.theta, 1_000_000, 5, it)
        g.refine(1.5)
    theta = torch.tensor(w.theta[:3], dtype=torch.float64, device="cuda", requires_grad=True)
    I = vegas_integral(theta, g, w.integrand, 2_000_000, 5, 3, fused=True, fixed=w.theta[3:])
    I.backward()
    gt = theta.grad.cpu().numpy()
    assert gt.shape == (3,)
    n_p = (w.dim - 4) // 3
    # FP32 per-sample products: the identity holds to FP32 rounding of the sums
    assert abs(w.theta[2] * gt[2] / (2 * n_p * I.item()) - 1) < 1e-5


def test_parameter_split_is_enforced():
    """theta holds exactly the differentiated parameters; the rest go in
    `fixed`, so no parameter outside the adjoint ever gets a gradient."""
    announce("autograd parameter split")
    assert L.integrand_info(W.WJETS, 10) == (7, 3)
    assert L.integrand_info(W.WHEL, 8) == (8, 3)
    assert L.integrand_info(W.PSVOL, 10) == (2, 0)
    assert L.integrand_info(W.GAUSS_AXES, 5) == (6, 6)
    g = Grid(8, 64)
    full = torch.tensor(W.WHEL_THETA, dtype=torch.float64, device="cuda", requires_grad=True)
    with pytest.raises(ValueError):
        vegas_integral(full, g, W.WHEL, 100_000, 1, 0)
    g10 = Grid(10, 64)
    th = torch.tensor(W.WJETS_THETA[3:5], dtype=torch.float64, device="cuda", requires_grad=True)
    with pytest.raises(ValueError):
        vegas_integral(th, g10, W.PSVOL, 100_000, 1, 0)


@pytest.mark.parametrize("fused", [False, True])
def test_backward_helicity_against_oracle_and_fd(fused):
    """u dbar -> W+ + 1 gluon (d = 8), FP64 instantiation: backward() equals
    the oracle's gradient on the same samples and grid, central differences
    with common random numbers (h = 1e-4 |theta|) and g_s dI/dg_s = 2 I."""
    announce(f"autograd whel d8 fp64 fused={fused}")
    d, N, ncall, seed, it = 8, 64, 60_000, 21, 2
    edges = O.integrate(W.WHEL, d, N, W.WHEL_THETA, 20_000, 2, 5).edges
    g = Grid(d, N)
    g.set_edges(edges)
    th0, fixed = W.WHEL_THETA[:3], W.WHEL_THETA[3:]
    theta = torch.tensor(th0, dtype=torch.float64, device="cuda", requires_grad=True)
    I = vegas_integral(theta, g, W.WHEL, ncall, seed, it, fused=fused, fixed=fixed, fp64=True)
    I.backward()
    G = theta.grad.cpu().numpy()
    assert G.shape == (3,)
    ref = O.iterate(W.WHEL, edges, W.WHEL_THETA, ncall, seed, it, want_grad=True)
    smp = O.eval_samples(W.WHEL, edges, W.WHEL_THETA, ncall, seed, it, 0, ncall)
    l1 = np.mean(np.abs(smp["jac"][:, None] * smp["grad"]), axis=0)
    assert np.all(np.abs(G - ref["grad"]) <= 1e-10 * l1), (G, ref["grad"], l1)
    assert abs(th0[2] * G[2] / (2 * I.item()) - 1) < 1e-12
    for p in range(2):
        h = 1e-4 * th0[p]
        tp, tm = list(th0), list(th0)
        tp[p] += h
        tm[p] -= h
        tpt = torch.tensor(tp, dtype=torch.float64, device="cuda")
        tmt = torch.tensor(tm, dtype=torch.float64, device="cuda")
        Ip = vegas_integral(tpt, g, W.WHEL, ncall, seed, it, fixed=fixed, fp64=True)
        Im = vegas_integral(tmt, g, W.WHEL, ncall, seed, it, fixed=fixed, fp64=True)
        fd = (Ip.item() - Im.item()) / (2 * h)
        assert abs(fd - G[p]) <= 1e-4 * l1[p], (p, fd, G[p], l1[p])


def test_backward_after_grid_change_is_refused():
    """The adjoint regenerates the forward pass's samples from (seed, it) and
    the grid: once the grid has moved it would differentiate a different
    estimator, so both the library and backward() refuse."""
    announce("grid-state guard")
    w = W.C1
    g = Grid(w.dim, w.nbins)
    theta = torch.tensor(w.theta, dtype=torch.float64, device="cuda", requires_grad=True)
    I = vegas_integral(theta, g, w.integrand, 50_000, 3, 0, fused=False)
    g.refine(1.5)
    with pytest.raises(VmcError) as e:
        I.backward()
    assert e.value.name == "VMC_E_GRID"
    # the fused form computed its gradient in the forward pass: unaffected
    theta.grad = None
    I = vegas_integral(theta, g, w.integrand, 50_000, 3, 1, fused=True)
    g.refine(1.5)
    I.backward()
    assert theta.grad is not None
    # the C ABI itself: every grid change invalidates the forward pass
    edges = g.get_edges()
    for change in (lambda: g.refine(1.5), lambda: g.set_edges(edges), lambda: g.stratify(1), lambda: g.reset()):
        g.iterate(w.integrand, w.theta, 50_000, 3, 2)
        g.adjoint(w.integrand, w.theta, 50_000, 3, 2)  # fine right after its forward pass
        v = g.version()
        change()
        assert g.version() > v
        with pytest.raises(VmcError) as e:
            g.adjoint(w.integrand, w.theta, 50_000, 3, 2)
        assert e.value.name == "VMC_E_GRID"
    g2 = Grid(w.dim, w.nbins)
    with pytest.raises(VmcError) as e:
        g2.adjoint(w.integrand, w.theta, 50_000, 3, 0)  # no forward pass at all
    assert e.value.name == "VMC_E_GRID"
