"""The adjoint behind torch.autograd: backward() of the single-iteration
estimate equals the adjoint pass, the fused pass, central differences with
common random numbers, and (for the physics toy) the exact coupling identity
g dI/dg = 2 n_p I."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1010_2107_amd import workloads as W
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
    theta = torch.tensor(w.theta, dtype=torch.float64, device="cuda", requires_grad=True)
    I = vegas_integral(theta, g, w.integrand, 2_000_000, 5, 3, fused=True)
    I.backward()
    gt = theta.grad.cpu().numpy()
    n_p = (w.dim - 4) // 3
    # FP32 per-sample products: the identity holds to FP32 rounding of the sums
    assert abs(w.theta[2] * gt[2] / (2 * n_p * I.item()) - 1) < 1e-5
    assert np.all(gt[3:] == 0)
