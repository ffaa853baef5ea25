"""Adjoint of the W + partons toy (resonance mass M, width Gamma, coupling g)
in the FP32 kernels that the forward+adjoint throughput is measured on.

- FP32 adjoint and fused passes against the oracle's FP64 gradient on the
  same samples and grid, d = 10 (two partons) and d = 16 (four partons),
  plain and stratified, under the built-in launch shape and under the
  8192-sample tiles the 5e7-sample iteration uses: |G_gpu - G_oracle| <=
  1e-5 x (1/N) sum |J df/dtheta| (the L1 scale: a gradient can be small
  through cancellation, as the derivative in M is across the resonance).
- FP64 instantiation against central differences of its own forward
  estimate with common random numbers (same seed, iteration and grid),
  h = 1e-4 |theta|: within 1e-4 of the L1 scale, and g dI/dg = 2 n_p I.
- At the full size of the four-parton configuration (5e7 samples, the
  bench's launch): the FP32 adjoint and fused passes against the FP64
  instantiation (itself pinned to the oracle per sample and through the
  sums above) at 1e-5 of the L1 scale, the adjoint pass against the fused
  pass to summation order, the coupling identity, and sampled per-sample
  FP32 gradients against the oracle's.
"""
import numpy as np
import pytest

import oracle as O
from paper_1010_2107_amd import workloads as W
from paper_1010_2107_amd.grid import Grid
from tests.gpu_util import announce, rel, require_gpu

pytestmark = pytest.mark.gpu
TH = W.WJETS_THETA


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


_EDGES = {}


def _adapted(d):
    """An adapted grid from three oracle iterations (cached per dimension)."""
    if d not in _EDGES:
        _EDGES[d] = O.integrate(W.WJETS, d, 64, TH, 100_000, 3, 77).edges
    return _EDGES[d]


def _l1(edges, ncall, seed, it, ng=1):
    smp = O.eval_samples(W.WJETS, edges, TH, ncall, seed, it, 0, ncall, ng=ng)
    return np.mean(np.abs(smp["jac"][:, None] * smp["grad"]), axis=0)


CASES = [
    ("d10_plain", 10, 1, 1_000_003, 0),
    ("d10_plain_tiles8192", 10, 1, 1_000_003, 8192),
    ("d16_plain", 16, 1, 500_001, 0),
    ("d16_plain_tiles8192", 16, 1, 500_001, 8192),
    ("d10_ng2", 10, 2, 2**10 * 300 + 7, 0),
    ("d16_ng2", 16, 2, 2**16 * 6 + 3, 0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_fp32_adjoint_matches_oracle_gradient(case):
    name, d, ng, ncall, tiles = case
    announce(f"fp32 adjoint vs oracle {name}")
    e = _adapted(d)
    seed, it = 1234, 5
    g = Grid(d, 64)
    g.stratify(ng)
    g.set_edges(e)
    if tiles:
        g.set_schedule(tiles, 0)
    ref = O.iterate(W.WJETS, e, TH, ncall, seed, it, ng=ng, want_grad=True)
    l1 = _l1(e, ncall, seed, it, ng)
    g.iterate(W.WJETS, TH, ncall, seed, it)
    g.adjoint(W.WJETS, TH, ncall, seed, it)
    adj = g.grad_result(3)
    g.fused(W.WJETS, TH, ncall, seed, it)
    fus = g.grad_result(3)
    r = g.result()
    print(f"{name}: G {adj['grad']} oracle {ref['grad']} L1 {l1}; |dG|/L1 adjoint "
          f"{np.abs(adj['grad'] - ref['grad']) / l1} fused {np.abs(fus['grad'] - ref['grad']) / l1}")
    assert np.all(np.abs(adj["grad"] - ref["grad"]) <= 1e-5 * l1)
    assert np.all(np.abs(fus["grad"] - ref["grad"]) <= 1e-5 * l1)
    # the fused pass's forward half is the forward pass
    assert rel(r["S1"], ref["S1"]) <= 1e-5
    if ng == 1:
        # the variance of each gradient estimate, (sum (J df)^2 / N - G^2) / (N - 1):
        # the sum of squares carries twice the per-sample relative error, and
        # the subtraction loses little here (G^2 is far below the mean square)
        assert np.all(np.abs(adj["grad_var"] - ref["grad_var"]) <= 1e-4 * ref["grad_var"])


@pytest.mark.parametrize("d", [10, 16])
def test_fp64_adjoint_against_central_differences(d):
    announce(f"fp64 adjoint vs FD d={d}")
    e = _adapted(d)
    ncall, seed, it = (200_003 if d == 10 else 100_003), 99, 3
    n_p = (d - 4) // 3
    g = Grid(d, 64)
    g.set_edges(e)
    g.fused(W.WJETS, TH, ncall, seed, it, fp64=True)
    I = g.result()["I"]
    G = g.grad_result(3)["grad"]
    ref = O.iterate(W.WJETS, e, TH, ncall, seed, it, want_grad=True)
    l1 = _l1(e, ncall, seed, it)
    assert np.all(np.abs(G - ref["grad"]) <= 1e-10 * l1)
    assert rel(TH[2] * G[2], 2 * n_p * I) <= 1e-12
    for p in range(3):
        h = 1e-4 * TH[p]
        tp, tm = list(TH), list(TH)
        tp[p] += h
        tm[p] -= h
        g.iterate(W.WJETS, tp, ncall, seed, it, fp64=True)
        Ip = g.result()["I"]
        g.iterate(W.WJETS, tm, ncall, seed, it, fp64=True)
        Im = g.result()["I"]
        fd = (Ip - Im) / (2 * h)
        print(f"d={d} p={p}: adjoint {G[p]:.10g} FD {fd:.10g} |diff|/L1 {abs(fd - G[p]) / l1[p]:.2e}")
        assert abs(fd - G[p]) <= 1e-4 * l1[p], (p, fd, G[p], l1[p])


def test_full_size_four_partons():
    """5e7 samples at d = 16, the bench's launch shape (8192-sample tiles)."""
    w = W.C4
    announce("fp32 adjoint full size d16 5e7")
    e = _adapted(w.dim)
    seed, it = w.seed, 7
    g = Grid(w.dim, w.nbins)
    g.set_edges(e)
    g.fused(w.integrand, w.theta, w.ncall, seed, it, fp64=True)
    ref_I = g.result()["I"]
    ref = g.grad_result(3)
    g.iterate(w.integrand, w.theta, w.ncall, seed, it)
    r = g.result()
    g.adjoint(w.integrand, w.theta, w.ncall, seed, it)
    adj = g.grad_result(3)
    g.fused(w.integrand, w.theta, w.ncall, seed, it)
    fus = g.grad_result(3)
    # L1 scale from a per-sample dump of 1e6 of the samples, with a margin
    # for its sampling error (the relative error of such a mean is < 1 %)
    dump = g.dump(w.integrand, w.theta, w.ncall, seed, it, 0, 1_000_000, fp64=True, want_grad=True)
    l1 = 0.9 * np.mean(np.abs(dump["jac"][:, None] * dump["grad"]), axis=0)
    print(f"full size: I fp32 {r['I']:.8g} fp64 {ref_I:.8g}; G fp32 {adj['grad']} fp64 {ref['grad']}; "
          f"|dG|/L1 {np.abs(adj['grad'] - ref['grad']) / l1}")
    assert rel(r["I"], ref_I) <= 1e-5
    assert np.all(np.abs(adj["grad"] - ref["grad"]) <= 1e-5 * l1)
    assert np.all(np.abs(fus["grad"] - ref["grad"]) <= 1e-5 * l1)
    # adjoint and fused passes add the same FP32 per-sample values
    assert np.all(np.abs(adj["gsum"] - fus["gsum"]) <= 1e-12 * np.abs(fus["gsum"]) + 1e-300)
    # g dI/dg = 2 n_p I: each sample's gradient is its weight times 2 n_p / g
    assert rel(w.theta[2] * adj["grad"][2], 2 * 4 * r["I"]) <= 1e-6
    # sampled per-sample FP32 gradients near the end of the range against the oracle
    s0, count = w.ncall - 20_000, 20_000
    got = g.dump(w.integrand, w.theta, w.ncall, seed, it, s0, count, want_grad=True)
    o = O.eval_samples(w.integrand, e, w.theta, w.ncall, seed, it, s0, count)
    both = (got["f"] != 0) & (o["f"] != 0)
    assert both.sum() > count // 10
    for p in range(3):
        err = np.abs(got["grad"][both, p] - o["grad"][both, p]) * o["jac"][both]
        scale = np.abs(o["grad"][both, p]) * o["jac"][both]
        assert np.sum(err) <= 2e-5 * np.sum(scale), (p, np.sum(err) / np.sum(scale))
