"""Forward passes of the integrands that split at the cuts (W + partons,
helicity amplitudes) in FP32, whose kernels queue the samples that pass and
run stage 2 on full waves.  In stratified (BASES) mode each queued weight
returns to its cube chunk through an LDS slot of the lane that drew it.
Checks:

- Replay: the oracle accumulates the GPU's own FP32 weights (dumped per
  sample) in FP64 (Kawabata's per-cube variance over ng^d cubes), and the
  cube maxima are the maxima of those weights (at least 0).  The dump runs
  the same stages in another kernel; the library fuses multiply-adds only
  within one source expression, so both kernels round each weight alike
  and the replayed sums differ by summation order only.  Bounds: S1, S2, I
  at 1e-7, the variance and the bins at 1e-6, each cube maximum at 1e-6
  relative, the zero-weight count exactly.  A weight added to the wrong
  cube would move that cube's terms by O(1).
- End to end against the oracle's FP64 integrand evaluated at the point
  the FP32 grid map forms (oracle.point32): S1 at 1e-5, S2 at 2e-5, bin
  planes at 1e-5 and 2e-5 norm-wise, V = sum_c (k S2_c - S1_c^2) at 2e-5
  times the amplification sum_c (k S2_c + S1_c^2) / V of its difference
  (computed from the oracle's weights), 99 % of the cube maxima at 1e-4
  (each is one sample's weight, so the per-sample bound applies).
  A few cube maxima may differ where an FP32 cut decision flips at a
  threshold.  The distance to the oracle at the FP64 point is printed; it
  adds the rounding of the point, which the resonance amplifies.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1010_2107_amd import WHEL, WJETS, Grid
from paper_1010_2107_amd import workloads as W
from tests.gpu_util import announce, normwise, rel, require_gpu

pytestmark = pytest.mark.gpu

CASES = [
    ("wjets_d10_ng2", WJETS, 10, W.WJETS_THETA, 2, 400),
    ("wjets_d16_ng2", WJETS, 16, W.WJETS_THETA, 2, 6),
    ("whel_d8_ng2", WHEL, 8, W.WHEL_THETA, 2, 400),
    ("whel_d11_ng2", WHEL, 11, W.WHEL_THETA, 2, 60),
    # ng = 3 does not divide the 64 bins: the FP32 bin map with the quotient
    # and remainder by ng
    ("wjets_d10_ng3", WJETS, 10, W.WJETS_THETA, 3, 3),
    ("whel_d8_ng3", WHEL, 8, W.WHEL_THETA, 3, 20),
]


@pytest.mark.parametrize("case", [("wjets_d10", WJETS, 10, W.WJETS_THETA), ("wjets_d16", WJETS, 16, W.WJETS_THETA),
                                  ("whel_d8", WHEL, 8, W.WHEL_THETA), ("whel_d11", WHEL, 11, W.WHEL_THETA)],
                         ids=lambda c: c[0])
def test_fp32_plain_staged_replay(case):
    """The plain kernel's stage-2 queue: the oracle's FP64 accumulation of the
    dumped FP32 weights gives the GPU's sums (bounds as above)."""
    require_gpu()
    name, iid, d, th = case
    announce(f"plain staged replay {name}")
    N, ncall = 64, 300_007
    e = O.integrate(iid, d, N, th, 40_000, 2, 32).edges
    g = Grid(d, N)
    g.set_edges(e)
    g.iterate(iid, th, ncall, 4321, 3)
    r = g.result()
    dump = g.dump(iid, th, ncall, 4321, 3, 0, ncall)
    rep = O.iterate(iid, e, th, ncall, 4321, 3, w_in=dump["w"])
    print(f"{name}: replay S1 {rel(r['S1'], rep['S1']):.1e} bins {normwise(g.bins.cpu().numpy(), rep['bins']):.1e}")
    for key in ("S1", "S2", "I"):
        assert rel(r[key], rep[key]) <= 1e-7, key
    assert normwise(g.bins.cpu().numpy(), rep["bins"]) <= 1e-6
    assert r["n_zero"] == int(np.count_nonzero(dump["w"] == 0))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fp32_stratified_matches_oracle(case):
    require_gpu()
    name, iid, d, th, ng, k = case
    announce(f"stratified fp32 {name}")
    N = 64
    M = ng ** d
    ncall = M * k + 7
    e = O.integrate(iid, d, N, th, 40_000, 2, 31).edges
    g = Grid(d, N)
    g.stratify(ng)
    g.set_edges(e)
    buf = torch.zeros(M, dtype=torch.float64, device="cuda")
    g.bind_cube_max(buf)
    g.iterate(iid, th, ncall, 1234, 5)
    r = g.result()
    assert r["n_eff"] == M * k and r["nonfinite"] == 0
    bins = g.bins.cpu().numpy()
    got_max = buf.cpu().numpy()

    # replay: the oracle's FP64 accumulation of the GPU's FP32 weights
    dump = g.dump(iid, th, ncall, 1234, 5, 0, r["n_eff"])
    rep = O.iterate(iid, e, th, ncall, 1234, 5, ng=ng, w_in=dump["w"])
    print(f"{name}: replay S1 {rel(r['S1'], rep['S1']):.1e} var {rel(r['var'], rep['var']):.1e} "
          f"bins {normwise(bins, rep['bins']):.1e}")
    for key in ("S1", "S2", "I"):
        assert rel(r[key], rep[key]) <= 1e-7, key
    assert rel(r["var"], rep["var"]) <= 1e-6
    assert normwise(bins, rep["bins"]) <= 1e-6
    assert r["n_zero"] == int(np.count_nonzero(dump["w"] == 0))
    w = dump["w"].astype(np.float64)
    want_max = np.zeros(M)
    np.maximum.at(want_max, np.arange(w.size) % M, w)
    assert np.all(np.abs(got_max - want_max) <= 1e-6 * want_max)

    # end to end against the FP64 integrand at the same (FP32-mapped) point
    ref = O.iterate(iid, e, th, ncall, 1234, 5, ng=ng, fp32_point=True)
    r64 = O.iterate(iid, e, th, ncall, 1234, 5, ng=ng)
    cm = np.zeros(M)
    with O.point32():
        O.cube_max(iid, e, th, ncall, 1234, 5, ng, cm)
    # V = sum_c (k S2_c - S1_c^2) is a difference: relative errors of the
    # terms (<= 2e-5, the squared sums) reach V amplified by
    # A = sum_c (k S2_c + S1_c^2) / V, computed from the oracle's weights
    ow = O.eval_samples(iid, e, th, ncall, 1234, 5, 0, M * k, ng=ng, fp32_point=True)["w"].reshape(k, M)
    s1c, s2c = ow.sum(axis=0), (ow * ow).sum(axis=0)
    amp = np.sum(k * s2c + s1c * s1c) / np.sum(k * s2c - s1c * s1c)
    for tag, o in (("fp32 point", ref), ("fp64 point", r64)):
        print(f"{name} vs oracle at the {tag}: S1 {rel(r['S1'], o['S1']):.1e} S2 {rel(r['S2'], o['S2']):.1e} "
              f"V {rel(r['V'], o['V']):.1e} (amplification {amp:.1f}) bins {normwise(bins[0], o['bins'][0]):.1e} "
              f"{normwise(bins[1], o['bins'][1]):.1e}")
    assert rel(r["S1"], ref["S1"]) <= 1e-5
    assert rel(r["S2"], ref["S2"]) <= 2e-5
    assert rel(r["V"], ref["V"]) <= 2e-5 * amp
    assert normwise(bins[0], ref["bins"][0]) <= 1e-5
    assert normwise(bins[1], ref["bins"][1]) <= 2e-5
    # a cube maximum is one sample's weight: the per-sample bound applies
    close = np.abs(got_max - cm) <= 1e-4 * np.abs(cm) + 1e-300
    print(f"{name}: cube maxima within 1e-4 of the oracle's: {close.mean():.4f}")
    assert close.mean() >= 0.99


@pytest.mark.parametrize("case", [("wjets_d10_ng2", WJETS, 10, W.WJETS_THETA, 2, 4096),
                                  ("whel_d8_ng2", WHEL, 8, W.WHEL_THETA, 2, 3000),
                                  ("wjets_d10_ng3", WJETS, 10, W.WJETS_THETA, 3, 70)],
                         ids=lambda c: c[0])
def test_queued_schedule_invariance(case):
    """The queued stratified kernel under the built-in schedule and under
    explicit ones (one lane per cube up to 256 lanes spanning the block's
    waves, one to four units per lane): every sample's FP32 weight is the
    same, so the FP64 sums agree to summation order (1e-12) and the
    zero-weight count exactly."""
    require_gpu()
    name, iid, d, th, ng, k = case
    announce(f"queued schedule invariance {name}")
    M = ng ** d
    ncall = M * k + 5
    e = O.integrate(iid, d, 64, th, 40_000, 2, 33).edges
    out = []
    for bs, ch in ((0, 0), (256, 1), (1024, 8), (256, 64), (512, 128), (256, 256)):
        if ch > k:
            continue
        g = Grid(d, 64)
        g.stratify(ng)
        g.set_edges(e)
        g.set_schedule(bs, ch)
        g.iterate(iid, th, ncall, 99, 2)
        out.append(((bs, ch), g.result(), g.bins.cpu().numpy()))
    _, r0, b0 = out[0]
    for sched, r, b in out[1:]:
        for key in ("S1", "S2", "V", "I"):
            assert rel(r[key], r0[key]) <= 1e-12, (sched, key)
        assert r["n_zero"] == r0["n_zero"], sched
        assert normwise(b, b0) <= 1e-12, sched
