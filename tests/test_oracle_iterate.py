"""Pins for one oracle iteration (steps 2-4 of the six-step structure, paper
Sec. 3.1) in plain (VEGAS) and stratified (BASES) mode, and for the driver
(steps 5-6, ITMX / ITMX1 / ITMX2 of Sec. 6.1).

Library re-derivations: per-axis bin sums equal numpy bincount over a
per-sample dump; the plain variance equals numpy's ddof=1 variance / N; the
stratified variance is rebuilt from a reshape of the per-sample weights by
cube.  Closed forms: the variance of the d=4 Gaussian estimate on the uniform
grid, the stratified variance 1/(12 M^3 k) of f = x, exact zero variance for
a constant, and the known integrals of the Gaussian configurations.
"""
import math
import os

import numpy as np
import pytest
from scipy import special

import oracle as O

C1 = dict(iid=O.GAUSS, d=4, N=50, theta=[0.5, 0.1])


def _grid(rng, d, N):
    w = rng.gamma(1.0, size=(d, N)) + 0.05
    e = np.concatenate([np.zeros((d, 1)), np.cumsum(w, axis=1)], axis=1)
    e /= e[:, -1:]
    e[:, -1] = 1.0
    return e


@pytest.mark.parametrize("ng", [1, 3])
def test_bins_and_totals_match_per_sample_dump(ng):
    rng = np.random.default_rng(ng)
    d, N, ncall = 3, 20, 3 * 3**3 * 5 + 7
    e = _grid(rng, d, N)
    th = [0.2, 0.7, 0.15]
    r = O.iterate(O.DGAUSS, e, th, ncall, 99, 4, ng=ng)
    n = r["n_eff"]
    s = O.eval_samples(O.DGAUSS, e, th, ncall, 99, 4, 0, n, ng=ng)
    w = s["w"]
    assert abs(r["S1"] - w.sum()) <= 1e-13 * np.abs(w).sum()
    assert abs(r["S2"] - (w * w).sum()) <= 1e-13 * (w * w).sum()
    for a in range(d):
        assert np.allclose(r["bins"][0, a], np.bincount(s["j"][:, a], w, minlength=N), rtol=1e-13, atol=0)
        assert np.allclose(r["bins"][1, a], np.bincount(s["j"][:, a], w * w, minlength=N), rtol=1e-13, atol=0)
    # the map and f: w = f(x) * J with x inside the bin of j
    for a in range(d):
        lo = e[a][s["j"][:, a]]
        hi = e[a][s["j"][:, a] + 1]
        assert np.all((s["x"][:, a] >= lo) & (s["x"][:, a] <= hi))
    if ng == 1:
        assert n == ncall
        assert abs(r["I"] - w.mean()) < 1e-15 * abs(w).mean() * 10
        assert abs(r["var"] / (np.var(w, ddof=1) / n) - 1) < 1e-10
    else:
        M = 3**d
        k = ncall // M
        assert n == k * M
        W = w.reshape(k, M)  # sample s = c + t M
        S1c, S2c = W.sum(axis=0), (W * W).sum(axis=0)
        V = np.sum(k * S2c - S1c**2)
        assert abs(r["V"] / V - 1) < 1e-10
        # per-cube unbiased variance of the cube mean, summed with weights 1/M^2
        ref_var = np.sum(np.var(W, axis=0, ddof=1) / k) / M**2
        assert abs(r["var"] / ref_var - 1) < 1e-10
        # cube coordinates: axis a of cube c is digit a of c in base ng
        c = np.arange(n) % M
        for a in range(d):
            ca = (c // 3**a) % 3
            y_lo = ca / 3.0
            jy = s["j"][:, a]
            assert np.all((jy >= np.floor(y_lo * N)) & (jy <= np.ceil((ca + 1) / 3.0 * N) - 1))


def test_replay_uses_given_weights():
    rng = np.random.default_rng(1)
    e = _grid(rng, 2, 10)
    ncall = 500
    w_in = rng.normal(size=ncall).astype(np.float32)
    r = O.iterate(O.LINEAR, e, [], ncall, 5, 0, w_in=w_in)
    w = w_in.astype(np.float64)
    assert r["S1"] == pytest.approx(w.sum(), rel=1e-14)
    assert r["S2"] == pytest.approx((w * w).sum(), rel=1e-14)


def test_constant_integrand_has_zero_variance():
    e = O.uniform_edges(2, 8)
    r = O.iterate(O.CONST, e, [2.5], 1000, 1, 0)
    assert r["I"] == 2.5 and r["var"] == 0.0
    r = O.iterate(O.CONST, e, [2.5], 4 * 4 * 10, 1, 0, ng=4)
    assert r["I"] == 2.5 and r["var"] == 0.0 and r["n_eff"] == 160
    r = O.iterate(O.CONST, e, [0.0], 100, 1, 0)
    assert r["I"] == 0.0 and r["var"] == 0.0
    r = O.iterate(O.CONST, e, [float("nan")], 100, 1, 0)
    assert r["nonfinite"] == 100 and math.isnan(r["I"])


@pytest.mark.slow
def test_stratified_variance_closed_form():
    # f = x on [0,1], M strata, k samples each: Var(I) = 1/(12 M^3 k)
    M, k, nseeds = 4, 2, 3000
    e = O.uniform_edges(1, 16)
    Is, vs = [], []
    for seed in range(nseeds):
        r = O.iterate(O.LINEAR, e, [], M * k, seed, 0, ng=M)
        Is.append(r["I"])
        vs.append(r["var"])
    expect = 1.0 / (12 * M**3 * k)
    assert abs(np.mean(Is) - 0.5) < 5 * math.sqrt(expect / nseeds)
    # mean of the unbiased estimator, and the empirical spread of I
    assert abs(np.mean(vs) / expect - 1) < 0.1
    assert abs(np.var(Is, ddof=1) / expect - 1) < 0.1


@pytest.mark.slow
def test_c1_first_iteration_variance_closed_form():
    # sigma_I^2 = (int f^2 - 1)/N, int f^2 = [erf(5 sqrt 2)/(0.1 sqrt(2 pi) erf(5)^2)]^4
    N, nseeds = 2000, 300
    e = O.uniform_edges(4, 50)
    f2 = (special.erf(5 * math.sqrt(2)) / (0.1 * math.sqrt(2 * math.pi) * special.erf(5) ** 2)) ** 4
    expect = (f2 - 1) / N
    Is, vs = [], []
    for seed in range(nseeds):
        r = O.iterate(O.GAUSS, e, C1["theta"], N, seed, 0)
        Is.append(r["I"])
        vs.append(r["var"])
    assert abs(np.mean(Is) - 1) < 5 * math.sqrt(expect / nseeds)
    assert abs(np.mean(vs) / expect - 1) < 0.15


def test_gradient_estimate_matches_closed_form():
    d, c, s = 3, np.array([0.3, 0.5, 0.7]), 0.15
    th = list(c) + [s]
    run_edges = O.integrate(O.GAUSS_AXES, d, 64, th, 20000, 5, 3).edges
    r = O.iterate(O.GAUSS_AXES, run_edges, th, 200000, 8, 9, want_grad=True)
    h = 0.5 * (special.erf((1 - c) / s) + special.erf(c / s))
    I = np.prod(h)
    dh_dc = (np.exp(-c**2 / s**2) - np.exp(-(1 - c)**2 / s**2)) / (s * math.sqrt(math.pi))
    dh_ds = (-(1 - c) * np.exp(-(1 - c)**2 / s**2) - c * np.exp(-c**2 / s**2)) / (s * s * math.sqrt(math.pi))
    exact = np.concatenate([I * dh_dc / h, [I * np.sum(dh_ds / h)]])
    z = (r["grad"] - exact) / np.sqrt(r["grad_var"])
    assert np.all(np.abs(z) < 4.5), z
    assert abs(r["I"] - I) / math.sqrt(r["var"]) < 4.5


def test_stratified_gradient_variance_matches_per_cube_form():
    rng = np.random.default_rng(4)
    e = _grid(rng, 2, 12)
    th = [0.4, 0.6, 0.2]
    ng, ncall = 3, 9 * 6
    r = O.iterate(O.GAUSS_AXES, e, th, ncall, 3, 1, ng=ng, want_grad=True)
    s = O.eval_samples(O.GAUSS_AXES, e, th, ncall, 3, 1, 0, ncall, ng=ng)
    k, M = 6, 9
    for p in range(3):
        W = (s["jac"] * s["grad"][:, p]).reshape(k, M)
        assert abs(r["grad"][p] - W.mean()) < 1e-13 * np.abs(W).mean()
        ref = np.sum(np.var(W, axis=0, ddof=1) / k) / M**2
        assert abs(r["grad_var"][p] / ref - 1) < 1e-9


def test_c1_vegas_converges():
    run = O.integrate(O.GAUSS, 4, 50, [0.5, 0.1], 10000, 10, 1234, alpha=1.5)
    assert abs(run.Ibar - 1) / run.sigbar < 3
    assert run.sigbar < 0.01
    assert run.chi2dof < 5


def test_bases_two_phase_driver_uses_phase_two_only():
    run = O.integrate(O.DGAUSS, 4, 32, [1 / 3, 2 / 3, 0.1], 4**4 * 6, 4, 77, ng=4, itmx2=3)
    assert len(run.I) == 3
    Ib, sb, _ = O.combine(run.I, run.var)
    assert Ib == run.Ibar and sb == run.sigbar
    assert abs(run.Ibar - 1) / run.sigbar < 4


def test_error_codes():
    e = O.uniform_edges(2, 8)
    with pytest.raises(O.OracleError):
        O.iterate(O.GAUSS, e, [0.5], 100, 1, 0)  # wrong theta length
    with pytest.raises(O.OracleError):
        O.iterate(42, e, [0.5], 100, 1, 0)  # unknown integrand
    with pytest.raises(O.OracleError):
        O.iterate(O.GAUSS, e, [0.5, 0.1], 1, 1, 0)  # ncall < 2
    with pytest.raises(O.OracleError):
        O.iterate(O.GAUSS, e, [0.5, 0.1], 4 * 4 + 3, 1, 0, ng=4)  # k < 2
    with pytest.raises(O.OracleError):
        O.iterate(O.WJETS, O.uniform_edges(9, 8), [0] * 7, 100, 1, 0)  # bad physics dimension


def test_sharded_iteration_equals_single_iteration():
    """Disjoint sample ranges summed give the single-range sums (the CPU
    rehearsal of splitting one iteration's samples across devices)."""
    import multiprocessing as mp
    rng = np.random.default_rng(12)
    e = _grid(rng, 4, 16)
    th = [0.4, 0.6, 0.15]
    ref = O.iterate(O.DGAUSS, e, th, 100_003, 5, 2)
    with mp.get_context("fork").Pool(3) as pool:
        got = O.iterate_sharded(O.DGAUSS, e, th, 100_003, 5, 2, pool, 5)
    for key in ("S1", "S2", "I", "var"):
        assert abs(got[key] - ref[key]) <= 1e-12 * abs(ref[key])
    assert np.allclose(got["bins"], ref["bins"], rtol=1e-12, atol=0)
    assert got["n_eff"] == ref["n_eff"]


def test_cpu_rate_child_runs_the_same_iteration(tmp_path):
    """The all-core CPU-baseline timer (a child process with a worker pool)
    evaluates the same iteration as the single-thread oracle."""
    import json
    import subprocess
    import sys
    rng = np.random.default_rng(13)
    e = _grid(rng, 4, 16)
    th = [0.4, 0.6, 0.15]
    np.save(tmp_path / "edges.npy", e)
    cfg = dict(integrand=O.DGAUSS, edges=str(tmp_path / "edges.npy"), theta=th, ncall=50_001, seed=5, it=2, nproc=2)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, "-m", "oracle.cpu_rate", json.dumps(cfg)], cwd=root, capture_output=True,
                       text=True, timeout=120, check=True)
    got = json.loads(p.stdout.strip().splitlines()[-1])
    ref = O.iterate(O.DGAUSS, e, th, 50_001, 5, 2)
    assert got["samples"] == 50_001 and got["procs"] == 2 and got["seconds"] > 0
    assert abs(got["I"] - ref["I"]) <= 1e-12 * abs(ref["I"])
    assert abs(got["var"] - ref["var"]) <= 1e-10 * abs(ref["var"])
