"""Pins for the oracle's SPRING event generation (unweighted events from the
BASES integration phase, paper Sec. 3.1; Kawabata's SPRING).

Hand-computed cases: the integer envelope of a few maxima and the cube
chosen by the 64-bit integers at both ends of every interval of a small
envelope.  Closed forms: a product of per-axis Gaussians on [0,1]^2 has
known marginal CDFs (erf), so the kept points are tested against them
(Kolmogorov-Smirnov per axis and a chi^2 over a 2-D cell grid); the keep
rate is the integral over the envelope's integral when nothing overflows;
a constant integrand keeps every trial and picks cubes uniformly.  The
per-cube maxima are re-derived from a per-sample dump with numpy.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

import oracle as O

TWO64 = 1 << 64


def test_envelope_hand_values():
    w = np.array([0.0, 2.0, 1.0, -1.0, np.nan, 1e-7, 2.0 - 2.0**-40])
    q, unit = O.spring_envelope(w)
    assert unit == 2.0 / 2**20
    # ceil(w/2 * 2^20): 0, 2^20, 2^19, 0 (negative), 0 (NaN), ceil(0.0524..) = 1,
    # and one ulp-level shortfall still rounds up to the full 2^20
    assert list(q) == [0, 2**20, 2**19, 0, 0, 1, 2**20]
    with pytest.raises(O.OracleError):
        O.spring_envelope(np.zeros(3))
    with pytest.raises(O.OracleError):
        O.spring_envelope(np.array([1.0, np.inf]))


def test_envelope_bounds_the_maxima():
    rng = np.random.default_rng(3)
    w = rng.lognormal(0.0, 3.0, size=4000)
    q, unit = O.spring_envelope(w)
    assert np.all(q.astype(np.float64) * unit >= w)
    assert np.all((q.astype(np.float64) - 1.0) * unit < w)  # the smallest such integer


def test_pick_hand_table():
    # q = (0, 3, 0, 5, 1): T = 9; r in 0..2 -> cube 1, 3..7 -> cube 3, 8 -> cube 4
    q = [0, 3, 0, 5, 1]
    want = {0: 1, 1: 1, 2: 1, 3: 3, 4: 3, 5: 3, 6: 3, 7: 3, 8: 4}
    T = 9
    for r, c in want.items():
        lo = -(-r * TWO64 // T)            # smallest r64 with floor(r64 T / 2^64) = r
        hi = -(-(r + 1) * TWO64 // T) - 1  # largest
        assert O.spring_pick(q, lo) == c, (r, "lo")
        assert O.spring_pick(q, min(hi, TWO64 - 1)) == c, (r, "hi")


def test_pick_frequencies_follow_quanta():
    rng = np.random.default_rng(5)
    q = rng.integers(0, 50, size=40).astype(np.uint64)
    q[[0, 7, 39]] = 0
    r64 = rng.integers(0, 2**63, size=40_000, dtype=np.uint64) * 2 + rng.integers(0, 2, size=40_000, dtype=np.uint64)
    picks = np.array([O.spring_pick(q, int(r)) for r in r64])
    counts = np.bincount(picks, minlength=q.size)
    assert np.all(counts[q == 0] == 0)
    p = q.astype(np.float64) / q.sum()
    nz = p > 0
    chi2 = np.sum((counts[nz] - len(r64) * p[nz]) ** 2 / (len(r64) * p[nz]))
    assert stats.chi2.sf(chi2, nz.sum() - 1) > 1e-4


def test_cube_max_matches_dump():
    rng = np.random.default_rng(8)
    d, N, ng = 2, 16, 3
    w0 = rng.gamma(1.0, size=(d, N)) + 0.1
    e = np.concatenate([np.zeros((d, 1)), np.cumsum(w0, axis=1)], axis=1)
    e /= e[:, -1:]
    th = [0.3, 0.6, 0.2]
    M, k = ng**d, 7
    ncall = M * k + 4
    wmax = O.cube_max(O.GAUSS_AXES, e, th, ncall, 11, 2, ng)
    s = O.eval_samples(O.GAUSS_AXES, e, th, ncall, 11, 2, 0, M * k, ng=ng)
    assert np.array_equal(wmax, s["w"].reshape(k, M).max(axis=0))
    # folding a second iteration keeps the larger of the two
    again = O.cube_max(O.GAUSS_AXES, e, th, ncall, 11, 3, ng, wmax.copy())
    s3 = O.eval_samples(O.GAUSS_AXES, e, th, ncall, 11, 3, 0, M * k, ng=ng)
    assert np.array_equal(again, np.maximum(wmax, s3["w"].reshape(k, M).max(axis=0)))


def _trunc_gauss_cdf(x, c, s):
    return (special.erf((x - c) / s) + special.erf(c / s)) / (special.erf((1 - c) / s) + special.erf(c / s))


@pytest.fixture(scope="module")
def gauss2_spring():
    # f = prod_a exp(-(x_a-c_a)^2/s^2)/(s sqrt(pi)) on [0,1]^2: BASES 4 + 3
    # iterations, cube maxima over the integration phase, then 300k trials
    c, s = np.array([0.35, 0.6]), 0.15
    th = list(c) + [s]
    ng, ncall = 8, 8 * 8 * 3000
    run = O.integrate(O.GAUSS_AXES, 2, 32, th, ncall, 4, 21, ng=ng, itmx2=3, cube_max_phase2=True)
    q, unit = O.spring_envelope(run.wmax)
    tr = O.spring_trials(O.GAUSS_AXES, run.edges, th, ng, q, unit, 99, 0, 0, 300_000)
    return dict(c=c, s=s, th=th, ng=ng, edges=run.edges, q=q, unit=unit, tr=tr)


def test_kept_points_follow_the_integrand(gauss2_spring):
    G = gauss2_spring
    tr = G["tr"]
    x = tr["x"][tr["kept"]]
    over = np.mean(tr["w"][tr["kept"]] > tr["env"][tr["kept"]])
    assert over < 2e-3
    assert len(x) > 20_000
    for a in range(2):
        ks = stats.kstest(x[:, a], lambda v: _trunc_gauss_cdf(v, G["c"][a], G["s"]))
        assert ks.pvalue > 1e-4, (a, ks)
    # 2-D cells: the density factorises, so a cell's probability is the
    # product of its marginal probabilities
    cuts = np.linspace(0, 1, 11)
    P = [np.diff(_trunc_gauss_cdf(cuts, G["c"][a], G["s"])) for a in range(2)]
    expect = np.outer(P[0], P[1]) * len(x)
    H, _, _ = np.histogram2d(x[:, 0], x[:, 1], bins=[cuts, cuts])
    m = expect > 20
    chi2 = np.sum((H[m] - expect[m]) ** 2 / expect[m])
    assert stats.chi2.sf(chi2, m.sum() - 1) > 1e-4


def test_keep_rate_is_integral_over_envelope(gauss2_spring):
    G = gauss2_spring
    tr = G["tr"]
    M = G["ng"] ** 2
    env_integral = G["q"].astype(np.float64).sum() * G["unit"] / M
    I = np.prod([0.5 * (special.erf((1 - c) / G["s"]) + special.erf(c / G["s"])) for c in G["c"]])
    p = I / env_integral
    n = len(tr["kept"])
    assert abs(tr["kept"].mean() - p) < 5 * math.sqrt(p * (1 - p) / n)


def test_points_lie_in_their_cube(gauss2_spring):
    G = gauss2_spring
    tr = G["tr"]
    e, ng = G["edges"], G["ng"]
    for a in range(2):
        ca = (tr["cube"] // ng**a) % ng
        # the image of [ca/ng, (ca+1)/ng] under the piecewise-linear map of axis a
        ygrid = np.linspace(0, 1, e.shape[1])
        lo = np.interp(ca / ng, ygrid, e[a])
        hi = np.interp((ca + 1) / ng, ygrid, e[a])
        assert np.all(tr["x"][:, a] >= lo - 1e-15) and np.all(tr["x"][:, a] <= hi + 1e-15)
    # a cube with zero envelope is never chosen
    assert np.all(G["q"][tr["cube"]] > 0)


def test_constant_integrand_keeps_everything():
    ng, d = 4, 2
    e = O.uniform_edges(d, 8)
    wmax = np.full(ng**d, 2.5)
    q, unit = O.spring_envelope(wmax)
    tr = O.spring_trials(O.CONST, e, [2.5], ng, q, unit, 3, 1, 10**10, 20_000)
    assert tr["kept"].all() and np.all(tr["w"] == 2.5) and np.all(tr["env"] == 2.5)
    counts = np.bincount(tr["cube"], minlength=ng**d)
    chi2 = np.sum((counts - 20_000 / ng**d) ** 2 / (20_000 / ng**d))
    assert stats.chi2.sf(chi2, ng**d - 1) > 1e-4
    with pytest.raises(O.OracleError):
        O.spring_trials(O.CONST, e, [2.5], 1, q, unit, 3, 1, 0, 10)  # plain grid: no cubes
