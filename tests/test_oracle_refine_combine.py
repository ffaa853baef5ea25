"""Pins for the oracle's grid refinement (step 5 of the six-step structure,
paper Sec. 3.1; grid spacing re-defined from the per-bin variance
information, Sec. 2) and for the combination of iterations.

Refinement pins: invariants (edges strictly increasing from 0 to 1, bins
partition [0,1]), fixed points (uniform weights; alpha = 0; an all-zero axis),
and the defining property that every new bin carries the same share of the
damped weight -- checked by integrating a step density computed here in an
independent matrix form.
Combination pins: hand-worked numbers and numpy's weighted average.
"""
import math

import numpy as np
import pytest

import oracle as O


def _random_grid(rng, d, nbins):
    w = rng.gamma(0.7, size=(d, nbins)) + 1e-3
    e = np.concatenate([np.zeros((d, 1)), np.cumsum(w, axis=1)], axis=1)
    e /= e[:, -1:]
    e[:, -1] = 1.0
    return e


def _damped_weights(b2, alpha):
    """Smoothing as a tridiagonal matrix (3-point mean, 2-point at the
    ends), then r = ((1-rho)/(-ln rho))^alpha with its limits at 0 and 1."""
    N = b2.size
    A = np.zeros((N, N))
    for i in range(N):
        lo, hi = max(i - 1, 0), min(i + 1, N - 1)
        A[i, lo:hi + 1] = 1.0 / (hi - lo + 1)
    dbar = A @ b2
    rho = dbar / dbar.sum()
    with np.errstate(divide="ignore", invalid="ignore"):
        base = np.where(rho > 0, (1.0 - rho) / -np.log(rho), 0.0)
        base = np.where(rho >= 1, 1.0, base)
    return base**alpha


@pytest.mark.parametrize("N,alpha", [(4, 1.5), (50, 1.5), (128, 0.5), (64, 2.0), (256, 1.5)])
def test_refine_equal_damped_weight_per_new_bin(N, alpha):
    rng = np.random.default_rng(N)
    d = 3
    e = _random_grid(rng, d, N)
    b2 = rng.gamma(0.3, size=(d, N))
    b2[1, : N // 3] = 0.0  # empty stretch
    out = O.refine(e, b2, alpha)
    for a in range(d):
        r = _damped_weights(b2[a], alpha)
        dens = r / np.diff(e[a])  # density of damped weight on the old bins
        cum_old = np.concatenate([[0.0], np.cumsum(r)])

        def W(x):  # damped weight to the left of x
            j = np.clip(np.searchsorted(e[a], x, side="right") - 1, 0, N - 1)
            return cum_old[j] + dens[j] * (x - e[a][j])

        shares = np.diff([W(x) for x in out[a]])
        assert np.allclose(shares, cum_old[-1] / N, rtol=1e-10, atol=1e-12 * cum_old[-1])


@pytest.mark.parametrize("N", [2, 3, 50, 128])
def test_refine_invariants(N):
    rng = np.random.default_rng(7 + N)
    e = _random_grid(rng, 4, N)
    b2 = rng.random((4, N)) ** 4
    out = O.refine(e, b2, 1.5)
    assert np.all(out[:, 0] == 0.0) and np.all(out[:, -1] == 1.0)
    assert np.all(np.diff(out, axis=1) > 0)
    assert np.allclose(np.diff(out, axis=1).sum(axis=1), 1.0, atol=1e-15)


def test_refine_fixed_points():
    N = 50
    e = O.uniform_edges(2, N)
    out = O.refine(e, np.ones((2, N)) * 3.7, 1.5)
    assert np.allclose(out, e, atol=2e-15, rtol=0)
    rng = np.random.default_rng(1)
    e2 = _random_grid(rng, 2, N)
    b2 = rng.random((2, N))
    assert np.allclose(O.refine(e2, b2, 0.0), e2, atol=2e-15, rtol=0)  # alpha = 0
    b2[1] = 0.0
    out = O.refine(e2, b2, 1.5)
    assert np.array_equal(out[1], e2[1])  # all-zero axis left alone
    assert not np.allclose(out[0], e2[0])


def test_refine_concentrates_bins_where_weight_is():
    N = 4
    e = O.uniform_edges(1, N)
    out = O.refine(e, np.array([[1.0, 1.0, 1.0, 5.0]]), 1.5)
    w = np.diff(out[0])
    assert w[3] < w[0] and w[3] < w[1]  # heavy bin narrowed
    assert np.all(np.diff(out[0]) > 0)


# Hand-worked refinements.  Each case writes out, for its own numbers, the
# steps of the classic VEGAS re-binning (Lepage 1978): 3-point smoothing of
# the per-bin sums of w^2 (2-point at the ends), normalisation to rho_j,
# damping r_j = ((1 - rho_j) / (-ln rho_j))^alpha, and new edges that cut the
# piecewise-constant density r_j / width_j into N pieces of equal weight T.
# The bin each new edge falls into was located by hand from the cumulative
# sums, and the rounded values were computed on paper as a check on the
# arithmetic below.
def _hand_case_a():
    """N = 4, uniform edges, sums of w^2 (1, 1, 1, 5), alpha = 1.5."""
    # smoothed: (1+1)/2, (1+1+1)/3, (1+1+5)/3, (1+5)/2 = 1, 1, 7/3, 3; sum 22/3
    # rho = 3/22, 3/22, 7/22, 9/22
    r1 = ((19 / 22) / math.log(22 / 3)) ** 1.5   # bins 0 and 1
    r7 = ((15 / 22) / math.log(22 / 7)) ** 1.5   # bin 2
    r9 = ((13 / 22) / math.log(22 / 9)) ** 1.5   # bin 3
    T = (2 * r1 + r7 + r9) / 4
    # cumulative sums 0, r1, 2 r1, 2 r1 + r7, 2 r1 + r7 + r9:
    # T lies in bin 1, 2T in bin 2, 3T in bin 3
    e1 = 0.25 + (T - r1) / r1 * 0.25
    e2 = 0.50 + (2 * T - 2 * r1) / r7 * 0.25
    e3 = 0.75 + (3 * T - 2 * r1 - r7) / r9 * 0.25
    return (np.array([0.0, 0.25, 0.5, 0.75, 1.0]), np.array([1.0, 1.0, 1.0, 5.0]), 1.5,
            np.array([0.0, e1, e2, e3, 1.0]), (0.34334, 0.61596, 0.81772))


def _hand_case_b():
    """N = 3, edges (0, 0.5, 0.75, 1), sums of w^2 (4, 1, 1), alpha = 1."""
    # smoothed: (4+1)/2, (4+1+1)/3, (1+1)/2 = 5/2, 2, 1; sum 11/2
    # rho = 5/11, 4/11, 2/11
    r0 = (6 / 11) / math.log(11 / 5)
    r1 = (7 / 11) / math.log(11 / 4)
    r2 = (9 / 11) / math.log(11 / 2)
    T = (r0 + r1 + r2) / 3
    # cumulative sums 0, r0, r0 + r1, r0 + r1 + r2: T in bin 0, 2T in bin 1
    e1 = 0.0 + T / r0 * 0.5
    e2 = 0.5 + (2 * T - r0) / r1 * 0.25
    return (np.array([0.0, 0.5, 0.75, 1.0]), np.array([4.0, 1.0, 1.0]), 1.0, np.array([0.0, e1, e2, 1.0]),
            (0.433847, 0.702181))


def _hand_case_c():
    """N = 4, uniform edges, sums of w^2 (0, 0, 0, 8), alpha = 1: the first
    two smoothed sums are zero, so no new edge may land in those bins."""
    # smoothed: 0, 0, 8/3, 4; sum 20/3; rho = 0, 0, 2/5, 3/5; r = 0 at rho = 0
    r2 = (3 / 5) / math.log(5 / 2)
    r3 = (2 / 5) / math.log(5 / 3)
    T = (r2 + r3) / 4
    # cumulative sums 0, 0, 0, r2, r2 + r3: T in bin 2, 2T and 3T in bin 3
    e1 = 0.50 + T / r2 * 0.25
    e2 = 0.75 + (2 * T - r2) / r3 * 0.25
    e3 = 0.75 + (3 * T - r2) / r3 * 0.25
    return (np.array([0.0, 0.25, 0.5, 0.75, 1.0]), np.array([0.0, 0.0, 0.0, 8.0]), 1.0,
            np.array([0.0, e1, e2, e3, 1.0]), (0.637238, 0.770470, 0.885236))


HAND_CASES = {"a": _hand_case_a, "b": _hand_case_b, "c": _hand_case_c}


@pytest.mark.parametrize("name", sorted(HAND_CASES))
def test_refine_hand_worked(name):
    edges, b2, alpha, want, paper_values = HAND_CASES[name]()
    # the arithmetic above reproduces the values worked out on paper
    assert np.allclose(want[1:-1], paper_values, atol=2e-6), want
    got = O.refine(edges[None, :], b2[None, :], alpha)[0]
    assert np.max(np.abs(got - want)) <= 1e-14, (got, want)


def test_refine_rejects_bad_arguments():
    with pytest.raises(O.OracleError):
        O.refine(O.uniform_edges(1, 4), np.ones((1, 4)), -1.0)
    with pytest.raises(O.OracleError):
        O.refine(O.uniform_edges(1, 1), np.ones((1, 1)), 1.5)


def test_combine_hand_worked():
    Ib, sb, chi = O.combine([1.0, 3.0], [1.0, 1.0])
    assert Ib == 2.0 and abs(sb - 1 / math.sqrt(2)) < 1e-16 and chi == 2.0
    Ib, sb, chi = O.combine([1.0, 2.0], [1.0, 4.0])
    # weights 1 and 1/4: mean (1 + 0.5)/1.25 = 1.2; chi2 = 0.04 + 0.64/4 = 0.2
    assert abs(Ib - 1.2) < 1e-15 and abs(sb - math.sqrt(1 / 1.25)) < 1e-15 and abs(chi - 0.2) < 1e-15


def test_combine_vs_numpy_weighted_average():
    rng = np.random.default_rng(3)
    I = 1 + 0.01 * rng.normal(size=12)
    var = (0.01 * rng.random(12) + 0.001) ** 2
    Ib, sb, chi = O.combine(I, var)
    assert abs(Ib - np.average(I, weights=1 / var)) < 1e-14
    assert abs(sb - np.sum(1 / var) ** -0.5) < 1e-16
    ref = np.sum((I - np.average(I, weights=1 / var)) ** 2 / var) / 11
    assert abs(chi / ref - 1) < 1e-12


def test_combine_exact_and_single():
    Ib, sb, chi = O.combine([2.0, 4.0, 7.0], [0.0, 0.0, 1.0])
    assert Ib == 3.0 and sb == 0.0
    Ib, sb, chi = O.combine([5.0], [4.0])
    assert Ib == 5.0 and sb == 2.0 and math.isnan(chi)
