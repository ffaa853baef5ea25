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
