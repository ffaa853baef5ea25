"""Pins for the oracle's Gaussian integrands and their parameter gradients.

Closed forms from the configurations: the single Gaussian of the d=4 case and
the double Gaussian of the d=8 case integrate to exactly 1 on the unit cube;
the per-axis Gaussian product integrates to prod_a (1/2)[erf((1-c_a)/s) +
erf(c_a/s)].  The tests integrate the oracle's f with adaptive quadrature
(scipy) or tensor Gauss-Legendre, and differentiate it by central finite
differences, so a dropped factor or a wrong sign in f or in df/dtheta fails.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O


def f1(iid, theta, d=1):
    return lambda x: O.integrand(iid, np.full(d, x) if d == 1 else x, theta)


def test_c1_single_gaussian_normalisation():
    # configuration: exp(-(x-0.5)^2/0.01) / (0.1 sqrt(pi) erf 5) per axis
    th = [0.5, 0.1]
    val, err = integrate.quad(lambda x: O.integrand(O.GAUSS, [x], th), 0, 1, epsabs=1e-14, epsrel=1e-13,
                              points=[0.5], limit=200)
    assert abs(val - 1.0) < 1e-12
    centre = O.integrand(O.GAUSS, [0.5] * 4, th)
    assert abs(centre / (1.0 / (0.1 * math.sqrt(math.pi) * math.erf(5.0))) ** 4 - 1) < 1e-14
    rng = np.random.default_rng(0)
    for _ in range(20):
        x = rng.random(4)
        prod = np.prod([O.integrand(O.GAUSS, [xi], th) for xi in x])
        assert abs(O.integrand(O.GAUSS, x, th) / prod - 1) < 1e-13


def _tensor_gl(fun, d, npts=48, nsub=8):
    """Composite tensor Gauss-Legendre on [0,1]^d (nsub panels per axis)."""
    xg, wg = np.polynomial.legendre.leggauss(npts)
    nodes = ((np.arange(nsub)[:, None] + 0.5 * (xg[None, :] + 1.0)) / nsub).ravel()
    weights = np.tile(0.5 * wg / nsub, nsub)
    tot = 0.0
    for idx in itertools.product(range(nodes.size), repeat=d):
        tot += np.prod(weights[list(idx)]) * fun(nodes[list(idx)])
    return tot


@pytest.mark.parametrize("theta", [[1 / 3, 2 / 3, 0.1], [0.25, 0.6, 0.15]])
def test_double_gaussian_integrates_to_one(theta):
    val, _ = integrate.quad(lambda x: O.integrand(O.DGAUSS, [x], theta), 0, 1, epsabs=1e-14, epsrel=1e-13,
                            points=theta[:2], limit=200)
    assert abs(val - 1.0) < 1e-12
    v2 = _tensor_gl(lambda x: O.integrand(O.DGAUSS, x, theta), 2, npts=24, nsub=6)
    assert abs(v2 - 1.0) < 1e-12


def _axes_closed_form(c, s):
    c = np.asarray(c)
    return np.prod(0.5 * (special.erf((1 - c) / s) + special.erf(c / s)))


def _axes_closed_grad(c, s):
    c = np.asarray(c, dtype=float)
    h = 0.5 * (special.erf((1 - c) / s) + special.erf(c / s))
    dh_dc = (np.exp(-c**2 / s**2) - np.exp(-(1 - c)**2 / s**2)) / (s * np.sqrt(np.pi))
    dh_ds = (-(1 - c) * np.exp(-(1 - c)**2 / s**2) - c * np.exp(-c**2 / s**2)) / (s * s * np.sqrt(np.pi))
    I = np.prod(h)
    return np.concatenate([I * dh_dc / h, [I * np.sum(dh_ds / h)]])


@pytest.mark.parametrize("d,c,s", [(2, [0.3, 0.7], 0.12), (3, [0.2, 0.5, 0.8], 0.2), (2, [0.45, 0.55], 0.05)])
def test_gauss_axes_closed_form_and_gradient(d, c, s):
    th = list(c) + [s]
    val = _tensor_gl(lambda x: O.integrand(O.GAUSS_AXES, x, th), d, npts=20 if d == 3 else 32, nsub=6)
    assert abs(val - _axes_closed_form(c, s)) < 1e-12
    if d == 2:
        gq = _tensor_gl(lambda x: O.integrand(O.GAUSS_AXES, x, th, want_grad=True)[1], d, npts=32, nsub=6)
        assert np.allclose(gq, _axes_closed_grad(c, s), rtol=0, atol=1e-11)


@pytest.mark.parametrize("iid,theta,d", [
    (O.GAUSS, [0.5, 0.1], 4),
    (O.GAUSS, [0.3, 0.2], 3),
    (O.DGAUSS, [1 / 3, 2 / 3, 0.1], 8),
    (O.GAUSS_AXES, [0.2, 0.4, 0.6, 0.8, 0.1], 4),
    (O.CONST, [2.5], 3),
])
def test_parameter_gradient_vs_central_difference(iid, theta, d):
    rng = np.random.default_rng(11)
    th = np.array(theta, dtype=float)
    for _ in range(25):
        x = np.clip(th[0] + 0.15 * rng.normal(size=d), 0.01, 0.99) if iid != O.CONST else rng.random(d)
        f, g = O.integrand(iid, x, th, want_grad=True)
        for p in range(g.size):
            h = 1e-6 * max(1.0, abs(th[p]))
            tp, tm = th.copy(), th.copy()
            tp[p] += h
            tm[p] -= h
            fd = (O.integrand(iid, x, tp) - O.integrand(iid, x, tm)) / (2 * h)
            scale = max(abs(fd), abs(f) * 1e-3, 1e-300)
            assert abs(g[p] - fd) <= 1e-5 * scale + 1e-12 * abs(f) / h


def test_double_gaussian_gradient_of_integral_vanishes():
    # I(theta) = 1 for every theta, so the integral of df/dtheta is 0
    th = [0.3, 0.65, 0.12]
    gq = _tensor_gl(lambda x: O.integrand(O.DGAUSS, x, th, want_grad=True)[1], 2, npts=32, nsub=6)
    assert np.allclose(gq, 0.0, atol=1e-11)


def test_param_counts_and_unknown_integrand():
    assert O.nparams(O.GAUSS, 4) == 2
    assert O.nparams(O.DGAUSS, 8) == 3
    assert O.nparams(O.GAUSS_AXES, 7) == 8
    assert O.nparams(O.WJETS, 10) == 7
    assert O.ngrad(O.WJETS, 16) == 3
    assert O.nparams(99, 4) < 0
    assert math.isnan(O.integrand(99, [0.5], [1.0]))
