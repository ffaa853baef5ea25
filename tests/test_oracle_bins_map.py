"""Pins for the oracle's uniform, bin index and grid map (step 2 of the
six-step structure, paper Sec. 3.1; the grid of Sec. 2).

The oracle computes the bin index with integer shifts and masks.  The tests
compare it with the real-number definition j = floor(y N), delta = y N - j,
evaluated in exact binary floating point (or exact rationals where a division
by ng is involved), exhaustively over every 23-bit mantissa m where cheap.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

ALL_M = np.arange(1 << 23, dtype=np.uint64)


@pytest.mark.parametrize("nbins", [50, 64, 128, 256, 2])
def test_plain_bin_exhaustive(nbins):
    rng = np.random.default_rng(nbins)
    low = rng.integers(0, 512, size=ALL_M.size, dtype=np.uint64)  # bits the uniform ignores
    words = ((ALL_M << np.uint64(9)) | low).astype(np.uint32)
    j, delta = O.bins_of_words(words, nbins)
    u = (2.0 * ALL_M.astype(np.float64) + 1.0) / 2.0**24  # exact
    yN = u * nbins  # exact: < 2^9 with 24+9 significant bits
    jref = np.floor(yN)
    assert np.array_equal(j, jref.astype(np.int32))
    assert np.array_equal(delta, yN - jref)
    assert delta.min() > 0.0 and delta.max() < 1.0


def test_uniform_range_and_centres():
    assert O.uniform(0) == 2.0**-24
    assert O.uniform(0xFFFFFFFF) == 1.0 - 2.0**-24
    assert O.uniform(0x1FF) == O.uniform(0)  # low 9 bits ignored


@pytest.mark.parametrize("nbins,ng", [(50, 2), (64, 4), (128, 4), (50, 3), (64, 6), (60, 7), (256, (1 << 24) + 3),
                                      (256, (1 << 31) - 1)])
def test_strat_bin_vs_real_definition(nbins, ng):
    rng = np.random.default_rng(1000 * nbins + ng)
    n = 1 << 18
    m = rng.integers(0, 1 << 23, size=n, dtype=np.uint64)
    m[:4] = [0, 1, (1 << 23) - 1, (1 << 23) - 2]
    cc = rng.integers(0, ng, size=n).astype(np.int32)
    words = (m << np.uint64(9)).astype(np.uint32)
    j, delta = O.bins_of_words(words, nbins, ng=ng, cube_coord=cc)
    u = (2.0 * m.astype(np.float64) + 1.0) / 2.0**24
    yN = (cc + u) * nbins / ng  # rounded; exact rationals decide the close calls
    jref = np.floor(yN).astype(np.int64)
    close = np.abs(yN - np.round(yN)) < 1e-9
    for i in np.nonzero(close)[0]:
        q = (Fraction(int(cc[i])) + Fraction(2 * int(m[i]) + 1, 1 << 24)) * nbins / ng
        jref[i] = q.numerator // q.denominator
    assert np.array_equal(j.astype(np.int64), jref)
    c64 = cc.astype(np.int64)
    assert np.all((j >= c64 * nbins // ng) & (j <= ((c64 + 1) * nbins - 1) // ng))
    assert np.allclose(delta, yN - jref, atol=1e-12, rtol=0)


def _random_grid(rng, d, nbins):
    w = rng.gamma(0.5, size=(d, nbins)) + 1e-3
    e = np.concatenate([np.zeros((d, 1)), np.cumsum(w, axis=1)], axis=1)
    e /= e[:, -1:]
    e[:, -1] = 1.0
    return e


def test_uniform_grid_is_identity():
    d, N = 3, 50
    e = O.uniform_edges(d, N)
    rng = np.random.default_rng(1)
    for _ in range(200):
        j = rng.integers(0, N, size=d)
        delta = rng.random(d)
        x, J = O.grid_map(e, j, delta)
        assert np.allclose(x, (j + delta) / N, rtol=0, atol=1e-15)
        assert abs(J - 1.0) < 1e-13


def test_jacobian_integrates_to_one_and_map_is_continuous():
    rng = np.random.default_rng(2)
    d, N = 4, 37
    e = _random_grid(rng, d, N)
    total = np.zeros(d)
    for a in range(d):
        ea = e[a:a + 1]
        s = 0.0
        for jb in range(N):
            _, Ja = O.grid_map(ea, [jb], [0.5])
            s += Ja / N  # int_0^1 J_a(y) dy, J_a constant on each y-bin
            if jb < N - 1:
                x_hi, _ = O.grid_map(ea, [jb], [1.0])
                x_lo, _ = O.grid_map(ea, [jb + 1], [0.0])
                assert x_hi[0] == x_lo[0]
        total[a] = s
    assert np.allclose(total, 1.0, rtol=0, atol=1e-13)


def test_change_of_variables_exact_for_polynomials():
    # int_0^1 g(x(y)) J(y) dy == int_0^1 g(x) dx; x(y) is linear on each y-bin,
    # so 4-point Gauss-Legendre per bin is exact for a degree-5 polynomial g.
    rng = np.random.default_rng(3)
    N = 23
    e = _random_grid(rng, 1, N)
    coef = rng.normal(size=6)
    g = np.polynomial.Polynomial(coef)
    exact = g.integ()(1.0) - g.integ()(0.0)
    xg, wg = np.polynomial.legendre.leggauss(4)
    t = 0.5 * (xg + 1.0)
    acc = 0.0
    for jb in range(N):
        for tk, wk in zip(t, wg):
            x, J = O.grid_map(e, [jb], [tk])
            acc += 0.5 * wk * g(x[0]) * J / N
    assert abs(acc - exact) < 1e-13 * max(1.0, abs(exact))
