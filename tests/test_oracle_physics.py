"""Pins for the oracle's physics-shaped integrand: massless phase space,
acceptance cuts, colour-ordered denominators and the Breit-Wigner factor.

The paper's process is u dbar -> W+(-> mu+ nu) + n gluons with a 3(n+2)-4
dimensional phase space plus 2 PDF dimensions (Sec. 5).  The toy keeps that
shape.  Pins used here:
  * textbook massless phase-space volumes V_2 = 1/(8 pi), V_3 = s/(256 pi^3);
  * momentum conservation, masslessness and sum_{i<j} s_ij = s per event;
  * distributions equal to those of classic RAMBO (Kleiss-Stirling-Ellis),
    implemented independently below in numpy, by two-sample KS tests;
  * the flat 3-body Dalitz density;
  * the 4-parton cyclic sum closed form (s^2+t^2+u^2)/(s^2 t^2 u^2);
  * exact coupling scaling and a unit-normalised Breit-Wigner;
  * the PDF x phase-space integral against 2-D adaptive quadrature.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O

G_DEFAULT = math.sqrt(4 * math.pi * 0.118)
THETA = [80.4, 2.1, G_DEFAULT, 14000.0, 20.0, 2.5, 0.4]


def minkowski(a, b):
    return a[..., 0] * b[..., 0] - np.sum(a[..., 1:] * b[..., 1:], axis=-1)


def test_phase_space_volumes():
    assert abs(O.ps_volume(2, 123.0) - 1 / (8 * math.pi)) < 1e-16
    s = 7.5e5
    assert abs(O.ps_volume(3, s) / (s / (256 * math.pi**3)) - 1) < 1e-14
    # recursion V_n(s) = int dM^2/(2pi) V_2(s; M) V_{n-1}(M^2), V_2 with one massive = (1-M^2/s)/(8pi)
    for n in (3, 4, 5, 6):
        val, _ = integrate.quad(lambda m2: (1 - m2 / s) / (8 * math.pi) * O.ps_volume(n - 1, m2) / (2 * math.pi),
                                0, s, epsrel=1e-12)
        assert abs(val / O.ps_volume(n, s) - 1) < 1e-10


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_rambo_diet_event_invariants(n):
    rng = np.random.default_rng(n)
    rs = 1234.5
    for _ in range(200):
        p, w = O.rambo_diet(n, rs, rng.random(3 * n - 4))
        assert abs(w - O.ps_volume(n, rs * rs)) <= 1e-15 * abs(w)
        tot = p.sum(axis=0)
        assert np.allclose(tot, [rs, 0, 0, 0], rtol=0, atol=1e-9 * rs)
        assert np.all(np.abs(minkowski(p, p)) < 1e-9 * rs * rs)
        sij = sum(2 * minkowski(p[i], p[k]) for i in range(n) for k in range(i + 1, n))
        assert abs(sij - rs * rs) < 1e-9 * rs * rs


def test_mass_fraction_solve():
    rng = np.random.default_rng(5)
    for n in (4, 6):
        for i in range(2, n):
            k = n - i
            for r in rng.random(20):
                t = O.solve_mass_fraction(n, i, r)
                F = (k + 1) * t**k - k * t**(k + 1)
                assert abs(F - r) < 1e-14
                if k == 1:
                    assert abs(t - (1 - math.sqrt(1 - r))) < 1e-14


def classic_rambo(n, rs, rng, nev):
    """Kleiss-Stirling-Ellis RAMBO (massless): isotropic q with energy
    density q e^-q, then a conformal boost to the total-momentum frame."""
    c = 2 * rng.random((nev, n)) - 1
    phi = 2 * np.pi * rng.random((nev, n))
    q0 = -np.log(rng.random((nev, n)) * rng.random((nev, n)))
    s = np.sqrt(1 - c * c)
    q = np.stack([q0, q0 * s * np.cos(phi), q0 * s * np.sin(phi), q0 * c], axis=-1)
    Q = q.sum(axis=1)
    M = np.sqrt(minkowski(Q, Q))
    b = -Q[:, 1:] / M[:, None]
    x = rs / M
    gam = Q[:, 0] / M
    a = 1 / (1 + gam)
    bq = np.einsum("ej,enj->en", b, q[..., 1:])
    p = np.empty_like(q)
    p[..., 0] = x[:, None] * (gam[:, None] * q[..., 0] + bq)
    p[..., 1:] = x[:, None, None] * (q[..., 1:] + b[:, None, :] * (q[..., 0:1] + a[:, None, None] * bq[..., None]))
    return p


@pytest.mark.parametrize("n", [3, 4, 6])
def test_rambo_diet_matches_classic_rambo(n):
    rng = np.random.default_rng(100 + n)
    rs = 1000.0
    nev = 4000
    diet = np.array([O.rambo_diet(n, rs, rng.random(3 * n - 4))[0] for _ in range(nev)])
    ref = classic_rambo(n, rs, rng, nev)
    # RAMBO is symmetric in the particles; compare symmetrised observables
    for obs in (lambda p: 2 * minkowski(p[:, 0], p[:, 1]),
                lambda p: 2 * minkowski(p[:, 0], p[:, n - 1]),
                lambda p: 2 * minkowski(p[:, n - 2], p[:, n - 1]),
                lambda p: p[:, 0, 0],
                lambda p: p[:, n - 1, 3] / p[:, n - 1, 0],
                lambda p: np.hypot(p[:, 1, 1], p[:, 1, 2])):
        res = stats.ks_2samp(obs(diet), obs(ref[:, rng.permutation(n)]))
        assert res.pvalue > 1e-4


def test_three_body_dalitz_is_flat():
    rng = np.random.default_rng(9)
    rs = 100.0
    s12, s23 = [], []
    for _ in range(20000):
        p, _ = O.rambo_diet(3, rs, rng.random(5))
        s12.append(2 * minkowski(p[0], p[1]))
        s23.append(2 * minkowski(p[1], p[2]))
    s12 = np.array(s12) / rs**2
    s23 = np.array(s23) / rs**2
    # uniform on the triangle s12 + s23 <= 1: s12 marginal density 2(1 - s12)
    u = 1 - (1 - s12) ** 2
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    # conditional on s12, s23 uniform on [0, 1-s12]
    v = s23 / (1 - s12)
    assert stats.kstest(v, "uniform").pvalue > 1e-4


def test_mean_invariants():
    rng = np.random.default_rng(21)
    n, rs = 5, 50.0
    acc = np.zeros((n, n))
    nev = 6000
    for _ in range(nev):
        p, _ = O.rambo_diet(n, rs, rng.random(3 * n - 4))
        acc += 2 * minkowski(p[:, None, :], p[None, :, :])
    mean = acc / nev / rs**2
    iu = np.triu_indices(n, 1)
    # symmetric phase space: <s_ij> = s / C(n, 2)
    assert np.allclose(mean[iu], 1 / math.comb(n, 2), atol=0.01)


def test_cycle_counts_and_four_point_closed_form():
    assert [O.num_cycles(m) for m in (3, 4, 5, 6)] == [1, 3, 12, 60]
    rng = np.random.default_rng(4)
    for _ in range(20):
        s, t, u = rng.random(3) * 100 + 1
        S = np.array([[0, s, u, t], [s, 0, t, u], [u, t, 0, s], [t, u, s, 0]], dtype=float)
        ref = (s * s + t * t + u * u) / (s * s * t * t * u * u)
        assert abs(O.cyclic_sum(S) / ref - 1) < 1e-13


def test_cyclic_sum_is_permutation_symmetric_and_matches_brute_force():
    import itertools
    rng = np.random.default_rng(6)
    for m in (5, 6):
        A = rng.random((m, m)) + 0.1
        S = A + A.T
        np.fill_diagonal(S, 0)
        base = O.cyclic_sum(S)
        for _ in range(5):
            perm = rng.permutation(m)
            assert abs(O.cyclic_sum(S[np.ix_(perm, perm)]) / base - 1) < 1e-13
        # brute force over all m! orders: every distinct cycle appears 2m times
        tot = 0.0
        for o in itertools.permutations(range(m)):
            tot += 1.0 / np.prod([S[o[i], o[(i + 1) % m]] for i in range(m)])
        assert abs(tot / (2 * m) / base - 1) < 1e-12


def _event(pts, etas, phis):
    p = []
    for pt, eta, phi in zip(pts, etas, phis):
        p.append([pt * math.cosh(eta), pt * math.cos(phi), pt * math.sin(phi), pt * math.sinh(eta)])
    return np.array(p)


def test_cuts_thresholds():
    eps = 1e-9
    # n_p = 2: partons 0,1, electron 2, neutrino 3 (unconstrained)
    base = dict(pts=[50, 60, 40, 5], etas=[0.0, 1.0, -1.0, 4.9], phis=[0.0, 2.0, 4.0, 1.0])

    def ok(**kw):
        d = {k: list(v) for k, v in base.items()}
        yb = kw.pop("yb", 0.0)
        for k, (i, v) in kw.items():
            d[k][i] = v
        return O.pass_cuts(2, _event(d["pts"], d["etas"], d["phis"]), yb, 20.0, 2.5, 0.4)

    assert ok()
    assert ok(pts=(0, 20 + eps)) and not ok(pts=(0, 20 - eps))
    assert ok(pts=(2, 20 + eps)) and not ok(pts=(2, 20 - eps))
    assert ok(etas=(2, -2.5 + eps)) and not ok(etas=(2, -2.5 - eps))
    assert ok(etas=(1, 2.5 - eps)) and not ok(etas=(1, 2.5 + eps))
    # lab rapidity = CM rapidity + boost
    assert ok(etas=(1, 2.0), yb=0.5 - eps) and not ok(etas=(1, 2.0), yb=0.5 + eps)
    # Delta R between parton 0 (eta 0, phi 0) and parton 1, phi wrap-around
    assert ok(etas=(1, 0.0), phis=(1, 0.4 + eps)) and not ok(etas=(1, 0.0), phis=(1, 0.4 - eps))
    assert not ok(etas=(1, 0.0), phis=(1, 2 * math.pi - 0.4 + eps))
    assert ok(etas=(1, 0.0), phis=(1, -0.4 - eps))
    # electron-parton separation counts; the neutrino does not
    assert not ok(etas=(2, 0.0), phis=(2, 0.1))
    assert ok(etas=(3, 0.0), phis=(3, 0.0))


def _random_points(d, n, rng):
    return rng.random((n, d))


@pytest.mark.parametrize("d", [10, 16])
def test_wjets_coupling_scaling_and_bw_derivatives(d):
    rng = np.random.default_rng(d)
    n_p = (d - 4) // 3
    found = 0
    for x in _random_points(d, 3000, rng):
        ev = O.wjets_event(x, THETA, want_grad=True)
        if ev["f"] == 0:
            continue
        found += 1
        th2 = list(THETA)
        th2[2] = 2.0 * THETA[2]
        f2 = O.integrand(O.WJETS, x, th2)
        assert abs(f2 / ev["f"] / 2.0 ** (2 * n_p) - 1) < 1e-13
        g = ev["grad"]
        assert abs(THETA[2] * g[2] / ev["f"] - 2 * n_p) < 1e-13
        for p in (0, 1):
            h = 1e-6 * THETA[p]
            tp, tm = list(THETA), list(THETA)
            tp[p] += h
            tm[p] -= h
            fd = (O.integrand(O.WJETS, x, tp) - O.integrand(O.WJETS, x, tm)) / (2 * h)
            assert abs(fd - g[p]) <= 1e-6 * abs(ev["f"]) / THETA[p] * 100 + 1e-7 * abs(g[p])
        if found >= 30:
            break
    assert found >= 10


def _bw(m2, M, G):
    # unit-normalised over m^2: int bw dm^2 = 1
    return (M * G / math.pi) / ((m2 - M * M) ** 2 + M * M * G * G)


def test_breit_wigner_reference_is_unit_normalised():
    lo, _ = integrate.quad(lambda m2: _bw(m2, 80.4, 2.1), -np.inf, 80.4**2, limit=400, epsabs=1e-13)
    hi, _ = integrate.quad(lambda m2: _bw(m2, 80.4, 2.1), 80.4**2, np.inf, limit=400, epsabs=1e-13)
    assert abs(lo + hi - 1) < 1e-8


def _accepted_points(d, rng, want):
    out = []
    for x in rng.random((20000, d)):
        if O.integrand(O.WJETS, x, THETA) > 0:
            out.append(x)
            if len(out) == want:
                break
    return out


@pytest.mark.parametrize("d", [10, 16])
def test_wjets_mass_and_width_dependence_is_the_breit_wigner(d):
    rng = np.random.default_rng(3 * d)
    for x in _accepted_points(d, rng, 15):
        ev = O.wjets_event(x, THETA)
        for M2, G2 in ((75.0, 2.1), (80.4, 0.7), (91.2, 2.5)):
            th = list(THETA)
            th[0], th[1] = M2, G2
            ratio = O.integrand(O.WJETS, x, th) / ev["f"]
            ref = _bw(ev["m2"], M2, G2) / _bw(ev["m2"], THETA[0], THETA[1])
            assert abs(ratio / ref - 1) < 1e-12


@pytest.mark.parametrize("d", [10, 16])
def test_wjets_is_product_of_pinned_factors(d):
    """f = [PDF x phase-space part] x g^(2 n_p) x BW x 2 s^4 x cyclic sum,
    each factor pinned on its own (quadrature, closed forms, RAMBO)."""
    rng = np.random.default_rng(5 * d)
    n_p = (d - 4) // 3
    for x in _accepted_points(d, rng, 15):
        ev = O.wjets_event(x, THETA)
        ps = O.integrand(O.PSVOL, x, [14000.0, 20.0])
        rs = math.sqrt(ev["shat"])
        mom = [np.array([rs / 2, 0, 0, rs / 2]), np.array([rs / 2, 0, 0, -rs / 2])] + list(ev["p"][:n_p])
        m = len(mom)
        S = np.array([[0.0 if i == k else 2 * minkowski(mom[i], mom[k]) for k in range(m)] for i in range(m)])
        ref = ps * THETA[2] ** (2 * n_p) * _bw(ev["m2"], THETA[0], THETA[1]) * 2 * ev["shat"] ** 4 * O.cyclic_sum(S)
        assert abs(ev["f"] / ref - 1) < 1e-12


def test_wjets_event_kinematics():
    rng = np.random.default_rng(77)
    for d in (10, 16):
        n = (d - 4) // 3 + 2
        for x in rng.random((50, d)):
            ev = O.wjets_event(x, THETA)
            assert ev["x1"] * ev["x2"] >= ((1 + n - 2) * 20.0) ** 2 / 14000.0**2 * (1 - 1e-12)
            assert abs(ev["shat"] - ev["x1"] * ev["x2"] * 14000.0**2) < 1e-6 * ev["shat"]
            p = ev["p"]
            assert np.allclose(p.sum(0), [math.sqrt(ev["shat"]), 0, 0, 0], atol=1e-7 * math.sqrt(ev["shat"]))
            pe, pn = p[n - 2], p[n - 1]
            assert abs(ev["m2"] - 2 * minkowski(pe, pn)) < 1e-9 * ev["shat"]


@pytest.mark.slow
@pytest.mark.parametrize("d", [10])
def test_pdf_times_phase_space_vs_quadrature(d):
    """MC estimate of int dx1 dx2 F(x1) F(x2) V_n(x1 x2 S)/(2 x1 x2 S) over
    x1 x2 > tau0 (no cuts, |M|^2 = 1) against 2-D adaptive quadrature."""
    n_p = (d - 4) // 3
    n = n_p + 2
    S = 14000.0**2
    tau0 = ((1 + n_p) * 20.0) ** 2 / S
    F = lambda x: x**-1.5 * (1 - x) ** 3

    def integrand(l2, l1):  # over ln x1, ln x2
        x1, x2 = math.exp(l1), math.exp(l2)
        return x1 * x2 * F(x1) * F(x2) * O.ps_volume(n, x1 * x2 * S) / (2 * x1 * x2 * S)

    L = math.log(tau0)
    ref, err = integrate.dblquad(integrand, L, 0, lambda l1: L - l1, lambda l1: 0.0, epsrel=1e-10)
    run = O.integrate(O.PSVOL, d, 64, [14000.0, 20.0], 40000, 8, 4321)
    assert abs(run.Ibar - ref) / run.sigbar < 4
