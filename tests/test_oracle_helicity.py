"""Pins for the oracle's helicity-amplitude integrand u dbar -> W+(-> mu+ nu)
+ n gluons (paper Sec. 5, eq. 1 and Table 4; n <= 2).

The oracle builds the amplitudes from 2-component Weyl spinor chains and
colour-ordered partial amplitudes.  The brute force here shares none of
that: 4x4 Dirac matrices in the Dirac basis, fermion spins summed by traces
(sum u ubar = pslash), the three-gluon vertex transcribed from the Feynman
rule with all momenta incoming, explicit linear gluon polarisations in a
frame of its own, and the colour sum from explicit SU(3) generators
(Gell-Mann / 2, f^abc from commutators).  Also pinned: the Ward identity
(a gluon polarisation replaced by its momentum), gauge shifts of the
polarisations, Lorentz invariance of the helicity sum, the cuts on
hand-built events, and the integrand as the product of its factors.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle as O

dp = ctypes.POINTER(ctypes.c_double)
GF, MWREF = 1.1663787e-5, 80.4
THETA = np.array([80.4, 2.1, math.sqrt(4 * math.pi * 0.118), 14000.0, 20.0, 2.5, 5.0, 20.0])


def _lib():
    L = O.lib()
    L.orc_whel_partials.argtypes = [ctypes.c_int, dp, dp, dp]
    L.orc_whel_me2.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp]
    L.orc_whel_me2.restype = ctypes.c_double
    L.orc_whel_pass_cuts.argtypes = [ctypes.c_int, dp] + [ctypes.c_double] * 5
    L.orc_whel_event.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, dp]
    L.orc_whel_event.restype = ctypes.c_double
    return L


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(dp)


# ---------------------------------------------------------------- kinematics
def _massless(rng, E):
    c = rng.uniform(-1, 1)
    ph = rng.uniform(0, 2 * math.pi)
    s = math.sqrt(1 - c * c)
    return E * np.array([1.0, s * math.cos(ph), s * math.sin(ph), c])


def _event(rng, n, rs=500.0):
    """pu, pd along +-z, and n+2 massless outgoing momenta summing to them
    (random directions, then a common rescaling in the rest frame)."""
    while True:
        ks = [_massless(rng, rng.uniform(0.3, 1.0)) for _ in range(n + 2)]
        P = np.sum(ks, axis=0)
        M = math.sqrt(P[0] ** 2 - P[1:] @ P[1:])
        b = -P[1:] / P[0]
        g = 1 / math.sqrt(1 - b @ b)
        out = []
        for k in ks:  # boost to the rest frame of P, then scale to sqrt(s) = rs
            bp = b @ k[1:]
            e = g * (k[0] + bp)
            v = k[1:] + ((g - 1) * bp / (b @ b) + g * k[0]) * b
            out.append(np.concatenate([[e], v]) * rs / M)
        pu = np.array([rs / 2, 0, 0, rs / 2])
        pd = np.array([rs / 2, 0, 0, -rs / 2])
        mom = np.concatenate([pu, pd] + out)
        if all(o[0] > 5 for o in out):
            return mom


def _mdot(a, b):
    return a[0] * b[0] - a[1:] @ b[1:]


# ---------------------------------------------------------------- brute force
s1 = np.array([[0, 1], [1, 0]], complex)
s2 = np.array([[0, -1j], [1j, 0]], complex)
s3 = np.array([[1, 0], [0, -1]], complex)
Z2, I2 = np.zeros((2, 2), complex), np.eye(2, dtype=complex)
G0 = np.block([[I2, Z2], [Z2, -I2]])
GI = [np.block([[Z2, s], [-s, Z2]]) for s in (s1, s2, s3)]
GAM = [G0] + GI                      # gamma^mu, Dirac basis
G5 = np.block([[Z2, I2], [I2, Z2]])
PL = (np.eye(4) - G5) / 2
METRIC = np.diag([1.0, -1.0, -1.0, -1.0])


def slash(a):
    a = np.asarray(a)
    return a[0] * GAM[0] - a[1] * GAM[1] - a[2] * GAM[2] - a[3] * GAM[3]


def bar(M):
    return G0 @ M.conj().T @ G0


def _gellmann():
    l = np.zeros((8, 3, 3), complex)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7] = np.diag([1, 1, -2]) / math.sqrt(3)
    T = l / 2
    f = np.zeros((8, 8, 8))
    for a in range(8):
        for b in range(8):
            C = T[a] @ T[b] - T[b] @ T[a]
            for c in range(8):
                f[a, b, c] = (-2j * np.trace(C @ T[c])).real
    return T, f


TGEN, FABC = _gellmann()


def colour_matrix(n):
    """Col[c, c'] = sum over all colours of c_c conj(c_c') for the colour
    structures: n=0 delta_ji; n=1 T^a_ji; n=2 (T^a1 T^a2)_ji, (T^a2 T^a1)_ji,
    (f^{a1 a2 b} T^b)_ji.  Hermitian, complex off the (T T) block."""
    if n == 0:
        return np.array([[3.0]])
    if n == 1:
        return np.array([[sum(np.sum(np.abs(TGEN[a]) ** 2) for a in range(8))]])
    C = np.zeros((3, 3), complex)
    for a in range(8):
        for b in range(8):
            fT = np.einsum("c,cij->ij", FABC[a, b], TGEN)
            st = [TGEN[a] @ TGEN[b], TGEN[b] @ TGEN[a], fT]
            for i in range(3):
                for k in range(3):
                    C[i, k] += np.sum(st[i] * st[k].conj())
    return C


def transverse_pols(k, shift):
    """Two real linear polarisations of k in a frame of their own, plus
    `shift` k / |k| (a gauge change)."""
    kh = k[1:] / np.linalg.norm(k[1:])
    r = np.array([0.37, -0.81, 0.45])
    ea = r - (r @ kh) * kh
    ea /= np.linalg.norm(ea)
    eb = np.cross(kh, ea)
    return [np.concatenate([[0.0], e]) + shift * k / k[0] for e in (ea, eb)]


def brute_me2(n, mom, theta, shift=0.0):
    """sum over spins, gluon polarisations and colours of |M|^2."""
    M, Gam, gs = theta[:3]
    gw = math.sqrt(4 * math.sqrt(2) * GF * MWREF ** 2)
    pu, pd = mom[0:4], mom[4:8]
    ks = [mom[8 + 4 * i:12 + 4 * i] for i in range(n)]
    pmu, pnu = mom[8 + 4 * n:12 + 4 * n], mom[12 + 4 * n:16 + 4 * n]
    q = pmu + pnu
    Dw = _mdot(q, q) - M * M + 1j * M * Gam

    def prop(P):
        return 1j * slash(P) / _mdot(P, P)

    Wv = [1j * gw / math.sqrt(2) * GAM[r] @ PL for r in range(4)]  # W vertex, upper index rho
    # lepton line traces Lep[rho, rho'] = Tr[G_rho pslash_mu bar(G_rho') pslash_nu], G_rho lower index
    Glep = [1j * gw / math.sqrt(2) * (METRIC[r, r] * GAM[r]) @ PL for r in range(4)]
    Lep = np.array([[np.trace(Glep[r] @ slash(pmu) @ bar(Glep[s]) @ slash(pnu)) for s in range(4)]
                    for r in range(4)])
    Wprop = -1j / Dw  # times g_{rho sigma}: the lower-index lepton vertex carries the metric
    Col = colour_matrix(n)
    total = 0.0
    pol_sets = [[]] if n == 0 else (
        [[e] for e in transverse_pols(ks[0], shift)] if n == 1 else
        [[e1, e2] for e1 in transverse_pols(ks[0], shift) for e2 in transverse_pols(ks[1], -0.6 * shift)])
    for eps in pol_sets:
        gv = [1j * gs * slash(np.conj(e)) for e in eps]  # outgoing gluon: conj(eps)
        struct = []  # per colour structure: Gamma^rho (4 of them)

        def line(seq):
            """seq: vertices from the u end as (matrix or 'W', momentum out);
            returns Gamma^rho for rho = 0..3 (matrices left = dbar end)."""
            res = []
            for r in range(4):
                G = np.eye(4, dtype=complex)
                P = pu.copy()
                for idx, (V, out) in enumerate(seq):
                    if idx > 0:
                        G = prop(P) @ G
                    G = (Wv[r] if isinstance(V, str) else V) @ G
                    P = P - out
                res.append(G)
            return res

        if n == 0:
            struct = [line([("W", q)])]
        elif n == 1:
            a, b = line([(gv[0], ks[0]), ("W", q)]), line([("W", q), (gv[0], ks[0])])
            struct = [[a[r] + b[r] for r in range(4)]]
        else:
            k1, k2 = ks
            # (T^a1 T^a2)_ji: gluon 1 nearer the dbar end
            seqs12 = [[(gv[1], k2), (gv[0], k1), ("W", q)], [(gv[1], k2), ("W", q), (gv[0], k1)],
                      [("W", q), (gv[1], k2), (gv[0], k1)]]
            seqs21 = [[(gv[0], k1), (gv[1], k2), ("W", q)], [(gv[0], k1), ("W", q), (gv[1], k2)],
                      [("W", q), (gv[0], k1), (gv[1], k2)]]
            L12 = [line(sq) for sq in seqs12]
            L21 = [line(sq) for sq in seqs21]
            # three-gluon vertex, momenta incoming: (a1, mu, -k1), (a2, nu, -k2), (b, lam, K)
            K = k1 + k2
            e1, e2 = np.conj(eps[0]), np.conj(eps[1])
            p1, p2, p3 = -k1, -k2, K
            Vlam = (_mdot(e1, e2) * (p1 - p2) + e2 * _mdot(p2 - p3, e1) + e1 * _mdot(p3 - p1, e2)) * gs
            # gluon propagator -i g/K^2 and quark vertex i g_s gamma^sigma (T^b)
            Jt = 1j * gs * slash(Vlam) * (-1j) / _mdot(K, K)
            Lt = [line([(Jt, K), ("W", q)])[r] + line([("W", q), (Jt, K)])[r] for r in range(4)]
            struct = [[sum(Lx[r] for Lx in L12) for r in range(4)], [sum(Lx[r] for Lx in L21) for r in range(4)],
                      Lt]
        nc = len(struct)
        Kmat = np.zeros((nc, nc), complex)
        for c in range(nc):
            for c2 in range(nc):
                acc = 0.0
                for r in range(4):
                    for s in range(4):
                        acc += np.trace(struct[c][r] @ slash(pu) @ bar(struct[c2][s]) @ slash(pd)) * Lep[r, s]
                Kmat[c, c2] = acc
        total += np.real(np.sum(Col * Kmat)) * abs(Wprop) ** 2
    return total


# ---------------------------------------------------------------- the pins
@pytest.mark.parametrize("n", [0, 1, 2])
def test_helicity_sum_equals_dirac_trace_brute_force(n):
    L = _lib()
    rng = np.random.default_rng(10 + n)
    for _ in range(4):
        mom = _event(rng, n)
        hel_sum = sum(L.orc_whel_me2(n, _c(mom), h, _c(THETA)) for h in range(1 << n))
        ref = brute_me2(n, mom, THETA)
        assert abs(hel_sum / ref - 1) < 1e-11, (n, hel_sum, ref)
        # a gauge shift of the polarisations leaves the brute force alone
        if n > 0:
            assert abs(brute_me2(n, mom, THETA, shift=0.8) / ref - 1) < 1e-11


def test_colour_matrices():
    assert np.allclose(colour_matrix(1), [[4.0]])
    C = colour_matrix(2)
    # (T T)-structures: 16/3 and -2/3; sum f^abc Tr(T^a T^b T^c) = (i/4) f^abc f^abc = 6 i;
    # sum f^abc f^abd Tr(T^c T^d) = N (N^2-1) / 2 = 12
    assert np.allclose(C, [[16 / 3, -2 / 3, 6j], [-2 / 3, 16 / 3, -6j], [-6j, 6j, 12]])


def test_n0_closed_form():
    """u dbar -> mu+ nu through the W: the V-A angular factor
    (pu.pmu)(pd.pnu); sum over colours and spins
    = 3 (g_W^2/2)^2 16 (pu.pmu)(pd.pnu) / |D|^2."""
    L = _lib()
    rng = np.random.default_rng(3)
    gw2 = 4 * math.sqrt(2) * GF * MWREF ** 2
    for _ in range(5):
        mom = _event(rng, 0)
        pu, pd, pmu, pnu = mom[0:4], mom[4:8], mom[8:12], mom[12:16]
        q = pmu + pnu
        D = (_mdot(q, q) - THETA[0] ** 2) ** 2 + (THETA[0] * THETA[1]) ** 2
        ref = 3 * (gw2 / 2) ** 2 * 16 * _mdot(pu, pmu) * _mdot(pd, pnu) / D
        assert abs(L.orc_whel_me2(0, _c(mom), 0, _c(THETA)) / ref - 1) < 1e-12


@pytest.mark.parametrize("n", [1, 2])
def test_ward_identity(n):
    L = _lib()
    rng = np.random.default_rng(20 + n)
    for _ in range(4):
        mom = _event(rng, n)
        ks = [mom[8 + 4 * i:12 + 4 * i] for i in range(n)]
        phys = [transverse_pols(k, 0.0)[0] for k in ks]
        scale = []
        for which in range(n):
            eps = np.zeros(8 * n)
            for i in range(n):
                eps[8 * i:8 * i + 4] = phys[i]
            A_phys = np.zeros(4)
            L.orc_whel_partials(n, _c(mom), _c(eps), A_phys.ctypes.data_as(dp))
            eps[8 * which:8 * which + 4] = ks[which] / ks[which][0]  # epsilon -> k / E
            A = np.zeros(4)
            L.orc_whel_partials(n, _c(mom), _c(eps), A.ctypes.data_as(dp))
            scale = np.max(np.abs(A_phys))
            assert np.max(np.abs(A)) < 1e-11 * scale, (n, which, A, A_phys)


def _boost(v, b):
    g = 1 / math.sqrt(1 - b @ b)
    bp = b @ v[1:]
    return np.concatenate([[g * (v[0] + bp)], v[1:] + ((g - 1) * bp / (b @ b) + g * v[0]) * b])


@pytest.mark.parametrize("n", [0, 1, 2])
def test_lorentz_invariance(n):
    L = _lib()
    rng = np.random.default_rng(30 + n)
    mom = _event(rng, n)
    b = np.array([0.3, -0.2, 0.5])
    mb = np.concatenate([_boost(mom[4 * i:4 * i + 4], b) for i in range(n + 4)])
    h0 = sum(L.orc_whel_me2(n, _c(mom), h, _c(THETA)) for h in range(1 << n))
    h1 = sum(L.orc_whel_me2(n, _c(mb), h, _c(THETA)) for h in range(1 << n))
    assert abs(h1 / h0 - 1) < 1e-10


def _pt_eta(px, py, pz):
    pt = math.hypot(px, py)
    return pt, math.asinh(pz / pt)


def test_cuts_hand_built():
    L = _lib()

    def vec(pt, eta, phi):
        return [pt * math.cosh(eta), pt * math.cos(phi), pt * math.sin(phi), pt * math.sinh(eta)]

    def ok(n, parts, yb=0.0):
        p = np.array(parts, dtype=float).reshape(-1)
        return L.orc_whel_pass_cuts(n, _c(p), yb, 20.0, 2.5, 5.0, 20.0)

    nu = vec(50, 0.0, 3.0)
    assert ok(0, [vec(20.01, 0.0, 0.0), nu]) == 1
    assert ok(0, [vec(19.99, 0.0, 0.0), nu]) == 0
    assert ok(0, [vec(30, 2.49, 0.0), nu]) == 1 and ok(0, [vec(30, 2.51, 0.0), nu]) == 0
    assert ok(0, [vec(30, 2.4, 0.0), nu], yb=0.2) == 0          # the lab rapidity counts
    assert ok(1, [vec(30, 4.99, 1.0), vec(30, 0, 0), nu]) == 1  # gluons up to |eta| < 5
    assert ok(1, [vec(30, 5.01, 1.0), vec(30, 0, 0), nu]) == 0
    # Durham pT_ij = min(pT_i, pT_j) Delta R: pT 25 and 40 at Delta R = 0.8 +- 0.001
    g1 = vec(25, 0.0, 0.0)
    mu = vec(30, 0, 2.0)
    assert ok(2, [g1, vec(40, 0.801, 0.0), mu, nu]) == 1
    assert ok(2, [g1, vec(40, 0.799, 0.0), mu, nu]) == 0
    assert ok(2, [g1, vec(40, 0.0, 0.801), mu, nu]) == 1
    # Delta phi wraps at pi
    assert ok(2, [vec(25, 0, 3.1), vec(40, 0, -3.1 + 0.79), mu, nu]) == 1  # dphi = 2 pi - 6.2 + 0.79 - ...
    # the neutrino is unconstrained
    assert ok(0, [vec(30, 0, 0), vec(1, 9.0, 0)]) == 1


@pytest.mark.parametrize("n", [0, 1, 2])
def test_event_is_product_of_factors(n):
    L = _lib()
    d = 3 * n + 5
    rng = np.random.default_rng(40 + n)
    done = 0
    while done < 10:
        x = rng.random(d)
        p = np.zeros(4 * (n + 2))
        aux = np.zeros(8)
        g = np.zeros(3)
        f = L.orc_whel_event(d, _c(x), _c(THETA), 8, p.ctypes.data_as(dp), aux.ctypes.data_as(dp),
                             g.ctypes.data_as(dp))
        if aux[7] == 0:
            assert f == 0.0
            continue
        x1, x2, shat, Jx, lum, Vn, m2 = aux[:7]
        rs = math.sqrt(shat)
        mom = np.concatenate([[rs / 2, 0, 0, rs / 2], [rs / 2, 0, 0, -rs / 2], p])
        # momentum conservation and the helicity chosen by the last variable
        assert np.allclose(np.sum(p.reshape(-1, 4), axis=0), [rs, 0, 0, 0], atol=1e-9 * rs)
        h = min(int(x[-1] * (1 << n)), (1 << n) - 1)
        me2 = L.orc_whel_me2(n, _c(mom), h, _c(THETA))
        assert abs(f / (lum * Jx * Vn / (2 * shat) * (1 << n) / 36.0 * me2) - 1) < 1e-13
        assert abs(Vn / O.ps_volume(n + 2, shat) - 1) < 1e-13
        # gradients: g_s scaling, and the W propagator derivatives by central differences
        assert abs(g[2] - f * 2 * n / THETA[2]) <= 1e-13 * abs(f) + 1e-300
        for i in (0, 1):
            hstep = 1e-5 * THETA[i]
            tp, tm = THETA.copy(), THETA.copy()
            tp[i] += hstep
            tm[i] -= hstep
            fp = L.orc_whel_event(d, _c(x), _c(tp), 8, p.ctypes.data_as(dp), None, None)
            fm = L.orc_whel_event(d, _c(x), _c(tm), 8, p.ctypes.data_as(dp), None, None)
            assert abs((fp - fm) / (2 * hstep) - g[i]) < 1e-6 * (abs(g[i]) + abs(f) / THETA[i])
        done += 1
