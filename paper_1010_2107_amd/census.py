"""FP32 flop census of one sample of the sample-and-accumulate kernel.

Counts the FP32 operations of the per-sample algorithm as written in the HIP
sources (add/sub/mul = 1, fma = 2).  Reciprocals, square roots and other
transcendentals are tallied in `trans` and are not counted as flops; integer
work, compares, min/max and the FP64 accumulation are not FP32 flops either.  The W + partons integrand has two paths:
samples that fail the cuts stop before the colour sum; `per_sample(...)`
returns both and the bench weights them with the measured accepted fraction.
Where the kernel evaluates a choice both ways (the two sides of the mass
step's start), only the side the algorithm needs is counted.
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import permutations

from . import workloads as W


@dataclass
class Census:
    flops_pass: int
    flops_fail: int
    trans_pass: int
    trans_fail: int

    def flops(self, frac_pass: float) -> float:
        return frac_pass * self.flops_pass + (1.0 - frac_pass) * self.flops_fail


def cycles(m):
    """Distinct cyclic orders of m objects (object 0 first, first < last)."""
    return [(0,) + p for p in permutations(range(1, m)) if p[0] < p[-1]]


def cycle_sum_flops(m):
    """Flops of the colour-ordered sum over cyclic orders.  Six objects use
    the meet-in-the-middle form: per object z opposite object 0, six two-step
    arcs (multiply, fma, multiply) and three fmas.  Other sizes use the
    subset dynamic programme over paths from object 0: each (set S, end v)
    with |S| >= 2 costs one multiply and |S|-2 fmas; closing the full paths
    costs one multiply, m-2 fmas and the final halving."""
    if m == 6:
        return 5 * (6 * 4 + 3 * 2)
    K = m - 1
    f = 0
    for mask in range(1, 1 << K):
        p = bin(mask).count("1")
        if p >= 2:
            f += p * (1 + 2 * (p - 2))
    return f + 1 + 2 * (K - 1) + 1


MAP_PER_AXIS = 4  # fma(delta, width, lo), N width, Jacobian product


# The flux factor ((1-xa)(1-xb))^3 of an accepted sample: each e^x - 1
# counted on its exp2 side (a scaling and a subtraction), their product, the
# cube and the product with the rest of the prefactor.
FLUX, FLUX_TRANS = 8, 2


MASS_START_DEG = 5  # degree of the fitted start polynomial (csrc/vmc_mass_start.hpp)


def _mass_step(K):
    """FP32 flops and transcendentals of one mass-fraction solve in the FP32
    kernels.  K = 1 is in closed form (1 - r, 1 + s, the product, and the
    scaling of the Newton step's reciprocal; the step itself is FP64).
    Otherwise: the start on the lane's side (1 - r and a scaling, then
    square roots for K = 2 and 4, log2, a scaling and exp2 for K = 3), the
    correction polynomial and its product with s, and the FP32 derivative of
    the Newton step, K (K+1) t^(K-1) (1 - t) (1 - v, K - 1 products and one
    more); the residual, the update and 1 - v are FP64 and not counted."""
    if K == 1:
        return 4, 3
    start = 2 + 2 * MASS_START_DEG + 1 + (1 if K == 3 else 0)
    deriv = 1 + (K - 1) + 1
    trans = {2: 1, 3: 2, 4: 1.5}.get(K, 2) + 1  # the start's roots or log2/exp2, and the reciprocal
    return start + deriv, trans


def wjets(n_p: int) -> Census:
    n = n_p + 2
    D = 3 * n_p + 4
    nv = n_p + 1
    f = t = 0
    f += MAP_PER_AXIS * D
    # parton fractions ln xa, ln xb, sqrt(tau) (one exp2), sqrt(s) and the
    # boost rapidity; the rest of the prefactor and the flux factor
    # ((1-xa)(1-xb))^3 are formed only for accepted samples
    f += 10
    t += 1
    # mass chain: one inverse-CDF solve per mass, then M_i = M_{i-1} sqrt(t)
    for K in range(n - 2, 0, -1):
        ff, tt = _mass_step(K)
        f += ff + 1
        t += tt + 1
    # two-body steps: the first needs no boost (13); each other one boosts
    # its massless momentum (17) and takes the recoil as Q - p (4), plus the
    # direction, energy and boost factors (13)
    f += 13 + (n - 2) * 34
    t += 3 + (n - 2) * 5
    # visible particles: pT^2, E + |pz|, rapidity (6, one rsqrt and one
    # log2), the unit transverse direction (2), |eta + y_boost| (1), and for
    # the partons 1 / pT^2 (1)
    f += 9 * nv + n_p
    t += 2 * nv
    # Delta R pairs: Delta eta, z, cos of the threshold angle by its series,
    # cos(Delta phi) from the unit directions
    f += 12 * nv * (nv - 1) // 2
    f_fail, t_fail = f + 1, t
    # accepted samples: the smaller light-cone component of each parton (1
    # and a reciprocal) and its two scaled invariants with a and b (4);
    # sqrt(s) again from ln xa + ln xb (3 and an exp2); s, c / sqrt(s) and
    # y_ab (3, one reciprocal); per parton pair the
    # invariant (8) and its scaled reciprocal (1); the cyclic sum; the
    # prefactor s^(n-3) s^4 pre L^2 x0 sqrt(S) / sqrt(s) (n - 3 + 8); the
    # Breit-Wigner factor (2 and a reciprocal) and the product f (6)
    m = n_p + 2
    f += 5 * n_p + 3 + 3 + 9 * (n_p * (n_p - 1) // 2) + cycle_sum_flops(m) + (n - 3 + 8) + 8 + FLUX
    t += n_p + 1 + 1 + n_p * (n_p - 1) // 2 + 1 + FLUX_TRANS
    return Census(int(round(f)), int(round(f_fail)), int(t), int(t_fail))


def whel(n: int) -> Census:
    """u dbar -> W + n gluons (helicity amplitudes), per the HIP source.
    Complex arithmetic: a product 6 flops (two multiplies, two fmas), a
    fused a b + c 8 (four fmas), s a + c 4; every product feeding a sum is
    fused into it in the source."""
    nf = n + 2
    D = 3 * n + 5
    f = t = 0
    f += MAP_PER_AXIS * D
    f += 9  # parton fractions, sqrt(tau) (one exp2), sqrt(s), boost rapidity
    t += 1
    for K in range(nf - 2, 0, -1):  # mass chain
        ff, tt = _mass_step(K)
        f += ff + 1
        t += tt + 1
    f += 13 + (nf - 2) * 34  # two-body steps: boosts and recoils as for wjets
    t += 3 + (nf - 2) * 5
    f += 10 * (n + 1)  # light-cone components, pT, rapidity, |eta + y_boost| of the gluons and the muon
    t += 3 * (n + 1)
    if n == 2:
        f += 12  # Durham pT_ij between the two gluons
        t += 3
    f_fail, t_fail = f + 1, t
    # (V.sigmabar) x: 28; plus a spinor: 32; its first component: 14, plus a
    # complex number: 16; a propagator (P^2, its reciprocal, P.sigma x): 29
    SBAR, SBAR_ADD, TOP, TOP_ADD, PROP = 28, 32, 14, 16, 29
    f += 5 * nf  # E = |p| of each final-state momentum (a square root each)
    t += nf
    f += 2 * 12 + 40  # lepton spinors and current
    t += 2
    if n == 0:
        f += TOP + 3
    elif n == 1:
        f += 15 + 2 * PROP + TOP + TOP_ADD + 4  # polarisation, two chains, |A|^2
        t += 3 + 2
    else:
        # polarisations (2 x 15); the three-gluon current: the dot products
        # (3 x 16), its scalars (8), K^2 (12) and its four components (4 x 18)
        f += 2 * 15 + 48 + 8 + 12 + 72
        f += 3 * PROP  # the chains' shared first propagators
        # each colour order: two vertex-propagator chains and a vertex, the
        # sums fused into the vertices (2 x SBAR_ADD + SBAR + 2 x PROP +
        # 2 x TOP_ADD); the three-gluon term TOP; the colour matrix (10)
        f += 2 * (2 * SBAR_ADD + SBAR + 2 * PROP + 2 * TOP_ADD) + TOP + 10
        t += 2 * 3 + 1 + 9
    f += 9 + n + 2  # sqrt(s) again (an exp2), s^n and the prefactor (a reciprocal)
    t += 2
    f += 8 + FLUX  # W propagator, product, flux factor
    t += 1 + FLUX_TRANS
    return Census(int(round(f)), int(round(f_fail)), int(t), int(t_fail))


def gaussian(integrand: int, d: int) -> Census:
    if integrand == W.GAUSS or integrand == W.GAUSS_AXES:
        fl = MAP_PER_AXIS * d + 3 * d + 2 + 1
        tr = 1
    elif integrand == W.DGAUSS:
        fl = MAP_PER_AXIS * d + 6 * d + 6 + 1
        tr = 2
    else:
        fl, tr = MAP_PER_AXIS * d + 1, 0
    return Census(fl, fl, tr, tr)


# The algorithm's FP32 operation count per sample, step by step as the
# method states the work rather than as the kernel arranges it: the colour
# sum with every cyclic order written out (60 orders of six objects for
# four partons), each invariant as a Minkowski product, RAMBO on diet with
# both momenta boosted at every two-body step, the cuts, the grid map
# (3 per axis).  Per-step estimates for the workloads the measurement
# quotes; the colour sum, the invariants and the Breit-Wigner factor run on
# accepted samples only.  (integrand, dim) -> (always, accepted only).
ALGORITHMIC = {
    # phase space 320, cuts 185, map 48, rest 50 | colour sum 420, invariants 105
    (W.WJETS, 16): (320 + 185 + 48 + 50, 420 + 105),
    # map 30, parton fractions and flux 20, phase space 125, cuts 95, rest 20 |
    # colour sum, invariants and Breit-Wigner 50
    (W.WJETS, 10): (30 + 20 + 125 + 95 + 20, 50),
    (W.DGAUSS, 8): (110, 0),
    (W.GAUSS, 4): (45, 0),
}


def algorithmic_flops(w, accepted_fraction: float) -> float | None:
    """The algorithm's FP32 flops per sample of a workload (ALGORITHMIC), or
    None where no such count is set (then the executed census applies)."""
    c = ALGORITHMIC.get((w.integrand, w.dim))
    if c is None:
        return None
    return c[0] + accepted_fraction * c[1]


def for_workload(w) -> Census:
    if w.integrand == W.WJETS:
        return wjets((w.dim - 4) // 3)
    if w.integrand == W.WHEL:
        return whel((w.dim - 5) // 3)
    return gaussian(w.integrand, w.dim)
