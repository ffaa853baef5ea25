"""Synthetic workloads: sizes, parameters and seeds of the five
configurations, and the seeded generator of the batched configuration's
per-integral parameters.  Inputs only -- none of the method's arithmetic.

The paper's own workload (u dbar -> W+ + n gluons with HELAS amplitudes and
CTEQ6L1 PDFs, Sec. 5, Tables 4-5) is not reproducible here; the W + partons
toy integrand stands in for it with the same shape (multiplicity, 14 TeV,
pT > 20 GeV, |eta| < 2.5) and NCALL of the same order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

# integrand ids (same numbering as include/vmc.h)
CONST, LINEAR, GAUSS, DGAUSS, GAUSS_AXES, WJETS, PSVOL, WHEL = range(8)

SQRT_S = 14000.0          # GeV, LHC (paper Sec. 6)
PT_MIN, ETA_MAX, DR_MIN = 20.0, 2.5, 0.4
ALPHA_S = 0.118           # paper Sec. 5
G_STRONG = math.sqrt(4.0 * math.pi * ALPHA_S)
M_W, GAMMA_W = 80.4, 2.1
WJETS_THETA = (M_W, GAMMA_W, G_STRONG, SQRT_S, PT_MIN, ETA_MAX, DR_MIN)
# the paper's process with helicity amplitudes (Sec. 5): muon |eta| < 2.5,
# gluon |eta| < 5, Durham pT_ij > 20 GeV between gluons
ETA_GLUON, PTIJ_MIN = 5.0, 20.0
WHEL_THETA = (M_W, GAMMA_W, G_STRONG, SQRT_S, PT_MIN, ETA_MAX, ETA_GLUON, PTIJ_MIN)


@dataclass(frozen=True)
class Workload:
    name: str
    integrand: int
    dim: int
    nbins: int
    ncall: int
    itmx: int
    theta: tuple
    seed: int = 1234
    alpha: float = 1.5
    ng: int = 1
    itmx2: int = 0
    I_ref: float | None = None
    grad_ref: tuple | None = None
    fd_h: float | None = None      # absolute FD step (None: relative 1e-4)


C1 = Workload("gauss_d4_plain", GAUSS, 4, 50, 10_000, 10, (0.5, 0.1), I_ref=1.0, grad_ref=(0.0, 0.0))
# BASES: ITMX1 = ITMX2 = 10 (the paper sets the two phases equal, Sec. 6.1)
C2 = Workload("dgauss_d8_bases", DGAUSS, 8, 128, 5_000_000, 10, (1 / 3, 2 / 3, 0.1), ng=4, itmx2=10, I_ref=1.0,
              grad_ref=(0.0, 0.0, 0.0), fd_h=1e-4)
C2_PLAIN = replace(C2, name="dgauss_d8_vegas", ng=1, itmx=20, itmx2=0)
C3 = Workload("wjets2_d10_vegas", WJETS, 10, 64, 10_000_000, 15, WJETS_THETA)
C4 = Workload("wjets4_d16_vegas", WJETS, 16, 64, 50_000_000, 20, WJETS_THETA)
# the BASES forms of the two: ng^d cubes of k samples (4^10 x 9 and 2^16 x
# 762, about the plain forms' calls), ITMX1 + ITMX2 = the plain ITMX
C3_BASES = replace(C3, name="wjets2_d10_bases", ncall=4**10 * 9, ng=4, itmx=8, itmx2=7)
C4_BASES = replace(C4, name="wjets4_d16_bases", ncall=2**16 * 762, ng=2, itmx=10, itmx2=10)
# u dbar -> W+(-> mu+ nu) + 2 gluons from helicity amplitudes, d = 11
C6 = Workload("whel2_d11_vegas", WHEL, 11, 64, 10_000_000, 15, WHEL_THETA)

CONFIGS = {w.name: w for w in (C1, C2, C2_PLAIN, C3, C4, C3_BASES, C4_BASES, C6)}
DEFAULT_BENCH = C4


def default_ng(ncall: int, dim: int, nbins: int) -> int:
    """BASES stratification when none is given: the largest divisor of nbins
    not above (ncall / 2)^(1/dim), so that every cube gets at least two
    samples (at least 2)."""
    top = int((ncall / 2) ** (1.0 / dim) + 1e-9)
    best = 2
    for ng in range(2, max(top, 2) + 1):
        if nbins % ng == 0:
            best = ng
    return best


def ngrad(w) -> int:
    """Number of differentiable parameters of a workload's integrand."""
    return {CONST: 1, LINEAR: 0, GAUSS: 2, DGAUSS: 3, GAUSS_AXES: w.dim + 1, WJETS: 3, PSVOL: 0,
            WHEL: 3}[w.integrand]


@dataclass
class BatchSpec:
    dims: np.ndarray
    centres: list
    sigmas: np.ndarray
    ncalls: np.ndarray
    nbins: int = 64
    itmx: int = 5      # warm-up iterations, left out of the combination
    itmx2: int = 5     # combined iterations
    seed: int = 1234
    freeze: bool = False  # VEGAS: the grids keep adapting in the combined iterations

    @property
    def n(self):
        return len(self.dims)

    def theta(self, k):
        return tuple(self.centres[k]) + (float(self.sigmas[k]),)


def batched_config(n=64, gen_seed=2107, nbins=64, itmx=5, itmx2=5, seed=1234) -> BatchSpec:
    """n per-axis Gaussian products: d uniform in [2,12], centres U(0.2,0.8),
    sigma log-uniform in [0.05, 0.2], calls log-uniform in [1e4, 1e7]; ten
    VEGAS iterations, the first five (grid warm-up) left out of the
    combination: with 1e4-1e5 calls in up to 12 dimensions the first
    iterations see almost none of a narrow peak and report tiny variances
    that would dominate a 1/var-weighted mean."""
    rng = np.random.default_rng(gen_seed)
    dims = rng.integers(2, 13, size=n)
    centres = [0.2 + 0.6 * rng.random(int(d)) for d in dims]
    sigmas = 0.05 * 4.0 ** rng.random(n)
    ncalls = np.round(10.0 ** (4.0 + 3.0 * rng.random(n))).astype(np.int64)
    return BatchSpec(dims=dims, centres=centres, sigmas=sigmas, ncalls=ncalls, nbins=nbins, itmx=itmx, itmx2=itmx2,
                     seed=seed)
