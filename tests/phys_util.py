"""Cut margins of oracle events, used to accept GPU/oracle disagreements on
cut decisions only for events that sit on a cut boundary (both decisions
are then correct at the working precision)."""
import math

import numpy as np

import oracle as O


def cut_margin(x, theta):
    """Smallest relative distance of an event to any cut threshold."""
    ev = O.wjets_event(x, theta)
    d = len(x)
    n_p = (d - 4) // 3
    p = ev["p"]
    ptmin, etamax, drmin = theta[4], theta[5], theta[6]
    yb = 0.5 * math.log(ev["x1"] / ev["x2"])
    m = np.inf
    etas, phis = [], []
    for i in range(n_p + 1):
        pt = math.hypot(p[i, 1], p[i, 2])
        eta = math.asinh(p[i, 3] / pt)
        etas.append(eta)
        phis.append(math.atan2(p[i, 2], p[i, 1]))
        m = min(m, abs(pt - ptmin) / ptmin, abs(abs(eta + yb) - etamax) / etamax)
    for i in range(n_p + 1):
        for k in range(i + 1, n_p + 1):
            dphi = abs(phis[i] - phis[k])
            if dphi > math.pi:
                dphi = 2 * math.pi - dphi
            dr = math.hypot(etas[i] - etas[k], dphi)
            m = min(m, abs(dr - drmin) / drmin)
    return m


def whel_cut_margin(x, theta):
    """Smallest relative distance of a u dbar -> W + n gluon event to any of
    its cut thresholds (gluon and muon pT and eta, gluon-pair pT_ij)."""
    ev = O.whel_event(x, theta)
    n = (len(x) - 5) // 3
    p, aux = ev["p"], ev["aux"]
    ptmin, eta_mu, eta_g, ptij = theta[4], theta[5], theta[6], theta[7]
    yb = 0.5 * math.log(aux[0] / aux[1])
    m = np.inf
    etas, phis, pts = [], [], []
    for i in range(n + 1):
        pt = math.hypot(p[i, 1], p[i, 2])
        eta = math.asinh(p[i, 3] / pt)
        etas.append(eta)
        phis.append(math.atan2(p[i, 2], p[i, 1]))
        pts.append(pt)
        emax = eta_g if i < n else eta_mu
        m = min(m, abs(pt - ptmin) / ptmin, abs(abs(eta + yb) - emax) / emax)
    for i in range(n):
        for k in range(i + 1, n):
            dphi = abs(phis[i] - phis[k])
            if dphi > math.pi:
                dphi = 2 * math.pi - dphi
            v = min(pts[i], pts[k]) * math.hypot(etas[i] - etas[k], dphi)
            m = min(m, abs(v - ptij) / ptij)
    return m
