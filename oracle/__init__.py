"""FP64 CPU oracle for the VEGAS/BASES iteration (arXiv:1010.2107).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It wraps the plain C
library ``liboracle.so`` built from ``vmc_oracle.c`` (see ``build.py``) and a
small Python driver for the iteration loop (paper Sec. 3.1, steps 1-6).  It
shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

CONST, LINEAR, GAUSS, DGAUSS, GAUSS_AXES, WJETS, PSVOL, WHEL = range(8)

_lib = None


def lib():
    """Load liboracle.so, building it first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b

        _b.build()
    L = ctypes.CDLL(_LIB_PATH)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    c_int, c_i64, c_u64, c_u32, c_d = (ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                       ctypes.c_uint32, ctypes.c_double)
    L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.orc_sample_words.argtypes = [c_u64, c_u32, c_u32, c_u32, c_int, u32p]
    L.orc_uniform.argtypes = [c_u32]
    L.orc_uniform.restype = c_d
    L.orc_bin_batch.argtypes = [c_i64, u32p, i32p, c_int, c_int, i32p, dp]
    L.orc_map.argtypes = [c_int, c_int, dp, i32p, dp, dp]
    L.orc_map.restype = c_d
    L.orc_integrand_nparams.argtypes = [c_int, c_int]
    L.orc_integrand_ngrad.argtypes = [c_int, c_int]
    L.orc_integrand.argtypes = [c_int, c_int, dp, dp, c_int, dp]
    L.orc_integrand.restype = c_d
    L.orc_rambo_diet.argtypes = [c_int, c_d, dp, dp]
    L.orc_rambo_diet.restype = c_d
    L.orc_massless_ps_volume.argtypes = [c_int, c_d]
    L.orc_massless_ps_volume.restype = c_d
    L.orc_solve_mass_fraction.argtypes = [c_int, c_int, c_d, dp]
    L.orc_pass_cuts.argtypes = [c_int, dp, c_d, c_d, c_d, c_d]
    L.orc_cyclic_sum.argtypes = [c_int, dp]
    L.orc_cyclic_sum.restype = c_d
    L.orc_num_cycles.argtypes = [c_int]
    L.orc_wjets_event.argtypes = [c_int, dp, dp, c_int, dp, dp, dp]
    L.orc_wjets_event.restype = c_d
    L.orc_iterate.argtypes = [c_int, c_int, c_int, dp, c_int, dp, c_int, c_i64, c_u64, c_u32,
                              c_u32, dp, ctypes.c_void_p, dp, fp]
    L.orc_eval_samples.argtypes = [c_int, c_int, c_int, dp, c_int, dp, c_int, c_i64, c_u64,
                                   c_u32, c_u32, c_i64, c_i64, u32p, i32p, dp, dp, dp, dp, dp]
    L.orc_refine.argtypes = [c_int, c_int, dp, dp, c_d, dp]
    L.orc_set_point32.argtypes = [c_int]
    L.orc_accumulate_range.argtypes = [c_int, c_int, c_int, dp, dp, c_int, c_i64, c_u64, c_u32, c_u32, c_i64,
                                       c_i64, dp, ctypes.c_void_p]
    L.orc_estimate_plain.argtypes = [ctypes.c_void_p, c_i64]
    L.orc_combine.argtypes = [c_int, dp, dp, dp, dp, dp]
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.orc_cube_max.argtypes = [c_int, c_int, c_int, dp, c_int, dp, c_int, c_i64, c_u64, c_u32, dp]
    L.orc_spring_envelope.argtypes = [c_i64, dp, u64p, dp]
    L.orc_spring_pick.argtypes = [c_i64, u64p, c_u64]
    L.orc_spring_pick.restype = c_i64
    L.orc_spring_trials.argtypes = [c_int, c_int, c_int, dp, c_int, dp, c_int, u64p, c_d, c_u64, c_u32, c_u64,
                                    c_i64, i64p, dp, dp, dp, dp, i32p]
    _lib = L
    return L


class IterResult(ctypes.Structure):
    _fields_ = [("S1", ctypes.c_double), ("S2", ctypes.c_double), ("V", ctypes.c_double),
                ("I", ctypes.c_double), ("var", ctypes.c_double), ("n_eff", ctypes.c_int64),
                ("nonfinite", ctypes.c_int64)]


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


# ------------------------------------------------------------------ Philox
def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def sample_words(seed, s, it, kid, d):
    out = np.zeros(d, dtype=np.uint32)
    lib().orc_sample_words(seed, s, it, kid, d, _ptr(out, ctypes.c_uint32))
    return out


def uniform(word):
    return lib().orc_uniform(int(word))


def bins_of_words(words, nbins, ng=1, cube_coord=None):
    w = np.ascontiguousarray(words, dtype=np.uint32).ravel()
    n = w.size
    cc = None if cube_coord is None else np.ascontiguousarray(cube_coord, dtype=np.int32).ravel()
    j = np.zeros(n, dtype=np.int32)
    delta = np.zeros(n, dtype=np.float64)
    lib().orc_bin_batch(n, _ptr(w, ctypes.c_uint32), _ptr(cc, ctypes.c_int32), ng, nbins,
                        _ptr(j, ctypes.c_int32), _ptr(delta, ctypes.c_double))
    return j, delta


def grid_map(edges, j, delta):
    e = _d(edges)
    d, n1 = e.shape
    jj = np.ascontiguousarray(j, dtype=np.int32)
    dd = _d(delta)
    x = np.zeros(d)
    J = lib().orc_map(d, n1 - 1, _ptr(e, ctypes.c_double), _ptr(jj, ctypes.c_int32),
                      _ptr(dd, ctypes.c_double), _ptr(x, ctypes.c_double))
    return x, J


# -------------------------------------------------------------- integrands
def nparams(integrand, d):
    return lib().orc_integrand_nparams(integrand, d)


def ngrad(integrand, d):
    return lib().orc_integrand_ngrad(integrand, d)


def integrand(integrand_id, x, theta, want_grad=False):
    xx = _d(x)
    th = _d(theta)
    d = xx.size
    g = np.zeros(max(ngrad(integrand_id, d), 1)) if want_grad else None
    f = lib().orc_integrand(integrand_id, d, _ptr(xx, ctypes.c_double), _ptr(th, ctypes.c_double),
                            th.size, _ptr(g, ctypes.c_double))
    if want_grad:
        return f, g[: ngrad(integrand_id, d)]
    return f


def rambo_diet(n, sqrt_shat, r):
    rr = _d(r)
    assert rr.size == 3 * n - 4
    p = np.zeros((n, 4))
    w = lib().orc_rambo_diet(n, sqrt_shat, _ptr(rr, ctypes.c_double), _ptr(p, ctypes.c_double))
    return p, w


def ps_volume(n, shat):
    return lib().orc_massless_ps_volume(n, shat)


def solve_mass_fraction(n, i, r):
    t = ctypes.c_double()
    _check(lib().orc_solve_mass_fraction(n, i, r, ctypes.byref(t)), "solve_mass_fraction")
    return t.value


def pass_cuts(n_p, p, y_boost, ptmin, etamax, drmin):
    pp = _d(p)
    return bool(lib().orc_pass_cuts(n_p, _ptr(pp, ctypes.c_double), y_boost, ptmin, etamax, drmin))


def cyclic_sum(s):
    ss = _d(s)
    return lib().orc_cyclic_sum(ss.shape[0], _ptr(ss, ctypes.c_double))


def num_cycles(m):
    return lib().orc_num_cycles(m)


def wjets_event(x, theta, want_grad=False):
    xx = _d(x)
    th = _d(theta)
    d = xx.size
    n = (d - 4) // 3 + 2
    p = np.zeros((n, 4))
    aux = np.zeros(8)
    g = np.zeros(3) if want_grad else None
    f = lib().orc_wjets_event(d, _ptr(xx, ctypes.c_double), _ptr(th, ctypes.c_double), th.size,
                              _ptr(p, ctypes.c_double), _ptr(aux, ctypes.c_double),
                              _ptr(g, ctypes.c_double))
    keys = ("x1", "x2", "shat", "Jx", "lum", "Vn", "m2", "pass")
    out = dict(f=f, p=p, **{k: aux[i] for i, k in enumerate(keys)})
    if want_grad:
        out["grad"] = g
    return out


# ------------------------------------------------------------ iteration
def whel_event(x, theta, want_grad=False):
    """u dbar -> W+(-> mu+ nu) + n gluons at one point: f, momenta (g..,
    mu, nu; partonic frame), aux (x1, x2, shat, Jx, lum, Vn, m_munu^2,
    pass) and, if asked, the gradient w.r.t. (M, Gamma, g_s)."""
    xx = _d(x)
    th = _d(theta)
    d = xx.size
    n = (d - 5) // 3
    p = np.zeros(4 * (n + 2))
    aux = np.zeros(8)
    g = np.zeros(3)
    L = lib()
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_whel_event.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, dp]
    L.orc_whel_event.restype = ctypes.c_double
    f = L.orc_whel_event(d, _ptr(xx, ctypes.c_double), _ptr(th, ctypes.c_double), th.size,
                         _ptr(p, ctypes.c_double), _ptr(aux, ctypes.c_double), _ptr(g, ctypes.c_double))
    out = dict(f=f, p=p.reshape(n + 2, 4), aux=aux)
    if want_grad:
        out["grad"] = g
    return out


def uniform_edges(d, nbins):
    return np.tile(np.arange(nbins + 1, dtype=np.float64) / nbins, (d, 1))


class point32:
    """Within this context the integrand sees the point as a single-precision
    grid map forms it (FP32 lower edge and scaled width per bin, one fused
    multiply-add with the in-bin offset), everything else staying FP64: a
    single-precision integrand can then be compared with the oracle on
    identical inputs."""

    def __init__(self, on=True):
        self.on = bool(on)

    def __enter__(self):
        lib().orc_set_point32(int(self.on))
        return self

    def __exit__(self, *exc):
        lib().orc_set_point32(0)
        return False


def iterate(integrand_id, edges, theta, ncall, seed, it, kid=0, ng=1, want_grad=False, w_in=None, fp32_point=False):
    """One iteration (steps 2-4): returns dict with S1, S2, V, I, var, n_eff,
    nonfinite, bins [2][d][N] and (if want_grad) per-parameter gradient sums.
    fp32_point: evaluate at the point an FP32 grid map forms (see point32)."""
    if fp32_point:
        with point32():
            return iterate(integrand_id, edges, theta, ncall, seed, it, kid, ng, want_grad, w_in)
    e = _d(edges)
    d, n1 = e.shape
    N = n1 - 1
    th = _d(theta)
    bins = np.zeros((2, d, N))
    res = IterResult()
    P = ngrad(integrand_id, d)
    g = np.zeros(5 * max(P, 1)) if want_grad else None
    wi = None if w_in is None else np.ascontiguousarray(w_in, dtype=np.float32)
    rc = lib().orc_iterate(integrand_id, d, N, _ptr(e, ctypes.c_double), ng, _ptr(th, ctypes.c_double),
                           th.size, int(ncall), int(seed), int(it), int(kid), _ptr(bins, ctypes.c_double),
                           ctypes.byref(res), _ptr(g, ctypes.c_double), _ptr(wi, ctypes.c_float))
    _check(rc, "orc_iterate")
    out = {f: getattr(res, f) for f, _ in IterResult._fields_}
    out["bins"] = bins
    if want_grad:
        gg = g[: 5 * P].reshape(P, 5) if P else np.zeros((0, 5))
        out["gsum"] = gg[:, 0].copy()
        out["gsumsq"] = gg[:, 1].copy()
        out["gV"] = gg[:, 2].copy()
        out["grad"] = gg[:, 3].copy()
        out["grad_var"] = gg[:, 4].copy()
    return out


def accumulate_range(integrand_id, edges, theta, ncall, seed, it, s0, s1, kid=0):
    """Plain-mode sums (S1, S2, bins, nonfinite) over samples [s0, s1)."""
    e = _d(edges)
    d, n1 = e.shape
    th = _d(theta)
    bins = np.zeros((2, d, n1 - 1))
    res = IterResult()
    _check(lib().orc_accumulate_range(integrand_id, d, n1 - 1, _ptr(e, ctypes.c_double), _ptr(th, ctypes.c_double),
                                      th.size, int(ncall), int(seed), int(it), int(kid), int(s0), int(s1),
                                      _ptr(bins, ctypes.c_double), ctypes.byref(res)), "orc_accumulate_range")
    return dict(S1=res.S1, S2=res.S2, nonfinite=res.nonfinite, bins=bins)


def _range_job(args):
    return accumulate_range(*args)


def iterate_sharded(integrand_id, edges, theta, ncall, seed, it, pool, nshards, kid=0):
    """Plain-mode iteration with the samples split into nshards contiguous
    ranges evaluated by `pool` (a multiprocessing pool); the shards' sums are
    added and the estimate formed from the totals, as a multi-device split of
    one iteration would do."""
    bounds = [ncall * i // nshards for i in range(nshards + 1)]
    jobs = [(integrand_id, edges, theta, ncall, seed, it, bounds[i], bounds[i + 1], kid) for i in range(nshards)]
    parts = pool.map(_range_job, jobs)
    res = IterResult()
    res.S1 = sum(p["S1"] for p in parts)
    res.S2 = sum(p["S2"] for p in parts)
    res.nonfinite = sum(p["nonfinite"] for p in parts)
    lib().orc_estimate_plain(ctypes.byref(res), int(ncall))
    out = {f: getattr(res, f) for f, _ in IterResult._fields_}
    out["bins"] = sum(p["bins"] for p in parts)
    return out


def eval_samples(integrand_id, edges, theta, ncall, seed, it, s0, count, kid=0, ng=1, fp32_point=False):
    if fp32_point:
        with point32():
            return eval_samples(integrand_id, edges, theta, ncall, seed, it, s0, count, kid, ng)
    e = _d(edges)
    d, n1 = e.shape
    th = _d(theta)
    P = max(ngrad(integrand_id, d), 0)
    out = dict(words=np.zeros((count, d), np.uint32), j=np.zeros((count, d), np.int32),
               x=np.zeros((count, d)), jac=np.zeros(count), f=np.zeros(count), w=np.zeros(count),
               grad=np.zeros((count, max(P, 1))))
    rc = lib().orc_eval_samples(integrand_id, d, n1 - 1, _ptr(e, ctypes.c_double), ng,
                                _ptr(th, ctypes.c_double), th.size, int(ncall), int(seed), int(it),
                                int(kid), int(s0), int(count), _ptr(out["words"], ctypes.c_uint32),
                                _ptr(out["j"], ctypes.c_int32), _ptr(out["x"], ctypes.c_double),
                                _ptr(out["jac"], ctypes.c_double), _ptr(out["f"], ctypes.c_double),
                                _ptr(out["w"], ctypes.c_double), _ptr(out["grad"], ctypes.c_double))
    _check(rc, "orc_eval_samples")
    out["grad"] = out["grad"][:, :P]
    return out


def refine(edges, b2, alpha):
    e = _d(edges)
    d, n1 = e.shape
    b = _d(b2)
    out = np.zeros_like(e)
    _check(lib().orc_refine(d, n1 - 1, _ptr(e, ctypes.c_double), _ptr(b, ctypes.c_double), alpha,
                            _ptr(out, ctypes.c_double)), "orc_refine")
    return out


def combine(I, var):
    Ia = _d(I)
    va = _d(var)
    Ib, sb, chi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_combine(Ia.size, _ptr(Ia, ctypes.c_double), _ptr(va, ctypes.c_double), ctypes.byref(Ib),
                      ctypes.byref(sb), ctypes.byref(chi))
    return Ib.value, sb.value, chi.value


# ------------------------------------------------------------ SPRING
def cube_max(integrand_id, edges, theta, ncall, seed, it, ng, wmax=None):
    """Fold the largest weight of each of the ng^d cubes of one stratified
    iteration into wmax (new zero array when None)."""
    e = _d(edges)
    d, n1 = e.shape
    th = _d(theta)
    out = np.zeros(ng ** d) if wmax is None else wmax
    assert out.dtype == np.float64 and out.flags.c_contiguous and out.size == ng ** d
    _check(lib().orc_cube_max(integrand_id, d, n1 - 1, _ptr(e, ctypes.c_double), ng, _ptr(th, ctypes.c_double),
                              th.size, int(ncall), int(seed), int(it), _ptr(out, ctypes.c_double)), "orc_cube_max")
    return out


def spring_envelope(wmax):
    """Integer envelope q (quanta of unit = max(wmax) / 2^20 per cube)."""
    w = _d(wmax)
    q = np.zeros(w.size, np.uint64)
    unit = ctypes.c_double()
    _check(lib().orc_spring_envelope(w.size, _ptr(w, ctypes.c_double), _ptr(q, ctypes.c_uint64),
                                     ctypes.byref(unit)), "orc_spring_envelope")
    return q, unit.value


def spring_pick(q, r64):
    """Cube chosen by the 64-bit integer r64 under envelope q."""
    qa = np.ascontiguousarray(q, dtype=np.uint64)
    P = np.zeros(qa.size + 1, np.uint64)
    P[1:] = np.cumsum(qa, dtype=np.uint64)
    return int(lib().orc_spring_pick(qa.size, _ptr(P, ctypes.c_uint64), int(r64)))


def spring_trials(integrand_id, edges, theta, ng, q, unit, seed, pass_, trial0, ntrials):
    """Per-trial record of SPRING trials trial0 .. trial0+ntrials-1."""
    e = _d(edges)
    d, n1 = e.shape
    th = _d(theta)
    qa = np.ascontiguousarray(q, dtype=np.uint64)
    out = dict(cube=np.zeros(ntrials, np.int64), x=np.zeros((ntrials, d)), w=np.zeros(ntrials),
               env=np.zeros(ntrials), u=np.zeros(ntrials), kept=np.zeros(ntrials, np.int32))
    _check(lib().orc_spring_trials(integrand_id, d, n1 - 1, _ptr(e, ctypes.c_double), ng, _ptr(th, ctypes.c_double),
                                   th.size, _ptr(qa, ctypes.c_uint64), float(unit), int(seed), int(pass_),
                                   int(trial0), int(ntrials), _ptr(out["cube"], ctypes.c_int64),
                                   _ptr(out["x"], ctypes.c_double), _ptr(out["w"], ctypes.c_double),
                                   _ptr(out["env"], ctypes.c_double), _ptr(out["u"], ctypes.c_double),
                                   _ptr(out["kept"], ctypes.c_int32)), "orc_spring_trials")
    out["kept"] = out["kept"].astype(bool)
    return out


# ------------------------------------------------------------ driver
@dataclass
class Run:
    I: list = field(default_factory=list)      # iterations of the last phase (the combined ones)
    var: list = field(default_factory=list)
    Ibar: float = float("nan")
    sigbar: float = float("nan")
    chi2dof: float = float("nan")
    edges: np.ndarray | None = None
    n_eff: int = 0
    wmax: np.ndarray | None = None
    I_all: list = field(default_factory=list)  # every iteration, both phases
    var_all: list = field(default_factory=list)
    edges_seq: list = field(default_factory=list)  # the grid each iteration sampled on


def integrate(integrand_id, d, nbins, theta, ncall, itmx, seed, alpha=1.5, ng=1, acc=0.0,
              itmx2=0, edges=None, cube_max_phase2=False):
    """VEGAS (itmx2 == 0) or BASES (itmx grid-optimisation iterations, then
    itmx2 integration iterations with the grid frozen; only the latter are
    combined).  Paper Sec. 3.1 steps 1-6 and Sec. 6.1 (ITMX, ACC, ITMX1/2).
    cube_max_phase2: also record each cube's largest weight over the
    integration phase (the input of SPRING) in run.wmax."""
    e = uniform_edges(d, nbins) if edges is None else _d(edges).copy()
    run = Run()
    if cube_max_phase2:
        run.wmax = np.zeros(ng ** d)
    it = 0
    phases = [(itmx, True)] + ([(itmx2, False)] if itmx2 else [])
    for nit, adapt in phases:
        Is, vs = [], []
        for _ in range(nit):
            run.edges_seq.append(e.copy())
            r = iterate(integrand_id, e, theta, ncall, seed, it, ng=ng)
            run.I_all.append(r["I"])
            run.var_all.append(r["var"])
            if cube_max_phase2 and not adapt:
                cube_max(integrand_id, e, theta, ncall, seed, it, ng, run.wmax)
            it += 1
            run.n_eff += r["n_eff"]
            Is.append(r["I"])
            vs.append(r["var"])
            if adapt:
                e = refine(e, r["bins"][1], alpha)
            Ib, sb, chi = combine(Is, vs)
            if acc > 0 and Ib != 0 and sb / abs(Ib) < acc:
                break
        run.I, run.var = Is, vs
        run.Ibar, run.sigbar, run.chi2dof = combine(Is, vs)
    run.edges = e
    return run
