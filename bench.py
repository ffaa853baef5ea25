"""Benchmark of the VEGAS/BASES hot path on one MI355X.

A step is one iteration of the workload: the sample-and-accumulate pass
(Philox words -> grid map -> integrand -> FP64 per-bin sums), the estimate
and running combination, and (in the grid-optimisation phase) the grid
refinement.  `value` is integrand evaluations per second over the timed
steps (fail-cut samples count as evaluations, as NCALL does in the paper).

Prints ONE JSON line.  `roofline` sets the forward kernel's census flops
(paper_1010_2107_amd/census.py) per launch, timed with HIP events on the
launch stream, against the published FP32 peak and against the FMA and LDS
atomic rates that probe kernels measure on the chip; `traffic` comes from
the committed hardware-counter summary when it was taken on the current
kernel sources.  `cpu_baseline` times the FP64 oracle on a bounded sample of
the same workload on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

def source_sha1():
    """Hash of the sources the sample kernels are built from (device headers,
    the integrand instantiations and the launch code) with comments and
    blank space removed, identifying the kernel build that a
    hardware-counter summary was taken on."""
    import glob
    import hashlib
    import re
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_1010_2107_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "*.hpp")) + glob.glob(os.path.join(csrc, "inst_*.hip")) +
                   [os.path.join(csrc, "vmc_capi.hip")])
    for f in files:
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(os.path.basename(f).encode())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def counter_summary(workload_name):
    """Key/value lines of the committed hardware-counter summary of the
    forward sample kernel, or None when it is missing or was taken on other
    kernel sources."""
    p = os.path.join(ROOT, "profiles", f"pmc_sample_kernel_{workload_name}.txt")
    if not os.path.exists(p):
        return None
    kv = {}
    for line in open(p):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv if kv.get("source-sha1") == source_sha1() else None


def measured_traffic(workload_name):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy
    calibration) from the counter summary, or None."""
    kv = counter_summary(workload_name)
    try:
        return float(kv["traffic_bytes_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


def measured_valu(workload_name):
    """VALU wave instructions per launch (SQ_INSTS_VALU) from the counter
    summary, or None."""
    kv = counter_summary(workload_name)
    try:
        return float(kv["SQ_INSTS_VALU"]) if kv else None
    except (KeyError, ValueError):
        return None


PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak (packed FMA): 256 CU x 2.4 GHz x 256 flop/clk


def run_loop(grid, w, steps, adjoint=False, fused=False):
    """Time `steps` iterations; returns (ms_total, kernel_ms, launches)."""
    import torch
    grid.reset()
    grid.stratify(w.ng)
    th = grid.theta_tensor(w.theta)
    torch.cuda.synchronize()
    grid.timing(True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for it in range(steps):
        if fused:
            grid.fused(w.integrand, th, w.ncall, w.seed, it)
        else:
            grid.iterate(w.integrand, th, w.ncall, w.seed, it)
            if adjoint:
                grid.adjoint(w.integrand, th, w.ncall, w.seed, it)
        if it < w.itmx:
            grid.refine(w.alpha)
        if w.itmx2 and it + 1 == w.itmx:
            grid.combine_reset()
    t1.record()
    torch.cuda.synchronize()
    kms, nl = grid.timing(False)
    return t0.elapsed_time(t1), kms, nl


def record_loop(grid, w, steps, adjoint=False, fused=False):
    """The loop of run_loop (reset, `steps` iterations with their refinement
    and the BASES phase switch) recorded once as a HIP graph, so that a
    replay launches the whole loop at once instead of three or four kernels
    per iteration from the host.  An eager run on a side stream first sets
    up the library's per-device state.  Returns the torch.cuda.CUDAGraph."""
    import torch
    th = grid.theta_tensor(w.theta)

    def issue():
        grid.reset()
        grid.stratify(w.ng)
        for it in range(steps):
            if fused:
                grid.fused(w.integrand, th, w.ncall, w.seed, it)
            else:
                grid.iterate(w.integrand, th, w.ncall, w.seed, it)
                if adjoint:
                    grid.adjoint(w.integrand, th, w.ncall, w.seed, it)
            if it < w.itmx:
                grid.refine(w.alpha)
            if w.itmx2 and it + 1 == w.itmx:
                grid.combine_reset()

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        issue()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        issue()
    return graph


def median_replay(graph, repeats):
    """Median wall time (ms, HIP events on the replay stream) of `repeats`
    replays of a recorded loop, with every time."""
    import torch
    times = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        graph.replay()
        t1.record()
        torch.cuda.synchronize()
        times.append(t0.elapsed_time(t1))
    return sorted(times)[len(times) // 2], times


def cpu_baseline(w, edges, budget_s=15.0):
    """The FP64 oracle, single thread, on a bounded sample of the workload:
    a short probe sets the sample count so that one oracle iteration on the
    GPU-adapted grid takes about `budget_s` seconds."""
    import oracle as O
    probe = 20_000 if w.ng <= 1 else None
    if w.ng <= 1:
        t0 = time.perf_counter()
        O.iterate(w.integrand, edges, w.theta, probe, w.seed, 999)
        rate = probe / (time.perf_counter() - t0)
        ncall = int(min(w.ncall, max(probe, budget_s * rate)))
    else:
        ncall = w.ncall
    t0 = time.perf_counter()
    r = O.iterate(w.integrand, edges, w.theta, ncall, w.seed, 1000, ng=w.ng)
    dt = time.perf_counter() - t0
    out = dict(value=r["n_eff"] / dt, unit="evals/s", cores=1, kind="oracle",
               sample=f"one oracle iteration of {r['n_eff']} samples of this workload on the GPU-adapted grid "
                      f"({dt:.1f} s, 1 thread, {platform.processor() or platform.machine()})")
    if w.ng <= 1:
        out["all_cores"] = cpu_baseline_all_cores(w, edges, min(w.ncall, 8 * ncall))
    return out


def cpu_baseline_all_cores(w, edges, ncall):
    """The same oracle with one iteration split into contiguous sample
    ranges over a pool of worker processes, one per host core available to
    this process (at most 16).  It runs in a child process that never
    touches the GPU (oracle/cpu_rate.py)."""
    import subprocess
    import tempfile

    import numpy as np
    try:
        nproc = max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        nproc = max(1, min(16, os.cpu_count() or 1))
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "edges.npy")
        np.save(path, np.asarray(edges, dtype=np.float64))
        cfg = dict(integrand=int(w.integrand), edges=path, theta=list(w.theta), ncall=int(ncall), seed=int(w.seed),
                   it=1001, nproc=nproc)
        try:
            p = subprocess.run([sys.executable, "-m", "oracle.cpu_rate", json.dumps(cfg)], cwd=ROOT,
                               capture_output=True, text=True, timeout=300)
            res = json.loads(p.stdout.strip().splitlines()[-1])
        except Exception as e:  # reported, not fatal: the GPU figures stand on their own
            return dict(error=f"{type(e).__name__}: {e}")
    return dict(value=res["samples"] / res["seconds"], unit="evals/s", cores=res["procs"], kind="oracle",
                sample=f"one oracle iteration of {res['samples']} samples split over {res['procs']} worker "
                       f"processes ({res['seconds']:.1f} s)")


def autograd_loop(grid, w, steps, fused=True):
    """`steps` iterations through torch.autograd: the forward pass
    (vegas_integral; fused: the gradient in the forward pass's kernel, else
    an adjoint pass at backward) and backward() on the differentiable
    parameters, then the refinement; returns the wall time in ms (HIP
    events)."""
    import torch

    from paper_1010_2107_amd import _lib as L
    from paper_1010_2107_amd.autograd import vegas_integral
    _, ng = L.integrand_info(w.integrand, w.dim)
    grid.reset()
    grid.stratify(w.ng)
    theta = torch.tensor(w.theta[:ng], dtype=torch.float64, device="cuda", requires_grad=True)
    fixed = tuple(w.theta[ng:])
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for it in range(steps):
        theta.grad = None
        vegas_integral(theta, grid, w.integrand, w.ncall, w.seed, it, fused=fused, fixed=fixed).backward()
        if it < w.itmx:
            grid.refine(w.alpha)
        if w.itmx2 and it + 1 == w.itmx:
            grid.combine_reset()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1)


def median_loop(grid, w, steps, repeats, **kw):
    """The run_loop of median wall time among `repeats` identical loops
    (same seeds, so the same samples and results), with every wall time."""
    runs = sorted((run_loop(grid, w, steps, **kw) for _ in range(repeats)), key=lambda r: r[0])
    return runs[len(runs) // 2], [r[0] for r in runs]


def measure_workload(grid, w, steps, warmup, repeats=5):
    """Forward loop (value), forward + separate adjoint, and fused loops,
    each the median of `repeats` replays of the loop recorded as a HIP
    graph; beside them the same loops launched call by call from the host
    (eager), whose per-launch kernel times feed the roofline."""
    from paper_1010_2107_amd import workloads as W
    if warmup:
        run_loop(grid, w, warmup)
    (ems, kms, nl), eager_ms = median_loop(grid, w, steps, repeats)
    eres = grid.result()
    ms, all_ms = median_replay(record_loop(grid, w, steps), repeats)
    res = grid.result()
    n = res["n_eff"] * steps
    out = dict(ms=ms, kms=kms, nl=nl, res=res, n_eff=res["n_eff"], value=n / (ms / 1e3), repeats_ms=all_ms,
               eager_value=eres["n_eff"] * steps / (ems / 1e3), eager_repeats_ms=eager_ms,
               graph_matches_eager=bool(abs(res["Ibar"] - eres["Ibar"]) <= 1e-9 * abs(eres["Ibar"])))
    if W.ngrad(w) > 0:
        ms_a, _ = median_replay(record_loop(grid, w, steps, adjoint=True), repeats)
        ms_f, _ = median_replay(record_loop(grid, w, steps, fused=True), repeats)
        (ems_a, _, _), _ = median_loop(grid, w, steps, repeats, adjoint=True)
        (ems_f, _, _), _ = median_loop(grid, w, steps, repeats, fused=True)
        out["fwd_adj_evals_per_s"] = n / (ms_a / 1e3)
        out["fused_evals_per_s"] = n / (ms_f / 1e3)
        out["eager_fwd_adj_evals_per_s"] = n / (ems_a / 1e3)
        out["eager_fused_evals_per_s"] = n / (ems_f / 1e3)
        autograd_loop(grid, w, steps)  # warm-up
        ag = sorted(autograd_loop(grid, w, steps) for _ in range(repeats))
        out["autograd_fwd_adj_evals_per_s"] = n / (ag[len(ag) // 2] / 1e3)
        ag2 = sorted(autograd_loop(grid, w, steps, fused=False) for _ in range(repeats))
        out["autograd_two_pass_fwd_adj_evals_per_s"] = n / (ag2[len(ag2) // 2] / 1e3)
    return out


def batched_leg():
    """The 64-integral batched configuration: one persistent launch per
    iteration (autotuned schedule) against the same integrals advanced one
    at a time through the single-grid calls."""
    import numpy as np
    import torch

    from paper_1010_2107_amd import workloads as W
    from paper_1010_2107_amd.autotune import autotune
    from paper_1010_2107_amd.batch import Batch
    from paper_1010_2107_amd.grid import Grid

    spec = W.batched_config()
    th = [spec.theta(k) for k in range(spec.n)]
    b = Batch(spec.dims, spec.ncalls, th, nbins=spec.nbins)
    (spt, blocks), _ = autotune(b, kind=1)
    calls = int(spec.ncalls.sum())

    itmx = spec.itmx + spec.itmx2

    def loop(kind):
        b.reset()
        torch.cuda.synchronize()
        b.timing(True)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        b.run(spec.seed, spec.itmx, spec.itmx2, kind=kind, freeze=spec.freeze)
        t1.record()
        torch.cuda.synchronize()
        kms, nl = b.timing(False)
        return t0.elapsed_time(t1), kms, nl

    loop(1)  # warm-up
    ms, kms, nl = loop(1)
    r = b.results()
    zs = []
    from scipy import special
    for k in range(spec.n):
        c, s_ = np.asarray(spec.centres[k]), spec.sigmas[k]
        I = np.prod(0.5 * (special.erf((1 - c) / s_) + special.erf(c / s_)))
        zs.append(abs(r["Ibar"][k] - I) / r["sigbar"][k])
    ms_f, _, _ = loop(3)
    # the same integrals one by one through the single-grid calls
    grids = {}
    for d in sorted(set(spec.dims.tolist())):
        grids[d] = Grid(d, spec.nbins)
    ths = [grids[spec.dims[k]].theta_tensor(th[k]) for k in range(spec.n)]

    def seq():
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for k in range(spec.n):
            g = grids[spec.dims[k]]
            g.reset()
            for it in range(itmx):
                if it == spec.itmx:
                    g.combine_reset()
                g.iterate(W.GAUSS_AXES, ths[k], int(spec.ncalls[k]), spec.seed, it)
                if it < spec.itmx or not spec.freeze:
                    g.refine(1.5)
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1)

    seq()
    ms_seq = seq()
    return {"integrals": spec.n, "total_calls_per_iteration": calls, "iterations": itmx,
            "phases": {"warm_up_not_combined": spec.itmx, "combined": spec.itmx2, "grid_frozen": spec.freeze},
            "schedule": {"samples_per_thread": spt, "blocks": blocks},
            "evals_per_s": calls * itmx / (ms / 1e3), "ms_per_iteration": ms / itmx,
            "kernel_ms_per_launch": kms / max(nl, 1),
            "fused_fwd_adj_evals_per_s": calls * itmx / (ms_f / 1e3),
            "sequential_single_grid_evals_per_s": calls * itmx / (ms_seq / 1e3),
            "max_z_vs_closed_form": float(max(zs)), "all_within_3_sigma": bool(max(zs) < 3)}


def spring_leg(trials=50_000_000, pilot=20_000_000, pilot_kept=20_000, max_overflow=1e-3):
    """SPRING event generation after a BASES run whose integration phase
    records the cube maxima: trials/s and kept events/s of one
    spring_generate launch, for the double Gaussian (d=8, 4^8 cubes) and for
    W + 2 partons (d=10, 2^10 cubes).  The recorded maxima come from a finite
    sample, so some trials exceed the envelope (overflow); the envelope's
    headroom over the maxima is the smallest of a ladder whose pilot run
    (other trial numbers, at least `pilot` trials and enough for about
    pilot_kept kept events, so that a fraction of max_overflow is resolved)
    keeps overflows at or below max_overflow of the kept events, and the
    timed run reports its overflow fraction."""
    import torch

    from paper_1010_2107_amd import workloads as W
    from paper_1010_2107_amd.driver import integrate
    from paper_1010_2107_amd.spring import Spring

    out = {}
    cases = [(W.C2, W.C2.ncall, W.C2.ng, W.C2.itmx, W.C2.itmx2),
             (W.C3, W.C3.ncall, 2, 5, 10)]
    for w, ncall, ng, itmx, itmx2 in cases:
        name = w.name if w is W.C2 else f"{w.name.split('_vegas')[0]}_bases_ng{ng}"
        buf = torch.zeros(ng ** w.dim, dtype=torch.float64, device="cuda")
        res = integrate(w.integrand, w.dim, w.nbins, w.theta, ncall, itmx, w.seed, ng=ng, itmx2=itmx2, cube_max=buf)
        sp = Spring(res.grid)
        cap = 1 << 22
        ev = torch.empty((cap, w.dim), dtype=torch.float32, device="cuda")
        tr = torch.empty(cap, dtype=torch.int64, device="cuda")
        ladder = []
        headroom = None
        n_pilot, h_prev = pilot, None
        for h_try in (1.0, 1.5, 2.0, 3.0, 4.0, 6.0, 8.0, 12.0, 16.0, 24.0, 32.0):
            if h_prev is not None:
                # the efficiency falls as 1/h: size the pilot for ~pilot_kept kept events
                eff_next = max(ladder[-1]["efficiency"], 1e-9) * h_prev / h_try
                n_pilot = int(min(max(pilot, pilot_kept / eff_next), 1_000_000_000))
            sp.setup(buf, h_try)
            sp.generate(w.integrand, w.theta, 7, 100, 0, n_pilot, ev, tr)
            hp = sp.header()
            frac = hp["over"] / max(hp["kept"], 1)
            ladder.append({"headroom": h_try, "trials": hp["trials"], "kept": hp["kept"],
                           "overflow_fraction_of_kept": frac, "efficiency": hp["kept"] / hp["trials"]})
            h_prev = h_try
            if frac <= max_overflow:
                headroom = h_try
                break
        if headroom is None:
            headroom = ladder[-1]["headroom"]
        t0 = time.perf_counter()
        sp.setup(buf, headroom)
        setup_ms = (time.perf_counter() - t0) * 1e3
        sp.generate(w.integrand, w.theta, 7, 0, 0, 1 << 20, ev, tr)  # warm-up
        sp.clear_counts()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sp.generate(w.integrand, w.theta, 7, 1, 0, trials, ev, tr)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        h = sp.header()
        out[name] = {"trials": h["trials"], "kept": h["kept"], "overflow": h["over"],
                     "overflow_fraction_of_kept": h["over"] / max(h["kept"], 1), "headroom": headroom,
                     "pilot_ladder": ladder,
                     "stored": min(h["slot"], cap), "ms": ms, "trials_per_s": h["trials"] / (ms / 1e3),
                     "events_per_s": h["kept"] / (ms / 1e3), "efficiency": h["kept"] / h["trials"],
                     "expected_efficiency": res.Ibar / h["env"], "cubes": h["ncubes"], "setup_ms": setup_ms,
                     "bases": {"ncall": ncall, "itmx1": itmx, "itmx2": itmx2, "Ibar": res.Ibar,
                               "sigbar": res.sigbar}}
        print(f"[bench] spring {name}: {out[name]['events_per_s']:.4g} events/s "
              f"({out[name]['trials_per_s']:.4g} trials/s), headroom {headroom}, overflow "
              f"{out[name]['overflow_fraction_of_kept']:.2e} of kept", file=sys.stderr, flush=True)
    return out


# The paper's GPU timings of its own process, u dbar -> W+ + n gluons, on a
# GTX285 (Table 7; NCALL = 1e6 for n <= 2, ITMX = 10 or ITMX1 = ITMX2 = 5),
# as calls per second: context only, other hardware.
PAPER_GTX285_CALLS_PER_S = {0: {"vegas": 1 / 0.0207e-6, "bases": 1 / 0.0260e-6},
                            1: {"vegas": 1 / 0.0318e-6, "bases": 1 / 0.0396e-6},
                            2: {"vegas": 1 / 0.0497e-6, "bases": 1 / 0.0563e-6}}


def paper_process_leg():
    """The paper's process at the paper's run sizes (Table 5: NCALL 1e6,
    ITMX 10 for VEGAS, ITMX1 = ITMX2 = 5 for BASES), helicity amplitudes in
    FP32, whole iteration loop timed (sample pass, publish, refine): the
    median of 5 replays of the loop recorded as a HIP graph, and of 5 eager
    loops."""
    import torch

    from paper_1010_2107_amd import workloads as W
    from paper_1010_2107_amd.grid import Grid

    out = {}
    for n in (0, 1, 2):
        d = 3 * n + 5
        ng = W.default_ng(1_000_000, d, 64)  # ng^d <= NCALL / 2
        for mode in ("vegas", "bases"):
            w = W.Workload(f"whel{n}_d{d}_{mode}", W.WHEL, d, 64, 1_000_000, 10 if mode == "vegas" else 5,
                           W.WHEL_THETA, ng=1 if mode == "vegas" else ng, itmx2=0 if mode == "vegas" else 5)
            g = Grid(d, 64)
            steps = w.itmx + w.itmx2
            run_loop(g, w, steps)  # warm-up
            (ems, kms, nl), _ = median_loop(g, w, steps, 5)
            ms, _ = median_replay(record_loop(g, w, steps), 5)
            r = g.result()
            rate = r["n_eff"] * steps / (ms / 1e3)
            out[w.name] = {"calls_per_s": rate, "eager_calls_per_s": r["n_eff"] * steps / (ems / 1e3),
                           "kernel_ms_per_launch": kms / max(nl, 1), "Ibar": r["Ibar"],
                           "sigbar": r["sigbar"], "paper_gtx285_calls_per_s": PAPER_GTX285_CALLS_PER_S[n][mode]}
    return out


def host_accumulate(w, j, nbins):
    """Steps 4 of the paper's split (Sec. 3.2) on the host: FP64 sums of the
    weights w [n] (FP32 from the GPU) and of their squares, in total and per
    axis and bin, from the bin indices j [n][d] (uint8, from the GPU)."""
    import numpy as np
    wv = np.asarray(w, dtype=np.float64)
    jv = np.asarray(j)
    d = jv.shape[1]
    bins = np.zeros((2, d, nbins))
    w2 = wv * wv
    for a in range(d):
        bins[0, a] = np.bincount(jv[:, a], weights=wv, minlength=nbins)
        bins[1, a] = np.bincount(jv[:, a], weights=w2, minlength=nbins)
    return float(wv.sum()), float(w2.sum()), bins


def host_refine(edges, b2, alpha):
    """Step 5 of the paper's split on the host: per axis, 3-point smoothing
    of the per-bin sums of w^2 (2-point at the ends), normalisation,
    damping ((1 - rho)/(-ln rho))^alpha (0 at rho = 0, 1 at rho = 1), and new
    edges that cut the damped weight into equal pieces (Lepage 1978).  An
    axis whose smoothed sum is not positive and finite is kept."""
    import numpy as np
    e = np.array(edges, dtype=np.float64)
    d, n1 = e.shape
    N = n1 - 1
    for a in range(d):
        c = np.asarray(b2[a], dtype=np.float64)
        sm = np.empty(N)
        sm[0] = (c[0] + c[1]) / 2.0
        sm[N - 1] = (c[N - 2] + c[N - 1]) / 2.0
        sm[1:N - 1] = (c[:N - 2] + c[1:N - 1] + c[2:]) / 3.0
        D = sm.sum()
        if not (D > 0.0 and np.isfinite(D)):
            continue
        rho = sm / D
        with np.errstate(divide="ignore", invalid="ignore"):
            base = np.where(rho <= 0.0, 0.0, np.where(rho >= 1.0, 1.0, (1.0 - rho) / -np.log(rho)))
        r = base ** alpha
        C = np.concatenate([[0.0], np.cumsum(r)])
        targets = np.arange(1, N) * (C[N] / N)
        j = np.minimum(np.searchsorted(C[1:], targets, side="right"), N - 1)  # smallest j with C[j+1] > target
        e[a, 1:N] = e[a, j] + (targets - C[j]) / r[j] * (e[a, j + 1] - e[a, j])
    return e


def host_accumulation_leg(iters=3):
    """The paper's split of the work (Sec. 3.2): the GPU generates the
    points and evaluates the integrand; the weights and the bin indices
    (both from the library's per-sample dump) are copied to pinned host
    memory; the host accumulates the sums and per-bin sums in FP64 and
    re-optimises the grid, whose edges go back to the GPU for the next
    iteration.  Same workload as the GPU-resident path, timed beside it."""
    import numpy as np
    import torch

    from paper_1010_2107_amd import workloads as W
    from paper_1010_2107_amd.grid import Grid

    w = W.C2_PLAIN
    d, N, n = w.dim, w.nbins, w.ncall
    g = Grid(d, N)
    th = g.theta_tensor(w.theta)
    wt = torch.empty(n, dtype=torch.float32, device="cuda")
    jt = torch.empty((n, d), dtype=torch.uint8, device="cuda")
    w_h = torch.empty(n, dtype=torch.float32, pin_memory=True)
    j_h = torch.empty((n, d), dtype=torch.uint8, pin_memory=True)
    split = {"gpu_ms": 0.0, "d2h_ms": 0.0, "host_accumulate_ms": 0.0, "host_refine_ms": 0.0, "h2d_edges_ms": 0.0}
    rel = 0.0
    edges = g.get_edges()
    for it in range(iters + 1):
        timed = it > 0  # the first iteration is warm-up
        t0 = time.perf_counter()
        g.dump_into(w.integrand, th, n, w.seed, it, 0, w=wt, bins=jt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        w_h.copy_(wt, non_blocking=True)
        j_h.copy_(jt, non_blocking=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        S1, S2, bins = host_accumulate(w_h.numpy(), j_h.numpy(), N)
        I = S1 / n
        var = (S2 / n - I * I) / (n - 1)
        t3 = time.perf_counter()
        edges = host_refine(edges, bins[1], w.alpha)
        t4 = time.perf_counter()
        if it == 1:  # the GPU-resident pass on the same grid and samples (untimed)
            g.iterate(w.integrand, th, n, w.seed, it)
            r = g.result()
            rel = max(abs(r["S1"] - S1) / abs(S1), abs(r["S2"] - S2) / S2)
        t5 = time.perf_counter()
        g.set_edges(edges)  # synchronous copy to the device
        t6 = time.perf_counter()
        if timed:
            split["gpu_ms"] += (t1 - t0) * 1e3
            split["d2h_ms"] += (t2 - t1) * 1e3
            split["host_accumulate_ms"] += (t3 - t2) * 1e3
            split["host_refine_ms"] += (t4 - t3) * 1e3
            split["h2d_edges_ms"] += (t6 - t5) * 1e3
    total_ms = sum(split.values())
    return {"workload": w.name, "iterations": iters, "evals_per_s": n * iters / (total_ms / 1e3),
            "ms_per_iteration": {k: v / iters for k, v in split.items()},
            "bytes_d2h_per_iteration": n * (4 + d), "host_cores": 1,
            "max_rel_diff_vs_gpu_sums": rel, "estimate_last_iteration": {"I": I, "var": var}}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the other workloads and the batched leg")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--pmc-mode", action="store_true",
                    help="for hardware-counter runs: a plain 1 GiB device copy (calibrates FETCH_SIZE and "
                         "WRITE_SIZE), then the workload's forward loop only")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding of the "
              "sample pass is a design note, not a built path", file=sys.stderr)
        return 2

    import torch

    from paper_1010_2107_amd import census
    from paper_1010_2107_amd import workloads as W
    from paper_1010_2107_amd.grid import Grid

    w = W.CONFIGS[args.workload] if args.workload else W.DEFAULT_BENCH
    steps = args.steps if args.steps is not None else w.itmx + w.itmx2
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.pmc_mode:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)  # 1 GiB read + 1 GiB written
        torch.cuda.synchronize()
        grid = Grid(w.dim, w.nbins)
        ms, kms, nl = run_loop(grid, w, steps)
        print(json.dumps({"pmc_mode": True, "workload": w.name, "steps": steps, "kernel_ms": kms / max(nl, 1),
                          "copy_bytes_each_way": src.numel() * 4, "source_sha1": source_sha1()}), flush=True)
        return 0
    print(f"[bench] workload {w.name} steps {steps} warmup {args.warmup}", file=sys.stderr, flush=True)
    grid = Grid(w.dim, w.nbins)
    m = measure_workload(grid, w, steps, args.warmup)
    res, n_eff = m["res"], m["n_eff"]
    edges = grid.get_edges()
    print(f"[bench] fwd {m['value']:.4g} evals/s, Ibar {res['Ibar']:.6g} +- {res['sigbar']:.3g}", file=sys.stderr,
          flush=True)
    z = None if w.I_ref is None or res["sigbar"] == 0 else abs(res["Ibar"] - w.I_ref) / res["sigbar"]
    ref_note = None
    if w.I_ref is None and w.integrand == W.WJETS:
        import json as _j
        p = os.path.join(ROOT, "tests", "golden", "wjets_reference.json")
        if os.path.exists(p):
            ref = _j.load(open(p)).get(str(w.dim))
            if ref:
                z = abs(res["Ibar"] - ref["Ibar"]) / math.hypot(res["sigbar"], ref["sigbar"])
                ref_note = {"I_ref": ref["Ibar"], "sig_ref": ref["sigbar"], "source": "FP64 oracle, independent seed"}

    # achieved: the algorithm's operation count per sample (census.ALGORITHMIC)
    # x samples per launch / average launch; beside it the same for the
    # FP32 operations the kernel's source executes (census.for_workload)
    cen = census.for_workload(w)
    frac_pass = 1.0 - res["n_zero"] / max(n_eff, 1)
    executed = cen.flops(frac_pass)
    alg = census.algorithmic_flops(w, frac_pass)
    flops = alg if alg is not None else executed
    avg_ms = m["kms"] / max(m["nl"], 1)
    achieved = flops * n_eff / (avg_ms / 1e3) / 1e12
    ex_achieved = executed * n_eff / (avg_ms / 1e3) / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(w.name),
            "kernel": "sample-and-accumulate (forward)", "avg_launch_ms": avg_ms, "launches": m["nl"],
            "flops_per_sample": flops,
            "flops_basis": "the algorithm's operation count per sample" if alg is not None
            else "the FP32 operations the kernel source executes per sample",
            "accepted_fraction": frac_pass, "samples_per_launch": n_eff,
            "executed": {"flops_per_sample": executed, "achieved": ex_achieved,
                         "frac": ex_achieved / PEAK_FP32_TFLOPS,
                         "note": "FP32 operations of the kernel source (the arithmetic it actually does)"}}
    # the kernel against the rates probe kernels measure on this chip: FP32 FMA
    # issue (packed FP32 off, at the clock held under load) and LDS FP64 adds
    from paper_1010_2107_amd import _lib as L
    import ctypes
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    fma = ctypes.c_double()
    L.call("vmc_probe_fp32_fma", 8192, 4096, ctypes.byref(fma), stream)
    roof["fp32_fma_probe"] = {"peak_tflops": fma.value / 1e12, "frac": achieved / (fma.value / 1e12),
                              "executed_frac": ex_achieved / (fma.value / 1e12),
                              "note": "8 independent FP32 FMA chains per lane, packed FP32 off"}
    # VALU issue estimate: the counted VALU wave instructions at the FMA
    # probe's issue rate (one wave FMA = 2 x 64 flops per 4 cycles per SIMD).
    # An estimate, not a bound: some instructions issue faster, so the ratio
    # can exceed 1; near 1 it says the VALU issue is what the launch waits on.
    valu = measured_valu(w.name)
    if valu:
        issue = fma.value / 128.0
        t_issue = valu / issue
        roof["valu_issue"] = {
            "valu_per_launch": valu, "valu_per_64_samples": valu * 64.0 / n_eff,
            "issue_time_ms": t_issue * 1e3, "issue_time_over_launch": t_issue / (avg_ms / 1e3),
            "note": "SQ_INSTS_VALU from the committed counter summary (same kernel sources) at the FMA probe's "
                    "issue rate; an estimate, not a bound"}
    else:
        roof["valu_issue"] = None
    peak = ctypes.c_double()
    L.call("vmc_probe_lds_atomics", 2048, 4096, ctypes.byref(peak), stream)
    lds_achieved = 2 * w.dim * n_eff / (avg_ms / 1e3)
    roof["lds_atomics"] = {"achieved_per_s": lds_achieved, "peak_per_s": peak.value,
                           "frac": lds_achieved / peak.value,
                           "note": "2 dim FP64 LDS adds per sample; peak from a conflict-free probe kernel"}
    line = {
        "metric": "integrand evals/s (fwd)", "value": m["value"], "unit": "evals/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": m["ms"] / steps, "repeats": len(m["repeats_ms"]),
        "loop_ms_of_repeats": m["repeats_ms"],
        "loop": "the K-step loop recorded once as a HIP graph and replayed (median of the repeats)",
        "eager_evals_per_s": m["eager_value"], "eager_loop_ms_of_repeats": m["eager_repeats_ms"],
        "graph_matches_eager": m["graph_matches_eager"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 integrand, f64 sums", "data": "synthetic (counter-based Philox samples)",
        "config": {"workload": w.name, "dim": w.dim, "nbins": w.nbins, "ncall": w.ncall, "n_eff": n_eff,
                   "iterations": steps, "mode": "bases-stratified" if w.ng > 1 else "vegas",
                   "ng": w.ng, "parallelism": "single-gpu"},
        "result": {"Ibar": res["Ibar"], "sigbar": res["sigbar"], "chi2dof": res["chi2dof"],
                   "I_ref": w.I_ref if ref_note is None else ref_note, "z": z,
                   "within_3_sigma": None if z is None else bool(z < 3)},
        "roofline": roof,
    }
    for key in ("fwd_adj_evals_per_s", "fused_evals_per_s", "eager_fwd_adj_evals_per_s", "eager_fused_evals_per_s",
                "autograd_fwd_adj_evals_per_s", "autograd_two_pass_fwd_adj_evals_per_s"):
        if key in m:
            line[key] = m[key]
    if not args.no_secondary:
        sec = {}
        for w2 in (W.C2, W.C2_PLAIN, W.C3, W.C6, W.C3_BASES, W.C4_BASES):
            if w2.name == w.name:
                continue
            g2 = Grid(w2.dim, w2.nbins)
            m2 = measure_workload(g2, w2, w2.itmx + w2.itmx2, 1)
            r2 = m2["res"]
            z2 = None if w2.I_ref is None else abs(r2["Ibar"] - w2.I_ref) / r2["sigbar"]
            golden = {W.WHEL: "whel_reference.json", W.WJETS: "wjets_reference.json"}.get(w2.integrand)
            if golden:  # independent-seed oracle references of the physics integrands
                p = os.path.join(ROOT, "tests", "golden", golden)
                ref = json.load(open(p)).get(str(w2.dim)) if os.path.exists(p) else None
                if ref:
                    z2 = abs(r2["Ibar"] - ref["Ibar"]) / math.hypot(r2["sigbar"], ref["sigbar"])
            sec[w2.name] = {k: m2[k] for k in ("value", "eager_value", "fwd_adj_evals_per_s", "fused_evals_per_s",
                                               "autograd_fwd_adj_evals_per_s",
                                               "autograd_two_pass_fwd_adj_evals_per_s", "graph_matches_eager")
                            if k in m2}
            sec[w2.name].update({"Ibar": r2["Ibar"], "sigbar": r2["sigbar"], "z": z2,
                                 "kernel_ms_per_launch": m2["kms"] / max(m2["nl"], 1)})
            print(f"[bench] {w2.name}: {m2['value']:.4g} evals/s", file=sys.stderr, flush=True)
        line["secondary"] = sec
        print("[bench] batched leg", file=sys.stderr, flush=True)
        line["batched"] = batched_leg()
        print("[bench] paper's process at the paper's sizes", file=sys.stderr, flush=True)
        line["paper_process"] = paper_process_leg()
        print("[bench] spring leg", file=sys.stderr, flush=True)
        line["spring"] = spring_leg()
        print("[bench] host-accumulation ablation", file=sys.stderr, flush=True)
        line["host_accumulation_ablation"] = host_accumulation_leg()
        gpu_path = sec.get(W.C2_PLAIN.name, {}).get("value")
        if gpu_path:
            line["host_accumulation_ablation"]["gpu_resident_evals_per_s"] = gpu_path
            line["host_accumulation_ablation"]["gpu_resident_speedup"] = \
                gpu_path / line["host_accumulation_ablation"]["evals_per_s"]
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, edges, args.cpu_budget)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
