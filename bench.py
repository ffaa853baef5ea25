"""Benchmark of the VEGAS/BASES hot path on one MI355X.

A step is one iteration of the workload: the sample-and-accumulate pass
(Philox words -> grid map -> integrand -> FP64 per-bin sums), the estimate
and running combination, and (in the grid-optimisation phase) the grid
refinement.  `value` is integrand evaluations per second over the timed
steps (fail-cut samples count as evaluations, as NCALL does in the paper).

Prints ONE JSON line.  See the design doc for the flop census, the roofline peak
and how the CPU baseline sample is chosen.
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
    """Hash of the kernel sources and the public header, identifying the
    kernel build that a hardware-counter summary was taken on."""
    import glob
    import hashlib
    h = hashlib.sha1()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1010_2107_amd", "csrc", "*"))) + [
        os.path.join(ROOT, "include", "vmc.h")]
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name):
    """HBM bytes per launch of the forward sample kernel from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy
    calibration), or None when the summary is missing or was taken on other
    kernel sources."""
    p = os.path.join(ROOT, "profiles", f"pmc_sample_kernel_{workload_name}.txt")
    if not os.path.exists(p):
        return None
    kv = {}
    for line in open(p):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source-sha1") != source_sha1():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak (packed FMA): 256 CU x 2.4 GHz x 256 flop/clk
PEAK_FP32_NONPACKED = 78.6   # the same without packed FP32 (this build disables packed FP32)


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
    return dict(value=r["n_eff"] / dt, unit="evals/s", cores=1, kind="oracle",
                sample=f"one oracle iteration of {r['n_eff']} samples of this workload on the GPU-adapted grid "
                       f"({dt:.1f} s, 1 thread, {platform.processor() or platform.machine()})")


def measure_workload(grid, w, steps, warmup):
    """Forward loop (value), forward + separate adjoint, and fused loops."""
    from paper_1010_2107_amd import workloads as W
    if warmup:
        run_loop(grid, w, warmup)
    ms, kms, nl = run_loop(grid, w, steps)
    res = grid.result()
    out = dict(ms=ms, kms=kms, nl=nl, res=res, n_eff=res["n_eff"], value=res["n_eff"] * steps / (ms / 1e3))
    if W.ngrad(w) > 0:
        ms_a, _, _ = run_loop(grid, w, steps, adjoint=True)
        ms_f, _, _ = run_loop(grid, w, steps, fused=True)
        out["fwd_adj_evals_per_s"] = res["n_eff"] * steps / (ms_a / 1e3)
        out["fused_evals_per_s"] = res["n_eff"] * steps / (ms_f / 1e3)
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

    cen = census.for_workload(w)
    frac_pass = 1.0 - res["n_zero"] / max(n_eff, 1)
    flops = cen.flops(frac_pass)
    avg_ms = m["kms"] / max(m["nl"], 1)
    achieved = flops * n_eff / (avg_ms / 1e3) / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(w.name),
            "frac_nonpacked_peak": achieved / PEAK_FP32_NONPACKED,
            "kernel": "sample-and-accumulate (forward)", "avg_launch_ms": avg_ms, "launches": m["nl"],
            "flops_per_sample": flops, "accepted_fraction": frac_pass, "samples_per_launch": n_eff}
    line = {
        "metric": "integrand evals/s (fwd)", "value": m["value"], "unit": "evals/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": m["ms"] / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 integrand, f64 sums", "data": "synthetic (counter-based Philox samples)",
        "config": {"workload": w.name, "dim": w.dim, "nbins": w.nbins, "ncall": w.ncall, "n_eff": n_eff,
                   "iterations": steps, "mode": "bases-stratified" if w.ng > 1 else "vegas",
                   "ng": w.ng, "parallelism": "single-gpu"},
        "result": {"Ibar": res["Ibar"], "sigbar": res["sigbar"], "chi2dof": res["chi2dof"],
                   "I_ref": w.I_ref if ref_note is None else ref_note, "z": z,
                   "within_3_sigma": None if z is None else bool(z < 3)},
        "roofline": roof,
    }
    for key in ("fwd_adj_evals_per_s", "fused_evals_per_s"):
        if key in m:
            line[key] = m[key]
    if not args.no_secondary:
        sec = {}
        for w2 in (W.C2, W.C2_PLAIN, W.C3):
            if w2.name == w.name:
                continue
            g2 = Grid(w2.dim, w2.nbins)
            m2 = measure_workload(g2, w2, w2.itmx + w2.itmx2, 1)
            r2 = m2["res"]
            z2 = None if w2.I_ref is None else abs(r2["Ibar"] - w2.I_ref) / r2["sigbar"]
            sec[w2.name] = {k: m2[k] for k in ("value", "fwd_adj_evals_per_s", "fused_evals_per_s") if k in m2}
            sec[w2.name].update({"Ibar": r2["Ibar"], "sigbar": r2["sigbar"], "z": z2,
                                 "kernel_ms_per_launch": m2["kms"] / max(m2["nl"], 1)})
            print(f"[bench] {w2.name}: {m2['value']:.4g} evals/s", file=sys.stderr, flush=True)
        line["secondary"] = sec
        print("[bench] batched leg", file=sys.stderr, flush=True)
        line["batched"] = batched_leg()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, edges, args.cpu_budget)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
