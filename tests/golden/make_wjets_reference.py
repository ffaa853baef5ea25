"""Write tests/golden/wjets_reference.json: reference integrals of the
W + 2 partons (d=10) and W + 4 partons (d=16) toy cross sections, computed
with the FP64 oracle only, on seeds independent of the GPU tests' seeds.

Each dimension gets NRUNS independent VEGAS runs (different Philox seeds),
each ITMX iterations of NCALL samples on 64 bins per axis; the runs'
combined estimates are independent and are merged with weights 1/sigma^2.
Run:  python tests/golden/make_wjets_reference.py   (about 30 minutes on 8 cores)
"""
import json
import math
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

THETA = (80.4, 2.1, math.sqrt(4 * math.pi * 0.118), 14000.0, 20.0, 2.5, 0.4)
NRUNS, NBINS = 8, 64
NCALL = {10: 5_000_000, 16: 5_000_000}
ITMX = {10: 10, 16: 15}


def one(args):
    import oracle as O
    d, seed = args
    run = O.integrate(O.WJETS, d, NBINS, THETA, NCALL[d], ITMX[d], seed)
    return dict(seed=seed, Ibar=run.Ibar, sigbar=run.sigbar, chi2dof=run.chi2dof)


def main():
    jobs = [(d, 900_000 + 100 * d + r) for d in (10, 16) for r in range(NRUNS)]
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(one, jobs)
    out = {"theta": THETA, "nbins": NBINS, "runs": NRUNS,
           "note": "written by tests/golden/make_wjets_reference.py from the FP64 oracle only"}
    for d in (10, 16):
        rs = [r for (dd, _), r in zip(jobs, res) if dd == d]
        w = [1 / r["sigbar"] ** 2 for r in rs]
        I = sum(wi * r["Ibar"] for wi, r in zip(w, rs)) / sum(w)
        s = sum(w) ** -0.5
        chi = sum((r["Ibar"] - I) ** 2 / r["sigbar"] ** 2 for r in rs) / (len(rs) - 1)
        out[str(d)] = {"ncall": NCALL[d], "itmx": ITMX[d], "Ibar": I, "sigbar": s, "chi2dof_between_runs": chi, "runs": rs}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wjets_reference.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: (v if not isinstance(v, dict) else {kk: vv for kk, vv in v.items() if kk != "runs"})
                      for k, v in out.items()}, indent=1))


if __name__ == "__main__":
    main()
