"""Write tests/golden/whel_reference.json: reference integrals of
u dbar -> W+(-> mu+ nu) + n gluons from helicity amplitudes (n = 1, d = 8;
n = 2, d = 11) computed with the FP64 oracle only, on a Philox seed
independent of the GPU tests' seed.

One VEGAS run per dimension (ITMX iterations of NCALL samples, 64 bins per
axis, damping 1.5), each iteration's samples split into contiguous ranges
over worker processes and summed (oracle.iterate_sharded), then refined and
combined with weights 1/var.
Run:  python tests/golden/make_whel_reference.py   (a few minutes on 8 cores)
"""
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402

THETA = (80.4, 2.1, math.sqrt(4 * math.pi * 0.118), 14000.0, 20.0, 2.5, 5.0, 20.0)
NBINS, ALPHA, SEED = 64, 1.5, 4321
RUNS = {8: (5_000_000, 10), 11: (10_000_000, 15)}


def main(nproc=8):
    out = {"theta": THETA, "nbins": NBINS, "alpha": ALPHA, "seed": SEED,
           "note": "written by tests/golden/make_whel_reference.py from the FP64 oracle only"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "whel_reference.json")
    with mp.get_context("fork").Pool(nproc) as pool:
        for d, (ncall, itmx) in RUNS.items():
            e = O.uniform_edges(d, NBINS)
            Is, vs = [], []
            t0 = time.time()
            for it in range(itmx):
                r = O.iterate_sharded(O.WHEL, e, THETA, ncall, SEED, it, pool, 4 * nproc)
                Is.append(r["I"])
                vs.append(r["var"])
                e = O.refine(e, r["bins"][1], ALPHA)
                print(f"d={d} it={it} I={r['I']:.6g} sd={math.sqrt(r['var']):.3g} ({time.time() - t0:.0f}s)",
                      flush=True)
            Ib, sb, chi = O.combine(Is, vs)
            out[str(d)] = {"ncall": ncall, "itmx": itmx, "Ibar": Ib, "sigbar": sb, "chi2dof": chi,
                           "I": Is, "var": vs}
            with open(path, "w") as f:
                json.dump(out, f, indent=1)
    print(json.dumps({k: {kk: vv for kk, vv in v.items() if kk not in ("I", "var")} if isinstance(v, dict) else v
                      for k, v in out.items()}, indent=1))


if __name__ == "__main__":
    main()
