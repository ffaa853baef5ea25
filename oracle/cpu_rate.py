"""Host-core timing of the FP64 oracle (test infrastructure: run only by the
CPU-baseline leg of the benchmark, in a process of its own that never
touches a GPU).

One plain-mode iteration is split into contiguous sample ranges that a pool
of worker processes (fork start) evaluates; the shards' sums are added as
``iterate_sharded`` does.  Usage:

    python -m oracle.cpu_rate '{"integrand": 5, "edges": "/path/edges.npy",
        "theta": [...], "ncall": 8000000, "seed": 1234, "it": 1001, "nproc": 16}'

prints one JSON object: samples, seconds, worker processes, and the
estimate of the iteration (I, var) so that the caller can check it.
"""
import json
import multiprocessing as mp
import sys
import time

import numpy as np

from oracle import iterate_sharded


def main(argv):
    cfg = json.loads(argv[1])
    edges = np.load(cfg["edges"])
    nproc = int(cfg["nproc"])
    with mp.get_context("fork").Pool(nproc) as pool:
        pool.map(abs, range(nproc))  # workers up before the clock starts
        t0 = time.perf_counter()
        r = iterate_sharded(cfg["integrand"], edges, cfg["theta"], int(cfg["ncall"]), int(cfg["seed"]),
                            int(cfg["it"]), pool, 4 * nproc)
        dt = time.perf_counter() - t0
    print(json.dumps({"samples": int(cfg["ncall"]), "seconds": dt, "procs": nproc, "I": r["I"], "var": r["var"]}))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
