"""Autotuner for the batched persistent launch: times candidate schedules
(samples per thread = tile size / 256, and persistent grid size) on the
batch itself and keeps the fastest; results are cached on disk, keyed by the
batch's shape (dimensions, call counts, bins), the pass kind and the device.

Every schedule gives the same samples (counter-based words), so tuning only
changes speed; results agree to FP64 summation order."""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np
import torch

SPT = (2, 4, 8, 16, 32, 64, 128)
BLOCKS = (512, 1024, 2048, 4096)


def cache_path():
    base = os.environ.get("VMC_AUTOTUNE_CACHE")
    if base:
        return base
    root = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(root, "paper_1010_2107_amd", "autotune.json")


def batch_key(batch, kind):
    dev = torch.cuda.get_device_name(batch.device)
    h = hashlib.sha1()
    h.update(batch.dims.tobytes())
    h.update(batch.ncalls.tobytes())
    h.update(f"{batch.nbins}|{kind}|{dev}".encode())
    return h.hexdigest()


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + f".{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1)
    os.replace(tmp, p)


def measure(batch, spt, blocks, kind=1, reps=3, seed=99):
    """Median kernel time (ms) of `reps` launches with this schedule."""
    batch.set_schedule(spt, blocks)
    batch.reset()
    if kind == 2:  # an adjoint pass differentiates the forward pass on the same grids
        batch.iterate(seed, 0, 1)
    batch.iterate(seed, 0, kind)  # warm-up
    torch.cuda.synchronize()
    batch.timing(True)
    times = []
    for r in range(reps):
        batch.iterate(seed, r + 1, kind)
        torch.cuda.synchronize()
        ms, _ = batch.timing(True)
        times.append(ms)
    batch.timing(False)
    return float(np.median(times))


def autotune(batch, kind=1, use_cache=True, candidates=None, verbose=False):
    """Pick (samples_per_thread, blocks) for `batch`, apply it and return it
    with the measured table."""
    key = batch_key(batch, kind)
    db = _load() if use_cache else {}
    if key in db:
        spt, blocks = db[key]["best"]
        batch.set_schedule(spt, blocks)
        batch.reset()
        return (spt, blocks), db[key]["table"]
    cands = candidates or [(s, b) for s in SPT for b in BLOCKS]
    table = []
    t0 = time.time()
    for s, b in cands:
        ms = measure(batch, s, b, kind)
        table.append((s, b, ms))
        if verbose:
            print(f"  spt {s:4d} blocks {b:5d}: {ms:.4f} ms", flush=True)
    best = min(table, key=lambda r: r[2])
    batch.set_schedule(best[0], best[1])
    batch.reset()
    if use_cache:
        db[key] = {"best": [best[0], best[1]], "table": table, "seconds": time.time() - t0}
        _store(db)
    return (best[0], best[1]), table
