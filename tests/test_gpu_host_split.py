"""The paper's split of the work (Sec. 3.2) run on the GPU and the host: the
library dumps each sample's FP32 weight and bin indices, the host
accumulates and refines (the bench's ablation leg).  Bin indices equal the
oracle's bit for bit; host sums against the oracle at the same FP32 point
(S1 and plane 0 1e-5, S2 and plane 1 2e-5) and against the oracle's replay
of the dumped weights (1e-12); the host refinement against the oracle's on
the oracle's sums (1e-12); and two host-split iterations against the
GPU-resident pass and its refinement on the same grid (same FP32 weights,
so 1e-12)."""
import numpy as np
import pytest
import torch

import bench
import oracle as O
from paper_1010_2107_amd import workloads as W
from paper_1010_2107_amd.grid import Grid
from tests.gpu_util import announce, normwise, rel, require_gpu

pytestmark = pytest.mark.gpu


def test_host_split_matches_oracle_and_gpu_resident_pass():
    require_gpu()
    w = W.C2_PLAIN
    d, N, ncall = w.dim, w.nbins, 200_003
    announce(f"host split {w.name} ncall={ncall}")
    g = Grid(d, N)
    ref_grid = Grid(d, N)
    edges = O.integrate(w.integrand, d, N, w.theta, 50_000, 2, 9).edges
    g.set_edges(edges)
    ref_grid.set_edges(edges)
    wt = torch.empty(ncall, dtype=torch.float32, device="cuda")
    jt = torch.empty((ncall, d), dtype=torch.uint8, device="cuda")
    for it in range(2):
        g.dump_into(w.integrand, w.theta, ncall, w.seed, it, 0, w=wt, bins=jt)
        wh, jh = wt.cpu().numpy(), jt.cpu().numpy()
        S1, S2, bins = bench.host_accumulate(wh, jh, N)
        if it == 0:
            smp = O.eval_samples(w.integrand, edges, w.theta, ncall, w.seed, it, 0, ncall, fp32_point=True)
            assert np.array_equal(jh.astype(np.int32), smp["j"])
            o32 = O.iterate(w.integrand, edges, w.theta, ncall, w.seed, it, fp32_point=True)
            assert rel(S1, o32["S1"]) <= 1e-5 and rel(S2, o32["S2"]) <= 2e-5
            assert normwise(bins[0], o32["bins"][0]) <= 1e-5 and normwise(bins[1], o32["bins"][1]) <= 2e-5
            rep = O.iterate(w.integrand, edges, w.theta, ncall, w.seed, it, w_in=wh)
            assert rel(S1, rep["S1"]) <= 1e-12 and rel(S2, rep["S2"]) <= 1e-12
            assert normwise(bins, rep["bins"]) <= 1e-12
            # the host refinement is the oracle's on the oracle's own sums
            assert np.max(np.abs(bench.host_refine(edges, o32["bins"][1], w.alpha) -
                                 O.refine(edges, o32["bins"][1], w.alpha))) <= 1e-12
        # the GPU-resident pass on the same grid adds the same FP32 weights
        ref_grid.iterate(w.integrand, w.theta, ncall, w.seed, it)
        r = ref_grid.result()
        assert rel(S1, r["S1"]) <= 1e-12 and rel(S2, r["S2"]) <= 1e-12
        assert normwise(bins, ref_grid.bins.cpu().numpy()) <= 1e-12
        new = bench.host_refine(edges, bins[1], w.alpha)
        ref_grid.refine(w.alpha)
        assert np.max(np.abs(new - ref_grid.get_edges())) <= 1e-12
        edges = new
        g.set_edges(edges)
        ref_grid.set_edges(edges)
