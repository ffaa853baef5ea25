"""Host driver of the iteration loop (step 6 of the six-step structure,
paper Sec. 3.1): VEGAS runs ITMX iterations; BASES runs ITMX1 grid-
optimisation iterations and then ITMX2 integration iterations with the grid
frozen, combining only the latter (Sec. 3.1 and 6.1).  Each iteration is
stream-ordered library work; the host reads results once at the end unless
an accuracy target (ACC) asks for a check after every iteration.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from .grid import Grid


@dataclass
class Result:
    I: np.ndarray
    var: np.ndarray
    Ibar: float
    sigbar: float
    chi2dof: float
    n_eff: int
    niter: int
    grid: Grid


def integrate(integrand, dim, nbins, theta, ncall, itmx, seed, alpha=1.5, ng=1, itmx2=0, acc=0.0, fp64=False,
              grid: Grid | None = None, it0=0, stream=None, cube_max: torch.Tensor | None = None,
              callback=None) -> Result:
    """cube_max (BASES only): a float64 device buffer of ng^dim entries that
    receives each cube's largest weight over the integration phase, the
    input of SPRING event generation.  callback(grid, k), if given, runs on
    the host before the sample pass of iteration k (k counts both phases),
    e.g. to log, checkpoint or replace the grid."""
    g = grid if grid is not None else Grid(dim, nbins)
    assert (g.dim, g.nbins) == (dim, nbins)
    g.reset(stream)
    g.stratify(ng)
    th = g.theta_tensor(theta)
    total = itmx + itmx2
    hist = torch.zeros((total, 2), dtype=torch.float64, device=g.device)
    it, k, n_eff = it0, 0, 0
    phases = [(itmx, True)] + ([(itmx2, False)] if itmx2 else [])
    for p, (nit, adapt) in enumerate(phases):
        if p > 0:
            g.combine_reset(stream)
            if cube_max is not None:
                cube_max.zero_()
                g.bind_cube_max(cube_max)
        for _ in range(nit):
            if callback is not None:
                callback(g, k)
            g.iterate(integrand, th, ncall, seed, it, fp64=fp64, stream=stream)
            hist[k] = g.scal[L.S_I:L.S_VAR + 1]
            k += 1
            it += 1
            if adapt:
                g.refine(alpha, stream)
            if acc > 0:
                r = g.result()
                if r["Ibar"] != 0 and r["sigbar"] / abs(r["Ibar"]) < acc:
                    break
    if cube_max is not None:
        g.bind_cube_max(None)
    r = g.result()
    h = hist[:k].cpu().numpy()
    return Result(I=h[:, 0], var=h[:, 1], Ibar=r["Ibar"], sigbar=r["sigbar"], chi2dof=r["chi2dof"],
                  n_eff=int(r["n_eff"]) * k, niter=r["niter"], grid=g)


class GraphedLoop:
    """The loop of integrate() (VEGAS, or BASES with its two phases, from a
    uniform grid) recorded once as a HIP graph over the library's
    stream-ordered launches and replayed by run(): one graph launch per
    integration instead of three or four launches per iteration, for runs
    whose iterations are short enough for launch gaps to show (the paper's
    process at NCALL 1e6 takes 20-60 us per iteration).  Every replay repeats
    the recorded run: the same seed and iteration numbers from a uniform
    grid, so the same samples.  Per-iteration host work (acc, callback) has
    no place in a graph and is not offered; the grid's other users must
    leave it alone between the recording and the last replay."""

    def __init__(self, integrand, dim, nbins, theta, ncall, itmx, seed, alpha=1.5, ng=1, itmx2=0, fp64=False,
                 grid: Grid | None = None, it0=0):
        self.grid = g = grid if grid is not None else Grid(dim, nbins)
        assert (g.dim, g.nbins) == (dim, nbins)
        self._th = g.theta_tensor(theta)  # device copy made before the recording
        self._hist = torch.zeros((itmx + itmx2, 2), dtype=torch.float64, device=g.device)
        self._args = (integrand, ncall, itmx, seed, alpha, ng, itmx2, fp64, it0)
        # an eager run on a side stream sets up the library's per-device state
        # (occupancy cache, cleared partial sums) before the recording
        side = torch.cuda.Stream(device=g.device)
        side.wait_stream(torch.cuda.current_stream(g.device))
        with torch.cuda.stream(side):
            self._issue()
        torch.cuda.current_stream(g.device).wait_stream(side)
        torch.cuda.synchronize(g.device)
        self._graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self._graph):
            self._issue()

    def _issue(self):
        """The launches of one run, on torch's current stream."""
        integrand, ncall, itmx, seed, alpha, ng, itmx2, fp64, it0 = self._args
        g = self.grid
        g.reset()
        g.stratify(ng)
        k, it = 0, it0
        for p, (nit, adapt) in enumerate([(itmx, True)] + ([(itmx2, False)] if itmx2 else [])):
            if p > 0:
                g.combine_reset()
            for _ in range(nit):
                g.iterate(integrand, self._th, ncall, seed, it, fp64=fp64)
                self._hist[k].copy_(g.scal[L.S_I:L.S_VAR + 1])
                k += 1
                it += 1
                if adapt:
                    g.refine(alpha)

    def replay(self):
        """Enqueue one run on the current stream (no host synchronisation)."""
        self._graph.replay()

    def run(self) -> Result:
        self.replay()
        r = self.grid.result()
        h = self._hist.cpu().numpy()
        return Result(I=h[:, 0], var=h[:, 1], Ibar=r["Ibar"], sigbar=r["sigbar"], chi2dof=r["chi2dof"],
                      n_eff=int(r["n_eff"]) * h.shape[0], niter=r["niter"], grid=self.grid)

