"""SPRING event generation on the GPU: unweighted events from the per-cube
maxima of the BASES integration phase (paper Sec. 3.1).  Argument
marshalling over the spring_* entry points of include/vmc.h; the buffers
are torch device tensors owned here.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from .grid import Grid, _ptr, _stream_ptr


class Spring:
    """Envelope and trial state for one stratified grid (its grid and
    stratification must stay as they were at setup)."""

    def __init__(self, grid: Grid):
        self.grid = grid
        sizes = (ctypes.c_size_t * 3)()
        L.call("spring_workspace_sizes", grid.handle, sizes)
        kw = dict(device=grid.device)
        self.prefix = torch.zeros(sizes[0] // 8, dtype=torch.int64, **kw)  # uint64 bit patterns
        self.guide = torch.zeros(sizes[1] // 4, dtype=torch.int32, **kw)   # uint32 bit patterns
        self.state = torch.zeros(sizes[2] // 8, dtype=torch.int64, **kw)
        self.ncubes = self.prefix.numel() - 1

    def setup(self, cube_max: torch.Tensor, headroom: float = 1.0, stream=None):
        """Envelope g_c = headroom x the quantised cube maxima (headroom >= 1)."""
        assert cube_max.dtype == torch.float64 and cube_max.numel() >= self.ncubes
        L.call("spring_setup", self.grid.handle, _ptr(cube_max), float(headroom), _ptr(self.prefix),
               _ptr(self.guide), _ptr(self.state), _stream_ptr(stream))

    def clear_counts(self, stream=None):
        L.call("spring_clear_counts", _ptr(self.state), _stream_ptr(stream))

    def header(self) -> dict:
        """Envelope and counters (synchronises)."""
        h = self.state[:16].cpu().numpy()
        d = h.view(np.float64)
        u = h.view(np.uint64)
        return dict(unit=float(d[L.SP_UNIT]), gmax=float(d[L.SP_GMAX]), total=int(u[L.SP_TOTAL]),
                    env=float(d[L.SP_ENV]), kbits=int(u[L.SP_KBITS]), ncubes=int(u[L.SP_NCUBES]),
                    trials=int(u[L.SP_TRIALS]), kept=int(u[L.SP_KEPT]), over=int(u[L.SP_OVER]),
                    slot=int(u[L.SP_SLOT]))

    def quanta(self) -> np.ndarray:
        """Envelope q_c in quanta (differences of the running sums)."""
        p = self.prefix.cpu().numpy().view(np.uint64)
        return np.diff(p)

    def generate(self, integrand, theta, seed, pass_, trial0, ntrials, events: torch.Tensor,
                 event_trial: torch.Tensor | None = None, fp64=False, stream=None):
        """Append the kept trials of [trial0, trial0+ntrials) to events
        ([max_events][dim], float32 or float64) and event_trial (int64)."""
        g = self.grid
        th = g.theta_tensor(theta)
        assert events.dtype == (torch.float64 if fp64 else torch.float32)
        assert events.dim() == 2 and events.shape[1] == g.dim and events.is_contiguous()
        if event_trial is not None:
            assert event_trial.dtype == torch.int64 and event_trial.numel() >= events.shape[0]
        L.call("spring_generate", g.handle, int(integrand), _ptr(th if th.numel() else None), th.numel(),
               _ptr(self.prefix), _ptr(self.guide), _ptr(self.state), int(seed), int(pass_), int(trial0),
               int(ntrials), events.shape[0], _ptr(events), _ptr(event_trial), L.FLAG_FP64 if fp64 else 0,
               _stream_ptr(stream))
        return th
