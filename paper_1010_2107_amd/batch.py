"""Python handle over a batch of integrals advanced by one persistent launch
per iteration (vmc_batch_* in include/vmc.h).  Torch supplies the device
buffers and the stream; the work runs in the library's kernels."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from .grid import _ptr, _stream_ptr


class Batch:
    """n per-axis Gaussian integrals (VMC_GAUSS_AXES), each with its own
    grid of `nbins` bins per axis, parameters, accumulators and call count."""

    def __init__(self, dims, ncalls, thetas, nbins=64, device="cuda"):
        self.dims = np.asarray(dims, dtype=np.int32)
        self.ncalls = np.asarray(ncalls, dtype=np.int64)
        self.n = len(self.dims)
        self.nbins = int(nbins)
        self.device = torch.device(device)
        assert len(thetas) == self.n
        h = ctypes.c_void_p()
        d = (ctypes.c_int * self.n)(*self.dims.tolist())
        nc = (ctypes.c_int64 * self.n)(*self.ncalls.tolist())
        L.call("vmc_batch_create", self.n, d, self.nbins, L.GAUSS_AXES, nc, ctypes.byref(h))
        self._h = h
        self._destroy = L.lib().vmc_batch_destroy  # outlives the module globals at exit
        # size the work-list buffer for the finest schedule (one tile per 256 samples)
        L.call("vmc_batch_set_schedule", h, 1, 0)
        self._sizes = self._query()
        meta_max = self._sizes[5]
        L.call("vmc_batch_set_schedule", h, 0, 0)
        sz = self._query()
        kw = dict(device=self.device)
        self.edges = torch.zeros(sz[0] // 8, dtype=torch.float64, **kw)
        self.table = torch.zeros(sz[1] // 4, dtype=torch.float32, **kw)
        self.bins = torch.zeros(sz[2] // 8, dtype=torch.float64, **kw)
        self.scal = torch.zeros((self.n, L.SCAL_LEN), dtype=torch.float64, **kw)
        th = np.concatenate([np.asarray(t, dtype=np.float64) for t in thetas])
        assert th.size * 8 == sz[4], (th.size, sz[4])
        self.theta = torch.tensor(th, dtype=torch.float64, **kw)
        self.meta = torch.zeros(meta_max, dtype=torch.uint8, **kw)
        L.call("vmc_batch_bind", h, _ptr(self.edges), _ptr(self.table), _ptr(self.bins), _ptr(self.scal),
               _ptr(self.theta), _ptr(self.meta), meta_max)
        self.off_bins = np.concatenate([[0], np.cumsum(2 * self.dims * self.nbins)])
        self.off_edges = np.concatenate([[0], np.cumsum(self.dims * (self.nbins + 1))])
        self.reset()

    def _query(self):
        sz = (ctypes.c_size_t * 6)()
        L.call("vmc_batch_workspace_sizes", self._h, sz)
        return list(sz)

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and destroy is not None:
            destroy(h)
            self._h = None

    def set_schedule(self, samples_per_thread=0, blocks=0):
        L.call("vmc_batch_set_schedule", self._h, int(samples_per_thread), int(blocks))

    def reset(self, stream=None):
        L.call("vmc_batch_reset", self._h, _stream_ptr(stream))

    def iterate(self, seed, it, kind=1, fp64=False, stream=None):
        """kind 1 forward, 2 adjoint, 3 forward and adjoint in one pass."""
        L.call("vmc_iterate_batched", self._h, int(seed), int(it), int(kind), L.FLAG_FP64 if fp64 else 0,
               _stream_ptr(stream))

    def refine(self, alpha=1.5, stream=None):
        L.call("vmc_refine_batched", self._h, float(alpha), _stream_ptr(stream))

    def set_edges(self, k, edges, stream=None):
        """Grid of integral k from host memory ([d_k][nbins + 1] doubles)."""
        e = np.ascontiguousarray(edges, dtype=np.float64)
        assert e.shape == (int(self.dims[k]), self.nbins + 1), e.shape
        L.call("vmc_batch_set_edges", self._h, int(k), e.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream))

    def combine_reset(self, stream=None):
        L.call("vmc_batch_combine_reset", self._h, _stream_ptr(stream))

    def run(self, seed, itmx, itmx2=0, alpha=1.5, kind=1, freeze=True):
        """itmx warm-up iterations that refine the grids, then itmx2 more,
        combining only the latter; freeze=True keeps the grids fixed in the
        second phase (BASES), freeze=False keeps refining (VEGAS with the
        warm-up iterations left out of the combination)."""
        it = 0
        for _ in range(itmx):
            self.iterate(seed, it, kind)
            self.refine(alpha)
            it += 1
        if itmx2:
            self.combine_reset()
            for _ in range(itmx2):
                self.iterate(seed, it, kind)
                if not freeze:
                    self.refine(alpha)
                it += 1
        return self.results()

    def timing(self, enable):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        L.call("vmc_batch_timing", self._h, int(bool(enable)), ctypes.byref(ms), ctypes.byref(n))
        return ms.value, n.value

    # ------------------------------------------------------------- results
    def results(self):
        s = self.scal.cpu().numpy()
        return dict(S1=s[:, L.S_S1], S2=s[:, L.S_S2], I=s[:, L.S_I], var=s[:, L.S_VAR], n_eff=s[:, L.S_NEFF],
                    Ibar=s[:, L.S_IBAR], sigbar=s[:, L.S_SIGBAR], chi2dof=s[:, L.S_CHI2],
                    nonfinite=s[:, L.S_NONFINITE])

    def grads(self):
        s = self.scal.cpu().numpy()
        out = []
        for k in range(self.n):
            g = s[k, L.S_GRAD:L.S_GRAD + 5 * (self.dims[k] + 1)].reshape(-1, 5)
            out.append(dict(gsum=g[:, 0], gsumsq=g[:, 1], grad=g[:, 3], grad_var=g[:, 4]))
        return out

    def bins_of(self, k):
        b = self.bins[self.off_bins[k]:self.off_bins[k + 1]].cpu().numpy()
        return b.reshape(2, self.dims[k], self.nbins)

    def edges_of(self, k):
        e = self.edges[self.off_edges[k]:self.off_edges[k + 1]].cpu().numpy()
        return e.reshape(self.dims[k], self.nbins + 1)
