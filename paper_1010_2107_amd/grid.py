"""Python handle over one grid of libvmc.so.

PyTorch provides the device buffers (caller-owned, bound to the handle) and
the stream; every step of an iteration runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Grid:
    """A (dim, nbins) VEGAS grid with its FP64 edges, FP32 table, bin sums
    and scalar block in device memory (paper Sec. 2: per-axis bins)."""

    def __init__(self, dim: int, nbins: int, device="cuda"):
        self.dim, self.nbins = int(dim), int(nbins)
        self.device = torch.device(device)
        sizes = (ctypes.c_size_t * 4)()
        L.call("vmc_workspace_sizes", self.dim, self.nbins, sizes)
        h = ctypes.c_void_p()
        L.call("vmc_create", self.dim, self.nbins, ctypes.byref(h))
        self._h = h
        # held by the instance: at interpreter exit the module globals may
        # already be gone when __del__ runs
        self._destroy = L.lib().vmc_destroy
        kw = dict(device=self.device)
        self.edges = torch.zeros((self.dim, self.nbins + 1), dtype=torch.float64, **kw)
        self.table = torch.zeros((self.dim, self.nbins, 2), dtype=torch.float32, **kw)
        # the bin sums [2][dim][nbins] head a buffer whose tail is library-private
        self._bins_buf = torch.zeros(sizes[2] // 8, dtype=torch.float64, **kw)
        nb = 2 * self.dim * self.nbins
        self.bins = self._bins_buf[:nb].view(2, self.dim, self.nbins)
        self.scal = torch.zeros(L.SCAL_LEN, dtype=torch.float64, **kw)
        assert self.edges.numel() * 8 == sizes[0] and self.table.numel() * 4 == sizes[1]
        assert self.scal.numel() * 8 == sizes[3]
        L.call("vmc_bind", h, _ptr(self.edges), _ptr(self.table), _ptr(self._bins_buf), _ptr(self.scal))
        self.ng = 1
        self.reset()

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and destroy is not None:
            destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    # ------------------------------------------------------------------ setup
    def reset(self, stream=None):
        L.call("vmc_reset", self._h, _stream_ptr(stream))

    def stratify(self, ng: int):
        ng = int(ng)
        if not 0 <= ng < 2**31:  # the C call takes an int
            raise ValueError(f"ng = {ng} outside [0, 2^31)")
        L.call("bases_stratify", self._h, ng)
        self.ng = max(int(ng), 1)

    def bind_cube_max(self, buf: torch.Tensor | None):
        """Record each cube's largest weight of every stratified forward pass
        into buf (float64, ng^dim entries, caller zeroes it); None unbinds."""
        if buf is None:
            L.call("bases_cube_max", self._h, None, 0)
            self._cube_max = None
            return
        assert buf.dtype == torch.float64 and buf.is_contiguous() and buf.device.type == "cuda"
        L.call("bases_cube_max", self._h, _ptr(buf), buf.numel())
        self._cube_max = buf  # keep the memory alive while bound

    def set_schedule(self, block_samples: int = 0, chunks_per_cube: int = 0):
        L.call("vmc_set_schedule", self._h, int(block_samples), int(chunks_per_cube))

    def theta_tensor(self, theta) -> torch.Tensor:
        if isinstance(theta, torch.Tensor):
            return theta.detach().to(device=self.device, dtype=torch.float64).contiguous()
        return torch.tensor(np.asarray(theta, dtype=np.float64).reshape(-1), dtype=torch.float64, device=self.device)

    # -------------------------------------------------------------- iteration
    def _run(self, name, integrand, theta, ncall, seed, it, fp64, stream):
        th = self.theta_tensor(theta)
        L.call(name, self._h, int(integrand), _ptr(th if th.numel() else None), th.numel(), int(ncall),
               int(seed), int(it), L.FLAG_FP64 if fp64 else 0, _stream_ptr(stream))
        return th

    def iterate(self, integrand, theta, ncall, seed, it, fp64=False, stream=None):
        """Steps 2-4 of one iteration plus its estimate (stream-ordered)."""
        return self._run("vmc_iterate", integrand, theta, ncall, seed, it, fp64, stream)

    def iterate_static(self, integrand, theta, ncall, seed, it, fp64=False, stream=None):
        """As iterate, with the blocks' partial sums in the library's static
        device array (vmc_iterate_static: no allocation, no workspace)."""
        return self._run("vmc_iterate_static", integrand, theta, ncall, seed, it, fp64, stream)

    def adjoint(self, integrand, theta, ncall, seed, it, fp64=False, stream=None):
        return self._run("vmc_iterate_adjoint", integrand, theta, ncall, seed, it, fp64, stream)

    def fused(self, integrand, theta, ncall, seed, it, fp64=False, stream=None):
        return self._run("vmc_iterate_fused", integrand, theta, ncall, seed, it, fp64, stream)

    def refine(self, alpha=1.5, stream=None):
        L.call("vmc_refine", self._h, float(alpha), _stream_ptr(stream))

    def combine_reset(self, stream=None):
        L.call("vmc_combine_reset", self._h, _stream_ptr(stream))

    def timing(self, enable: bool):
        """Return (summed ms, launches) of the sample kernels recorded since the
        last call, then switch recording on or off."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        L.call("vmc_timing", self._h, int(bool(enable)), ctypes.byref(ms), ctypes.byref(n))
        return ms.value, n.value

    # ---------------------------------------------------------------- results
    def result(self) -> dict:
        """Scalar block as a dict (synchronises)."""
        s = self.scal.cpu().numpy()
        return dict(S1=s[L.S_S1], S2=s[L.S_S2], V=s[L.S_V], nonfinite=int(s[L.S_NONFINITE]), I=s[L.S_I],
                    var=s[L.S_VAR], n_eff=int(s[L.S_NEFF]), n_zero=int(s[L.S_NZERO]), niter=int(s[L.S_NITER]), Ibar=s[L.S_IBAR],
                    sigbar=s[L.S_SIGBAR], chi2dof=s[L.S_CHI2])

    def version(self) -> int:
        """Grid-state version: advanced by bind, reset, stratify, refine and
        set_edges (an adjoint pass needs the version of its forward pass)."""
        v = ctypes.c_uint64()
        L.call("vmc_grid_version", self._h, ctypes.byref(v))
        return v.value

    def grad_result(self, ngrad: int) -> dict:
        g = self.scal[L.S_GRAD:L.S_GRAD + 5 * ngrad].cpu().numpy().reshape(ngrad, 5)
        return dict(gsum=g[:, 0], gsumsq=g[:, 1], gV=g[:, 2], grad=g[:, 3], grad_var=g[:, 4])

    def get_edges(self, stream=None) -> np.ndarray:
        out = np.zeros((self.dim, self.nbins + 1))
        L.call("vmc_get_edges", self._h, out.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream))
        return out

    def set_edges(self, edges, stream=None):
        e = np.ascontiguousarray(edges, dtype=np.float64)
        assert e.shape == (self.dim, self.nbins + 1)
        L.call("vmc_set_edges", self._h, e.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream))

    def dump_into(self, integrand, theta, ncall, seed, it, s0, words=None, w=None, f=None, jac=None, bins=None,
                  grad=None, stream=None):
        """Per-sample dump into caller tensors (device; any may be None):
        words [count][dim] int32, bins [count][dim] uint8, w / f / jac
        [count] and grad [count][ngrad], float32 or float64 (float64 selects
        the FP64 instantiation)."""
        outs = [t for t in (words, bins, w, f, jac, grad) if t is not None]
        count = outs[0].shape[0] if outs else 0
        assert all(t.shape[0] == count and t.is_contiguous() for t in outs)
        fl = [t for t in (w, f, jac, grad) if t is not None]
        fp64 = any(t.dtype == torch.float64 for t in fl)
        assert all(t.dtype == (torch.float64 if fp64 else torch.float32) for t in fl)
        assert words is None or (words.dtype == torch.int32 and tuple(words.shape) == (count, self.dim))
        assert bins is None or (bins.dtype == torch.uint8 and tuple(bins.shape) == (count, self.dim))
        if grad is not None:
            ngrad = L.integrand_info(integrand, self.dim, fp64)[1]
            assert tuple(grad.shape) == (count, ngrad), (tuple(grad.shape), ngrad)
        th = self.theta_tensor(theta)
        L.call("vmc_dump_samples", self._h, int(integrand), _ptr(th if th.numel() else None), th.numel(),
               int(ncall), int(seed), int(it), L.FLAG_FP64 if fp64 else 0, int(s0), int(count), _ptr(words),
               _ptr(bins), _ptr(w), _ptr(f), _ptr(jac), _ptr(grad), _stream_ptr(stream))

    def dump(self, integrand, theta, ncall, seed, it, s0, count, fp64=False, want_grad=False, stream=None):
        """Per-sample words, bin indices, w = f J, f, J (and df/dtheta with
        want_grad) of samples [s0, s0+count)."""
        dt = torch.float64 if fp64 else torch.float32
        kw = dict(device=self.device)
        out = dict(words=torch.zeros((count, self.dim), dtype=torch.int32, **kw),
                   bins=torch.zeros((count, self.dim), dtype=torch.uint8, **kw),
                   w=torch.zeros(count, dtype=dt, **kw), f=torch.zeros(count, dtype=dt, **kw),
                   jac=torch.zeros(count, dtype=dt, **kw))
        if want_grad:
            out["grad"] = torch.zeros((count, L.integrand_info(integrand, self.dim, fp64)[1]), dtype=dt, **kw)
        self.dump_into(integrand, theta, ncall, seed, it, s0, stream=stream, **out)
        res = {k: v.cpu().numpy() for k, v in out.items()}
        res["words"] = res["words"].view(np.uint32)
        return res
