"""vmc_iterate_static, the entry point that allocates nothing (its partial
sums live in the library's static device array), against vmc_iterate on the
same inputs, through the C ABI: two calls in a row, the second on a smaller
grid and call count, FP64 instantiation (sums to summation order, 1e-12)
and FP32 (the same per-sample weights, so the same bound), plain and
stratified.  The handle used with the static entry point is bound to a bins
buffer of just the 2 dim nbins published sums followed by sentinel values
that must stay untouched."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1010_2107_amd import _lib as L
from paper_1010_2107_amd import workloads as W
from paper_1010_2107_amd.grid import Grid
from tests.gpu_util import announce, normwise, rel, require_gpu

pytestmark = pytest.mark.gpu

SENTINEL = 12345.0


class ShortHandle:
    """A grid handle over caller buffers with only the published bin sums
    (plus a sentinel tail) in the bins buffer."""

    def __init__(self, d, N):
        self.d, self.N = d, N
        h = ctypes.c_void_p()
        L.call("vmc_create", d, N, ctypes.byref(h))
        self.h = h
        kw = dict(device="cuda")
        self.edges = torch.zeros((d, N + 1), dtype=torch.float64, **kw)
        self.table = torch.zeros((d, N, 2), dtype=torch.float32, **kw)
        self.bins_buf = torch.full((2 * d * N + 256,), SENTINEL, dtype=torch.float64, **kw)
        self.scal = torch.zeros(L.SCAL_LEN, dtype=torch.float64, **kw)
        L.call("vmc_bind", h, *(ctypes.c_void_p(t.data_ptr()) for t in (self.edges, self.table, self.bins_buf,
                                                                         self.scal)))
        L.call("vmc_reset", h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))

    def stratify(self, ng):
        L.call("bases_stratify", self.h, int(ng))

    def iterate_static(self, integrand, theta, ncall, seed, it, fp64):
        th = torch.tensor(theta, dtype=torch.float64, device="cuda")
        L.call("vmc_iterate_static", self.h, int(integrand), ctypes.c_void_p(th.data_ptr()), th.numel(), int(ncall),
               int(seed), int(it), L.FLAG_FP64 if fp64 else 0,
               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))

    def refine(self, alpha):
        L.call("vmc_refine", self.h, float(alpha), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))

    def bins(self):
        return self.bins_buf[: 2 * self.d * self.N].view(2, self.d, self.N).cpu().numpy()

    def tail_untouched(self):
        return bool(torch.all(self.bins_buf[2 * self.d * self.N:] == SENTINEL).item())

    def close(self):
        L.call("vmc_destroy", self.h)


CALLS = [  # (integrand, d, N, theta, ncall, ng): the second is smaller
    (W.DGAUSS, 8, 128, (1 / 3, 2 / 3, 0.1), 4**8 * 6 + 11, 4),
    (W.GAUSS, 4, 50, (0.5, 0.1), 20_003, 1),
]


@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_static_entry_point_matches_iterate(fp64):
    require_gpu()
    for k, (iid, d, N, theta, ncall, ng) in enumerate(CALLS):
        announce(f"static entry point call {k}: integrand {iid} d={d} N={N} ncall={ncall} ng={ng} fp64={fp64}")
        sh = ShortHandle(d, N)
        sh.stratify(ng)
        ref = Grid(d, N)
        ref.stratify(ng)
        for it in range(2):  # an iteration, a refinement, another iteration
            sh.iterate_static(iid, theta, ncall, 77, it, fp64)
            ref.iterate(iid, theta, ncall, 77, it, fp64=fp64)
            got = sh.scal.cpu().numpy()
            want = ref.scal.cpu().numpy()
            for slot in (L.S_S1, L.S_S2, L.S_I, L.S_V, L.S_IBAR):
                assert rel(got[slot], want[slot]) <= 1e-12, (k, it, slot, got[slot], want[slot])
            for slot in (L.S_VAR, L.S_SIGBAR):
                assert rel(got[slot], want[slot]) <= 1e-10, (k, it, slot)
            assert got[L.S_NEFF] == want[L.S_NEFF] and got[L.S_NITER] == want[L.S_NITER]
            assert got[L.S_NZERO] == want[L.S_NZERO] and got[L.S_NONFINITE] == want[L.S_NONFINITE] == 0
            assert normwise(sh.bins(), ref.bins.cpu().numpy()) <= 1e-12, (k, it)
            assert sh.tail_untouched(), (k, it)
            sh.refine(1.5)
            ref.refine(1.5)
            assert np.max(np.abs(sh.edges.cpu().numpy() - ref.edges.cpu().numpy())) <= 1e-12
        sh.close()
