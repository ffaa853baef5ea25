"""The calibration kernels behind the bench line's rates (vmc_probe_fp32_fma,
vmc_probe_lds_atomics): they run through the C ABI on the current stream,
reject bad arguments, and report rates inside the chip's envelope.

Bounds: the FP32 FMA rate lies below MI355X's 157.3 TFLOP/s packed-FMA peak
(the probe issues non-packed FMAs, half of that at the same clock) and above
a tenth of it; the LDS FP64 add rate lies below 256 CUs x 64 lanes per clock
x 2.5 GHz and above 1e11 per second.
"""
import ctypes

import pytest
import torch

from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_fma_probe_rate_in_envelope():
    require_gpu()
    from paper_1010_2107_amd import _lib as L
    announce("fp32 fma probe")
    rate = ctypes.c_double()
    L.call("vmc_probe_fp32_fma", 2048, 1024, ctypes.byref(rate), _stream())
    tflops = rate.value / 1e12
    assert 15.7 < tflops < 157.3, tflops


def test_lds_probe_rate_in_envelope():
    require_gpu()
    from paper_1010_2107_amd import _lib as L
    announce("lds atomic probe")
    rate = ctypes.c_double()
    L.call("vmc_probe_lds_atomics", 512, 1024, ctypes.byref(rate), _stream())
    assert 1e11 < rate.value < 256 * 64 * 2.5e9, rate.value


def test_probes_reject_bad_arguments():
    require_gpu()
    from paper_1010_2107_amd import _lib as L
    rate = ctypes.c_double()
    for name in ("vmc_probe_fp32_fma", "vmc_probe_lds_atomics"):
        with pytest.raises(L.VmcError):
            L.call(name, 0, 16, ctypes.byref(rate), _stream())
        with pytest.raises(L.VmcError):
            L.call(name, 16, 1 << 21, ctypes.byref(rate), _stream())
        with pytest.raises(L.VmcError):
            L.call(name, 16, 16, None, _stream())
