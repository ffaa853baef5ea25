"""Pins for the oracle's Philox4x32-10 and its counter layout.

External pin: rocRAND's Philox4x32-10 engine (a library implementation written
from the same SC'11 definition), compiled host-side from the ROCm headers.
Statistical pins: uniformity and serial correlation of the words.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
ROCM_INC = "/opt/rocm/include"


@pytest.fixture(scope="module")
def rocrand_philox():
    src = os.path.join(HERE, "pins", "philox_rocrand.cpp")
    if shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM_INC, "rocrand")):
        pytest.skip("g++ or rocRAND headers not available: Philox library pin unavailable")
    tmp = tempfile.mkdtemp(prefix="philox_pin_")
    exe = os.path.join(tmp, "philox_rocrand")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, src,
                           "-o", exe])

    def run(rows):
        inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint64).astype(np.uint32)

    yield run
    shutil.rmtree(tmp, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(7)
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [1, 2, 3, 4, 5, 6]]
    rows += rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64).tolist()
    ref = rocrand_philox(rows)
    mine = np.array([O.philox(r[:4], r[4:]) for r in rows], dtype=np.uint32)
    assert np.array_equal(mine, ref)


def test_sample_word_layout(rocrand_philox):
    # word a of sample s = word a%4 of the block with counter (s, a//4, it, kid),
    # key = (seed low 32 bits, seed high 32 bits)
    seed, it, kid, d = 0x0123456789ABCDEF, 7, 3, 10
    rows, expect_idx = [], []
    for s in (0, 1, 2**31 + 5, 2**32 - 1):
        for g in range(3):
            rows.append([s, g, it, kid, seed & 0xFFFFFFFF, seed >> 32])
    ref = rocrand_philox(rows).reshape(4, 3, 4)
    for si, s in enumerate((0, 1, 2**31 + 5, 2**32 - 1)):
        w = O.sample_words(seed, s, it, kid, d)
        assert np.array_equal(w, ref[si].ravel()[:d])


def _words(n, d=4, seed=1234, it=0):
    e = O.uniform_edges(d, 2)
    out = O.eval_samples(O.CONST, e, [1.0], n, seed, it, 0, n)
    return out["words"]


def test_uniformity_chi2():
    w = _words(1 << 16).ravel()  # 262144 words
    counts = np.bincount(w >> 24, minlength=256)
    exp = w.size / 256
    chi2 = ((counts - exp) ** 2 / exp).sum()
    # 255 dof: mean 255, sd ~22.6; 6 sd bounds
    assert 120 < chi2 < 390


def test_serial_correlation_and_word_independence():
    w = _words(1 << 15, d=8).astype(np.float64) / 2**32
    u = w.ravel()
    r1 = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r1) < 6 / np.sqrt(u.size)
    # different words of one sample, and the same word of neighbouring samples
    for a, b in ((0, 1), (0, 4), (3, 7)):
        r = np.corrcoef(w[:, a], w[:, b])[0, 1]
        assert abs(r) < 6 / np.sqrt(w.shape[0])
    r = np.corrcoef(w[:-1, 0], w[1:, 0])[0, 1]
    assert abs(r) < 6 / np.sqrt(w.shape[0])


def test_streams_differ_by_iteration_and_integral():
    a = O.sample_words(1234, 5, 0, 0, 8)
    b = O.sample_words(1234, 5, 1, 0, 8)
    c = O.sample_words(1234, 5, 0, 1, 8)
    dd = O.sample_words(1235, 5, 0, 0, 8)
    assert len({tuple(a), tuple(b), tuple(c), tuple(dd)}) == 4
