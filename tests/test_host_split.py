"""The paper's split of the work (Sec. 3.2), host side: the bench's host
accumulation and host refinement against the oracle (CPU only).  The
refinement is checked on random grids and per-bin sums, on an all-zero
axis, and on the hand-worked cases written out from the definition."""
import numpy as np
import pytest

import bench
import oracle as O
from tests.test_oracle_refine_combine import HAND_CASES


@pytest.mark.parametrize("d,N,alpha", [(3, 50, 1.5), (2, 2, 1.5), (4, 128, 0.7), (1, 256, 2.0)])
def test_host_refine_matches_oracle(d, N, alpha):
    rng = np.random.default_rng(d * N)
    w = rng.gamma(1.0, size=(d, N)) + 0.01
    e = np.concatenate([np.zeros((d, 1)), np.cumsum(w, axis=1)], axis=1)
    e /= e[:, -1:]
    e[:, -1] = 1.0
    b2 = rng.gamma(0.4, size=(d, N))
    b2[0, : N // 3] = 0.0
    if d > 1:
        b2[1] = 0.0  # all-zero axis stays
    got = bench.host_refine(e, b2, alpha)
    assert np.max(np.abs(got - O.refine(e, b2, alpha))) <= 1e-14
    if d > 1:
        assert np.array_equal(got[1], e[1])


@pytest.mark.parametrize("name", sorted(HAND_CASES))
def test_host_refine_hand_worked(name):
    edges, b2, alpha, want, _ = HAND_CASES[name]()
    got = bench.host_refine(edges[None, :], b2[None, :], alpha)[0]
    assert np.max(np.abs(got - want)) <= 1e-14


def test_host_accumulate_matches_oracle_replay():
    """Sums of given FP32 weights and bin indices equal the oracle's
    accumulation of the same weights on the same samples."""
    d, N, ncall = 3, 20, 5001
    e = O.uniform_edges(d, N)
    smp = O.eval_samples(O.GAUSS, e, (0.4, 0.2), ncall, 5, 1, 0, ncall)
    w32 = smp["w"].astype(np.float32)
    S1, S2, bins = bench.host_accumulate(w32, smp["j"].astype(np.uint8), N)
    ref = O.iterate(O.GAUSS, e, (0.4, 0.2), ncall, 5, 1, w_in=w32)
    assert abs(S1 - ref["S1"]) <= 1e-13 * abs(ref["S1"])
    assert abs(S2 - ref["S2"]) <= 1e-13 * ref["S2"]
    assert np.max(np.abs(bins - ref["bins"])) <= 1e-13 * np.max(np.abs(ref["bins"]))
