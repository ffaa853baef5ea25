"""The parameter helpers of workloads.py (no arithmetic of the method)."""
from paper_1010_2107_amd import workloads as W


def test_default_ng_follows_the_bases_rule():
    # largest divisor of nbins not above (ncall/2)^(1/d)
    assert W.default_ng(5_000_000, 8, 128) == W.C2.ng == 4
    assert W.default_ng(1_000_000, 5, 64) == 8     # (5e5)^(1/5) = 13.8
    assert W.default_ng(1_000_000, 11, 64) == 2    # (5e5)^(1/11) = 3.3
    assert W.default_ng(1_000_000, 8, 50) == 5     # 5.1: divisors of 50 up to 5
    assert W.default_ng(10, 16, 64) == 2           # never below 2
    for ng, d, n in ((4, 8, 128), (8, 5, 64), (2, 11, 64)):
        assert n % ng == 0 and ng ** d <= 5_000_000


def test_configs_are_consistent():
    for w in W.CONFIGS.values():
        assert w.ncall >= 2 and w.nbins >= 2 and w.itmx >= 1
        if w.integrand == W.WJETS:
            assert (w.dim - 4) % 3 == 0 and len(w.theta) == 7
        if w.integrand == W.WHEL:
            assert w.dim in (5, 8, 11) and len(w.theta) == 8
