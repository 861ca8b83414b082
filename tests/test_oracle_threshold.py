"""Pins of the heat-bath threshold against Algorithm 3's acceptance
probability p = e^h / (2 cosh h), evaluated here straight from that formula."""
import math

import numpy as np

TWO32 = 2.0 ** 32


def _paper_p(h):
    return math.exp(h) / (2.0 * math.cosh(h))


def test_threshold_within_half_ulp_of_paper_probability(oracle):
    hs = list(np.linspace(-10.0, 10.0, 4001)) + [1e-12, -1e-12, 0.4406867, -0.6585]
    for h in hs:
        T = oracle.threshold(h)
        assert abs(T / TWO32 - _paper_p(h)) <= 2.0 ** -33 + 1e-15, h


def test_threshold_symmetry_and_centre(oracle):
    assert oracle.threshold(0.0) == 2 ** 31
    assert oracle.threshold(-0.0) == 2 ** 31
    for h in np.linspace(1e-6, 12.0, 997):
        assert oracle.threshold(h) + oracle.threshold(-h) == 2 ** 32


def test_threshold_monotone_and_clamped(oracle):
    hs = np.linspace(-30.0, 30.0, 6001)
    T = np.array([oracle.threshold(h) for h in hs], dtype=np.int64)
    assert np.all(np.diff(T) >= 0)
    assert T[0] >= 1 and T[-1] <= 2 ** 32 - 1


def test_table_matches_class_fields(oracle):
    # class idx = 2k + [c = +1]; field h = J (n1 + n2) + q c with k of n1, n2 equal to +1
    for J, q in [(0.4, 0.6), (0.0, 0.0), (1.5, 2.0), (0.7, 0.0), (0.0, 0.3), (-0.3, 0.8)]:
        table = oracle.threshold_table(J, q)
        for k in range(3):
            for cplus in range(2):
                h = J * (2 * k - 2) + q * (2 * cplus - 1)
                assert abs(int(table[2 * k + cplus]) / TWO32 - _paper_p(h)) <= 2.0 ** -33 + 1e-15


def test_table_spot_values(oracle):
    # values quoted in the design notes for (J, q) = (0.4, 0.6)
    assert list(oracle.threshold_table(0.4, 0.6)) == [
        246205461, 1723623375, 994178485, 3300788811, 2571343921, 4048761835]
