"""Pins of the oracle's candidate selection (row statistics, threshold, peak rule).

Closed forms for the statistics of a spike and a two-level row, the plateau and
end rules on hand-made rows, and brute force against ``statistics.pstdev``
(exact rational arithmetic) on small random planes.
"""

import math
import statistics

import numpy as np
import pytest

from oracle.candidates import find_candidates, is_peak, row_statistics


@pytest.mark.parametrize("n,j,a", [(8, 3, 5.0), (1000, 0, 2.5), (4097, 4096, 1e3)])
def test_single_spike_closed_form(n, j, a):
    """N - 1 zeros and one value A: mu = A/N, sigma = A sqrt(N-1)/N, significance sqrt(N-1)."""
    row = np.zeros((1, n), dtype=np.float32)
    row[0, j] = a
    st = row_statistics(row)
    assert abs(st[0, 0] - a / n) <= 1e-15 * a
    assert abs(st[0, 1] - a * math.sqrt(n - 1) / n) <= 1e-13 * a
    c = find_candidates(row, math.sqrt(n - 1) * (1 - 1e-9))
    assert len(c) == 1 and c[0]["p"] == j and c[0]["t"] == 0
    assert abs(c[0]["sigma"] - math.sqrt(n - 1)) < 1e-9 * math.sqrt(n)
    assert len(find_candidates(row, math.sqrt(n - 1) * (1 + 1e-9))) == 0


def test_two_level_row_statistics():
    row = np.array([[0.0, 1.0] * 50], dtype=np.float32)
    st = row_statistics(row)
    assert st[0, 0] == 0.5 and st[0, 1] == 0.5


def test_peak_rule_plateaus_and_ends():
    assert list(np.nonzero(is_peak(np.array([0, 5, 5, 0])))[0]) == [1]
    assert list(np.nonzero(is_peak(np.array([5, 0, 0, 0])))[0]) == [0]
    # a flat start is a plateau whose leftmost point is the row's first
    assert list(np.nonzero(is_peak(np.array([0, 0, 0, 5])))[0]) == [0, 3]
    assert list(np.nonzero(is_peak(np.array([3, 3, 3])))[0]) == [0]
    assert list(np.nonzero(is_peak(np.array([1, 2, 1, 2, 2, 1, 0, 4])))[0]) == [1, 3, 7]
    assert list(np.nonzero(is_peak(np.array([7])))[0]) == [0]


def test_constant_row_has_no_candidates():
    row = np.full((2, 64), 3.25, dtype=np.float32)
    assert len(find_candidates(row, 0.0)) == 0
    assert np.all(row_statistics(row)[:, 1] == 0.0)


def test_row_template_mapping_and_order():
    plane = np.zeros((3, 10), dtype=np.float32)
    plane[0, 7] = 9
    plane[1, 2] = 9
    plane[2, 5] = 9
    c = find_candidates(plane, 1.0, row_template=[40, 12, 12])
    assert [(int(r["t"]), int(r["p"])) for r in c] == [(12, 2), (12, 5), (40, 7)]


def _brute(plane, k):
    out = []
    for i, row in enumerate(plane.tolist()):
        mu = statistics.fmean(row)
        sd = statistics.pstdev(row)
        n = len(row)
        for p in range(n):
            left_ok = p == 0 or row[p] > row[p - 1]
            right_ok = p == n - 1 or row[p] >= row[p + 1]
            if left_ok and right_ok and row[p] > mu + k * sd:
                out.append((i, p))
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_on_exponential_noise(seed):
    rng = np.random.default_rng(seed)
    plane = rng.exponential(1.0, size=(4, 3000)).astype(np.float32)
    plane[1, 100:104] = 30.0           # a plateau: one candidate at its left end
    for k in (1.0, 3.0):
        got = [(int(r["t"]), int(r["p"])) for r in find_candidates(plane, k)]
        assert got == _brute(plane, k)
    st = row_statistics(plane)
    for i in range(4):
        assert abs(st[i, 1] - statistics.pstdev(plane[i].tolist())) < 1e-12
