"""Pins of the oracle's seeded sketch draw (oracle/sampling.py): the
counter-based generator against NumPy's own Philox4x64-10, Floyd's
algorithm by exhaustive subset frequencies, Box-Muller by its closed form
at the ends of its input range and by the normal distribution."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import sampling as S


@pytest.mark.parametrize("key,start", [((0, 0), 0), ((5, 7), 0), ((2**64 - 1, 12345), 1000),
                                       ((2603_21379, 3), 2**40)])
def test_philox_matches_numpy_philox(key, start):
    # NumPy increments the 256-bit counter before producing each 4-word block
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array([start, 0, 0, 0], dtype=np.uint64))
    ref = bg.random_raw(4 * 6)
    ctr = np.zeros((6, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(start + 1, start + 7, dtype=np.uint64)
    got = S.philox4x64_10(ctr, key).reshape(-1)
    np.testing.assert_array_equal(got, ref)


def test_philox_higher_counter_words():
    key = (11, 13)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array([2**64 - 1, 4, 9, 1], dtype=np.uint64))
    ref = bg.random_raw(4)    # counter (0, 5, 9, 1) after the carry
    got = S.philox4x64_10(np.array([[0, 5, 9, 1]], dtype=np.uint64), key).reshape(-1)
    np.testing.assert_array_equal(got, ref)


def test_floyd_every_subset_equally_likely():
    N, s, trials = 6, 3, 20000
    subsets = {c: 0 for c in itertools.combinations(range(N), s)}
    for seed in range(trials):
        subsets[tuple(S.draw_indices(N, s, seed, 0))] += 1
    expect = trials / len(subsets)
    sd = math.sqrt(expect * (1 - 1 / len(subsets)))
    assert max(abs(c - expect) for c in subsets.values()) < 5 * sd
    # and every position of the sorted draw takes its exact marginal law
    chi2, p = stats.chisquare(list(subsets.values()))
    assert p > 1e-4


def test_floyd_sizes_and_ranges():
    np.testing.assert_array_equal(S.draw_indices(10, 10, 3, 1), np.arange(10))
    assert S.draw_indices(10, 0, 3, 1).size == 0
    big = S.draw_indices(10**9, 3000, 2603, 2)
    assert big.size == 3000 and np.all(np.diff(big) > 0) and big[0] >= 0 and big[-1] < 10**9
    # different units and seeds give different draws
    assert not np.array_equal(S.draw_indices(10**6, 50, 1, 0), S.draw_indices(10**6, 50, 1, 1))
    assert not np.array_equal(S.draw_indices(10**6, 50, 1, 0), S.draw_indices(10**6, 50, 2, 0))
    with pytest.raises(ValueError):
        S.draw_indices(5, 6, 0, 0)


def test_box_muller_closed_form_at_the_ends():
    top = np.uint64(2**64 - 1)   # u1 = 1: radius 0
    assert S.box_muller(np.array([top]), np.array([np.uint64(123456789)]))[0] == 0.0
    # u1 = 2^-53, u2 = 0: sqrt(-2 ln 2^-53) = sqrt(106 ln 2)
    z = S.box_muller(np.array([np.uint64(0)]), np.array([np.uint64(0)]))[0]
    assert z == pytest.approx(math.sqrt(106 * math.log(2)), rel=1e-15)
    # u2 = 1/2: cos(pi) = -1
    half = np.uint64(1 << 63)
    z = S.box_muller(np.array([np.uint64(0)]), np.array([half]))[0]
    assert z == pytest.approx(-math.sqrt(106 * math.log(2)), rel=1e-15)


def test_omega_is_standard_normal():
    om = S.draw_omega(400, 500, seed=2603, unit=1)
    z = om.reshape(-1)
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # columns uncorrelated
    c = np.corrcoef(om[:, :20].T)
    assert np.max(np.abs(c - np.eye(20))) < 5 / math.sqrt(400) + 0.05
