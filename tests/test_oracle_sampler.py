"""Pins for the oracle's sampler: a simple random sample of s distinct points
(Sec. 3.1: every X_i has cardinality s and is a simple random sample; Sec. 3.5:
uniform sampling)."""
import itertools

import numpy as np
import pytest
from scipy import stats

import oracle


@pytest.mark.parametrize("n,s", [(1, 1), (2, 1), (10, 10), (1000, 1), (1000, 999), (5000, 777)])
def test_sample_is_sorted_distinct_subset(n, s):
    for t in range(3):
        idx = oracle.sample(n, s, 42, t)
        assert idx.shape == (s,)
        assert np.all(np.diff(idx) > 0)
        assert idx.min() >= 0 and idx.max() < n


def test_full_sample_is_identity():
    assert np.array_equal(oracle.sample(257, 257, 5, 3), np.arange(257))


def test_sample_is_smallest_keys():
    # brute force: rank every (key, index) pair with numpy and keep the s smallest
    n, s, seed, t = 3000, 123, 77, 9
    keys = np.array([oracle.sample_key(seed, t, i) for i in range(n)], dtype=np.uint64)
    order = np.lexsort((np.arange(n), keys))
    want = np.sort(order[:s])
    assert np.array_equal(oracle.sample(n, s, seed, t), want)


def test_all_subsets_equally_likely():
    # m = 6, s = 3: the C(6,3) = 20 subsets must be equiprobable
    m, s, reps = 6, 3, 20000
    subsets = {c: i for i, c in enumerate(itertools.combinations(range(m), s))}
    counts = np.zeros(len(subsets), dtype=np.int64)
    for t in range(reps):
        counts[subsets[tuple(int(v) for v in oracle.sample(m, s, 2024, t))]] += 1
    assert stats.chisquare(counts).pvalue > 1e-4


def test_inclusion_probability():
    m, s, reps = 40, 7, 8000
    hits = np.zeros(m)
    for t in range(reps):
        hits[oracle.sample(m, s, 9, t)] += 1
    # each point is included with probability s/m
    assert stats.chisquare(hits, np.full(m, reps * s / m)).pvalue > 1e-4


def test_samples_differ_by_sample_index_and_seed():
    a = oracle.sample(10000, 100, 1, 0)
    assert not np.array_equal(a, oracle.sample(10000, 100, 1, 1))
    assert not np.array_equal(a, oracle.sample(10000, 100, 2, 0))
    assert np.array_equal(a, oracle.sample(10000, 100, 1, 0))


def test_invalid_sizes_rejected():
    with pytest.raises(ValueError):
        oracle.sample(5, 6, 1, 0)
