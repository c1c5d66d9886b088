"""Pins of the retrieval oracle (oracle/retrieval.py): brute force over all
k-subsets on tiny inputs, ties, NaN placement, errors."""
import itertools

import numpy as np
import pytest

from oracle import knn


def brute(d, k):
    """The k-subset with the smallest sorted (distance, index) list, by enumeration."""
    best = None
    for sub in itertools.combinations(range(len(d)), k):
        key = sorted((d[j], j) for j in sub)
        if best is None or key < best:
            best = key
    return [j for _, j in best]


@pytest.mark.parametrize("seed", range(6))
def test_matches_enumeration(seed):
    rng = np.random.default_rng(seed)
    d = rng.integers(0, 4, size=7).astype(np.float64) / 3.0   # many ties
    for k in range(1, 8):
        idx, val = knn(d, k)
        assert list(idx) == brute(list(d), k)
        assert np.array_equal(val, d[idx])


def test_ties_by_index_and_order():
    d = np.array([0.5, 0.1, 0.5, 0.1, 0.0])
    idx, val = knn(d, 5)
    assert list(idx) == [4, 1, 3, 0, 2]
    assert np.all(np.diff(val) >= 0)


def test_nan_sorts_last():
    d = np.array([np.nan, 2.0, np.inf, 1.0])
    idx, _ = knn(d, 4)
    assert list(idx) == [3, 1, 2, 0]


def test_bad_k():
    with pytest.raises(ValueError):
        knn(np.zeros(3), 0)
    with pytest.raises(ValueError):
        knn(np.zeros(3), 4)
