"""The library's Eq. (acc) helper (from per-topic journal counts) against the
oracle's pinned definition (from label lists), on random and edge cases."""

import numpy as np

import oracle
from paper_1510_05237_amd.accuracy import accuracy_from_counts


def _labels_to_counts(label_lists, n_j):
    return np.stack([np.bincount(np.asarray(l, np.int64), minlength=n_j) for l in label_lists])


def test_accuracy_matches_oracle_random():
    rng = np.random.default_rng(3)
    for _ in range(200):
        n_j = int(rng.integers(1, 9))
        k = int(rng.integers(1, 6))
        lists = [rng.integers(0, n_j, size=int(rng.integers(0, 60))) for _ in range(k)]
        got = accuracy_from_counts(_labels_to_counts(lists, n_j), n_j)
        want = [oracle.topic_accuracy(l, n_j) for l in lists]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_accuracy_edge_cases():
    # single journal topic, an even spread, at most one document, one journal
    counts = np.array([[7, 0, 0], [3, 3, 3], [1, 0, 0], [0, 0, 0]])
    np.testing.assert_allclose(accuracy_from_counts(counts, 3), [1.0, 0.0, 1.0, 1.0])
    np.testing.assert_allclose(accuracy_from_counts(np.array([[5], [0]]), 1), [1.0, 1.0])
    # the most uneven spread that is not a single journal lies strictly between
    a = accuracy_from_counts(np.array([[9, 1, 0]]), 3)[0]
    assert 0.0 < a < 1.0
