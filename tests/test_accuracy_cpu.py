"""The library's Eq. (acc) arithmetic (nmf_accuracy_from_counts, host code in
libnmf.so that needs no device) against the oracle's pinned definition (from
label lists), on random and edge cases."""

import numpy as np

import oracle
from paper_1510_05237_amd import NMFError, accuracy_from_counts


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


def test_accuracy_rejects_bad_counts():
    import pytest

    with pytest.raises(NMFError):
        accuracy_from_counts(np.array([[3, -1]]), 2)
    with pytest.raises((NMFError, ValueError)):
        accuracy_from_counts(np.zeros((1, 0), np.int64), 0)


def test_accuracy_large_counts_exact():
    """Counts near the largest corpus size (2^29 documents) stay exact in the
    library's 64-bit integer arithmetic."""
    n_j = 3
    row = np.array([[2 ** 28, 2 ** 27, 12345]])
    got = accuracy_from_counts(row, n_j)[0]
    same = sum(int(x) * (int(x) - 1) // 2 for x in row[0])
    from fractions import Fraction

    n_d = int(row.sum())
    q, r = divmod(n_d, n_j)
    alpha = Fraction(q * (n_j * (q - 1) + 2 * r), 2)
    beta = Fraction(n_d * (n_d - 1), 2)
    exact = (Fraction(same) - alpha) / (beta - alpha)
    assert abs(got - float(exact)) <= 1e-15
