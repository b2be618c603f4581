"""Document-clustering accuracy of Eq. (acc) (Section 3.2) from per-topic
journal counts.

For one topic, n_l documents of journal l belong to it (nonzero entry in
that column of V; the library counts them on the GPU with
``nmf_topic_counts``).  Among its n_D = sum n_l documents there are
S = sum n_l (n_l - 1) / 2 same-journal pairs out of beta = n_D (n_D - 1) / 2;
an even spread over the n_J journals gives alpha = q (n_J (q - 1) / 2 + r)
same-journal pairs with q, r = divmod(n_D, n_J).  The score
(S - alpha) / (beta - alpha) is 1 for a single-journal topic and 0 for an
even spread; topics with at most one document, or a corpus of one journal,
score 1.  Host arithmetic on k x n_J integers.
"""

from __future__ import annotations

import numpy as np


def accuracy_from_counts(counts, n_journals: int) -> np.ndarray:
    """Eq. (acc) for every topic; ``counts`` is k x n_journals (documents of
    each journal in each topic)."""
    cnt = np.asarray(counts, dtype=np.int64).reshape(-1, n_journals)
    out = np.ones(cnt.shape[0], dtype=np.float64)
    if n_journals <= 1:
        return out
    for c, row in enumerate(cnt):
        n_d = int(row.sum())
        if n_d <= 1:
            continue
        same = int((row * (row - 1)).sum()) // 2
        q, r = divmod(n_d, n_journals)
        # twice alpha and beta, to stay in integers
        alpha2 = q * (n_journals * (q - 1) + 2 * r)
        beta2 = n_d * (n_d - 1)
        out[c] = (2 * same - alpha2) / (beta2 - alpha2)
    return out
