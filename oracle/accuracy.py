"""Document-clustering accuracy of one topic, Eq. (acc) of Section 3.2.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A document belongs to a topic when its entry in that column of V is nonzero.
The score counts same-journal pairs among the topic's n_D documents, then
rescales so that a topic drawn from a single journal scores 1 and a topic
spread as evenly as possible over the n_J journals scores 0:

    Acc = (S - alpha) / (beta - alpha),
    alpha = floor(n_D/n_J) * (n_J (floor(n_D/n_J) - 1) / 2 + (n_D mod n_J)),
    beta  = n_D (n_D - 1) / 2,

with Acc = 1 when n_D <= 1 (the paper's convention).  Reading taken: with a
single journal (n_J = 1) every pair is a same-journal pair and alpha = beta,
so Acc = 1 there as well.
"""

from __future__ import annotations

import numpy as np


def alpha_beta(n_D: int, n_J: int):
    q, r = divmod(int(n_D), int(n_J))
    alpha = q * (n_J * (q - 1) / 2.0 + r)
    beta = n_D * (n_D - 1) / 2.0
    return alpha, beta


def topic_accuracy(labels, n_J: int) -> float:
    """Eq. (acc) for the journal labels of the documents in one topic."""
    labels = np.asarray(labels, dtype=np.int64)
    n_D = labels.size
    if n_D <= 1 or n_J <= 1:
        return 1.0
    counts = np.bincount(labels, minlength=n_J).astype(np.float64)
    same = float(np.sum(counts * (counts - 1.0) / 2.0))
    alpha, beta = alpha_beta(n_D, n_J)
    return (same - alpha) / (beta - alpha)
