"""Seeded synthetic term/document corpora and initial factors.

This package only draws inputs: it holds none of the factorization's
arithmetic, so both the HIP path and the CPU oracle can be fed from it.
"""

from .corpus import (  # noqa: F401
    Corpus,
    WORKLOADS,
    make_corpus,
    make_labeled_corpus,
    make_init,
    make_workload,
    zipf_terms,
    pairs_structure,
    per_doc_structure,
    batched_params,
    make_batch,
    sparse_factor_init,
)
