"""The seeded synthetic inputs have the structure the benchmark configurations
state (Zipf terms, exactly d distinct terms per document, lognormal counts
times TF-IDF weights, U0 uniform on [0, 1)), and the same seed gives the same
arrays."""

import numpy as np

import synth


def _inside_rows(indptr, nnz):
    """Mask over consecutive index pairs (p, p + 1) that lie in one row."""
    inside = np.ones(max(nnz - 1, 0), bool)
    b = indptr[1:-1]
    b = b[(b > 0) & (b < nnz)]
    inside[b - 1] = False
    return inside


def test_headline_corpus_recipe():
    c, u0, v0, p = synth.make_workload("plain_f32_100kx200k")
    assert (c.n, c.m, c.nnz) == (100_000, 200_000, 20_000_000)
    assert c.indptr.dtype == np.int64 and c.indices.dtype == np.int32 and c.data.dtype == np.float32
    # each document: exactly 100 distinct terms
    assert np.all(np.bincount(c.indices, minlength=c.m) == 100)
    d = np.diff(c.indices.astype(np.int64))
    assert np.all(d[_inside_rows(c.indptr, c.nnz)] > 0)  # documents ascending, no duplicate pair
    # values: lognormal(0, 1) counts times the TF-IDF weight ln((1 + m) / (1 + df)) + 1
    assert np.all(np.isfinite(c.data)) and c.data.min() > 0
    df = np.diff(c.indptr)
    idf = np.log((1.0 + c.m) / (1.0 + df)) + 1.0
    lc = np.log(c.data.astype(np.float64) / np.repeat(idf, df))
    assert abs(lc.mean()) < 0.01 and abs(lc.std() - 1.0) < 0.01
    # Zipf-heavy terms: the 128 most frequent hold about 38 % of the nonzeros
    share = np.sort(df)[::-1][:128].sum() / c.nnz
    assert 0.33 < share < 0.43, share
    # U0 ~ U[0, 1), rounded to float32
    assert u0.shape == (100_000, 50) and u0.dtype == np.float32
    assert u0.min() >= 0.0 and u0.max() < 1.0 and abs(float(u0.mean()) - 0.5) < 0.002


def test_pairs_corpus_and_seeds():
    c, _, _, p = synth.make_workload("plain_f64_2000x1000")
    assert (c.n, c.m, c.nnz) == (2000, 1000, 20_000)
    d = np.diff(c.indices.astype(np.int64))
    assert np.all(d[_inside_rows(c.indptr, c.nnz)] > 0)
    a = synth.make_corpus(700, 500, seed=5, alpha=1.1, nnz=12_000, dtype="f64")
    b = synth.make_corpus(700, 500, seed=5, alpha=1.1, nnz=12_000, dtype="f64")
    for x, y in ((a.indptr, b.indptr), (a.indices, b.indices), (a.data, b.data)):
        np.testing.assert_array_equal(x, y)
    e = synth.make_corpus(700, 500, seed=6, alpha=1.1, nnz=12_000, dtype="f64")
    assert not np.array_equal(a.indices, e.indices)
    u1, v1 = synth.make_init(700, 500, 4, seed=5)
    u2, v2 = synth.make_init(700, 500, 4, seed=5)
    np.testing.assert_array_equal(u1, u2)
    np.testing.assert_array_equal(v1, v2)
