"""Seeded synthetic term/document matrices shaped like the paper's corpora.

The paper factors term/document count matrices of text collections (Section 3:
rows are terms, columns are documents, entry (i, j) counts term i in document
j).  None of those collections is available here, so this module draws
stand-ins with the same structure:

* term frequencies follow a Zipf law (a few terms occur in almost every
  document, most terms are rare), so term rows are heavily skewed while
  document columns are uniform;
* counts are lognormal, then scaled by a smoothed inverse document frequency
  (TF-IDF), so every stored value is strictly positive (A >= 0, Eq. (1));
* initial factors are uniform on [0, 1).

Everything is drawn from ``numpy.random.Generator(PCG64(seed))`` in a fixed
order, so a (workload, seed) pair always gives the same bytes.  FP32
workloads round the values to float32 before anyone sees them; the oracle
then receives those rounded values widened to float64.

This module performs none of the factorization's arithmetic.
"""

from __future__ import annotations

import os
from dataclasses import dataclass, field
from typing import Callable, Dict, Optional

import numpy as np


@dataclass
class Corpus:
    """Sparse non-negative A (n terms x m docs) in CSR over term rows."""

    n: int
    m: int
    indptr: np.ndarray   # int64 [n + 1]
    indices: np.ndarray  # int32 [nnz], doc ids ascending within each term row
    data: np.ndarray     # float32 or float64 [nnz], all > 0
    dtype: str = "f64"   # "f32" | "f64"
    meta: Dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def scipy(self, dtype=np.float64):
        """The same matrix as a ``scipy.sparse.csr_matrix`` (values widened)."""
        import scipy.sparse as sp

        return sp.csr_matrix(
            (self.data.astype(dtype), self.indices.astype(np.int64), self.indptr),
            shape=(self.n, self.m),
        )

    def dense(self, dtype=np.float64) -> np.ndarray:
        out = np.zeros((self.n, self.m), dtype=dtype)
        rows = np.repeat(np.arange(self.n), np.diff(self.indptr))
        out[rows, self.indices] = self.data
        return out


# ---------------------------------------------------------------------------
# Sparsity structure
# ---------------------------------------------------------------------------


def zipf_terms(n: int, alpha: float, rng: np.random.Generator) -> Callable[[int], np.ndarray]:
    """Return ``draw(size)`` giving term ids with P(rank r) proportional to r^-alpha.

    Rank r (1-based) maps to term id ``perm[r - 1]`` for a seeded permutation,
    so the heavy rows are scattered over the id range rather than packed at 0.
    """
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(alpha))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    perm = rng.permutation(n).astype(np.int64)

    def draw(size: int) -> np.ndarray:
        r = np.searchsorted(cdf, rng.random(size), side="right")
        np.minimum(r, n - 1, out=r)
        return perm[r]

    return draw


def pairs_structure(n: int, m: int, nnz: int, alpha: float, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. (term ~ Zipf, doc ~ uniform) pairs, duplicates rejected, until
    exactly ``nnz`` distinct pairs exist.  Returns sorted keys term * m + doc."""
    if nnz > n * m:
        raise ValueError("nnz exceeds n*m")
    draw = zipf_terms(n, alpha, rng)
    keys = np.empty(0, dtype=np.int64)
    accept = 1.0  # fraction of the last round's draws that were new pairs
    while True:
        have = keys.size
        # size a round by the last acceptance rate, so that saturated head rows
        # (most draws repeat an existing pair) do not need many rounds
        batch = max(4096, int(1.25 * (nnz - have) / max(accept, 0.02)) + 1024)
        i = draw(batch)
        j = rng.integers(0, m, size=batch, dtype=np.int64)
        keys = np.concatenate([keys, i * m + j])
        first = _first_occurrences(keys, n * m)
        if first.size >= nnz:
            keys = keys[first[:nnz]]
            break
        accept = (first.size - have) / batch
        keys = keys[first]
    keys.sort()
    return keys


def _first_occurrences(keys: np.ndarray, bound: int) -> np.ndarray:
    """Ascending positions of the first occurrence of each distinct value of
    ``keys`` (all in [0, bound)): what ``np.unique(return_index=True)`` gives,
    sorted, but through one unstable sort of key * len + position."""
    size = keys.size
    if size == 0:
        return np.empty(0, dtype=np.int64)
    if bound * size >= 2**62:
        _, first = np.unique(keys, return_index=True)
        first.sort()
        return first
    c = keys * size + np.arange(size, dtype=np.int64)
    c.sort()
    k = c // size
    head = np.ones(size, dtype=bool)
    head[1:] = k[1:] != k[:-1]
    first = c[head] - k[head] * size
    first.sort()
    return first


_PER_DOC_CHUNK = 16384


def per_doc_structure(n: int, m: int, d: int, alpha: float, rng: np.random.Generator) -> np.ndarray:
    """Every doc gets exactly ``d`` distinct Zipf terms: the first ``d``
    distinct values in its own stream of draws.  Returns sorted keys."""
    if d > n:
        raise ValueError("terms per doc exceeds n")
    draw = zipf_terms(n, alpha, rng)
    width = 2 * d + 64
    parts = []
    for j0 in range(0, m, _PER_DOC_CHUNK):
        c = min(_PER_DOC_CHUNK, m - j0)
        x = draw(c * width).reshape(c, width)
        terms = _first_distinct(x, d)
        bad = np.nonzero(terms[:, -1] < 0)[0]
        for b in bad:  # rare: keep drawing for this doc until d distinct terms
            stream = list(x[b])
            while True:
                stream.extend(draw(width).tolist())
                t = _first_distinct(np.asarray(stream, dtype=np.int64)[None, :], d)[0]
                if t[-1] >= 0:
                    terms[b] = t
                    break
        docs = np.arange(j0, j0 + c, dtype=np.int64)[:, None]
        parts.append((terms * m + docs).ravel())
    keys = np.concatenate(parts)
    keys.sort()
    return keys


def _first_distinct(x: np.ndarray, d: int) -> np.ndarray:
    """Per row of x, the first d distinct values in order of appearance
    (padded with -1 where fewer exist)."""
    order = np.argsort(x, axis=1, kind="stable")
    xs = np.take_along_axis(x, order, axis=1)
    first_sorted = np.ones(xs.shape, dtype=bool)
    first_sorted[:, 1:] = xs[:, 1:] != xs[:, :-1]
    first = np.zeros(x.shape, dtype=bool)
    np.put_along_axis(first, order, first_sorted, axis=1)
    rank = np.cumsum(first, axis=1)
    keep = first & (rank <= d)
    out = np.full((x.shape[0], d), -1, dtype=np.int64)
    rows, cols = np.nonzero(keep)
    slot = rank[rows, cols] - 1
    out[rows, slot] = x[rows, cols]
    return out


# ---------------------------------------------------------------------------
# Values and the assembled corpus
# ---------------------------------------------------------------------------


def make_corpus(n: int, m: int, *, seed: int, alpha: float, dtype: str = "f64",
                nnz: Optional[int] = None, per_doc: Optional[int] = None) -> Corpus:
    """Build A: Zipf/uniform structure, lognormal counts, smoothed TF-IDF.

    Exactly one of ``nnz`` (i.i.d. pairs) or ``per_doc`` (fixed terms per doc)
    selects the structure.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if (nnz is None) == (per_doc is None):
        raise ValueError("give exactly one of nnz, per_doc")
    if nnz is not None:
        keys = pairs_structure(n, m, int(nnz), alpha, rng)
    else:
        keys = per_doc_structure(n, m, int(per_doc), alpha, rng)
    rows = keys // m
    cols = (keys - rows * m).astype(np.int32)
    counts_per_row = np.bincount(rows, minlength=n).astype(np.int64)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts_per_row, out=indptr[1:])
    del keys, rows
    counts = rng.lognormal(0.0, 1.0, size=cols.size)  # canonical (row, col) order
    idf = np.log((1.0 + m) / (1.0 + counts_per_row.astype(np.float64))) + 1.0
    data = counts * np.repeat(idf, counts_per_row)
    if dtype == "f32":
        data = data.astype(np.float32)
    elif dtype != "f64":
        raise ValueError(dtype)
    return Corpus(n, m, indptr, cols, data, dtype,
                  meta=dict(seed=seed, alpha=alpha, nnz=nnz, per_doc=per_doc))


def make_labeled_corpus(n: int, m: int, n_j: int, per_doc: int, *, seed: int, alpha: float = 1.1,
                        share: float = 0.3, dtype: str = "f64"):
    """A corpus with planted document labels ("journals"), for the clustering
    accuracy of Eq. (acc): (Corpus, labels int32[m]).

    Documents are dealt to the n_j journals evenly (seeded shuffle).  Each
    journal ranks the vocabulary by its own seeded permutation, and so does a
    background shared by all; every draw of a document's terms comes from its
    journal's Zipf ranking, or with probability ``share`` from the
    background's.  A document keeps its first ``per_doc`` distinct terms;
    values are lognormal counts scaled by the smoothed IDF as in
    ``make_corpus``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    labels = rng.permutation(np.arange(m) % n_j).astype(np.int32)
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(alpha))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    perms = np.stack([rng.permutation(n) for _ in range(n_j + 1)]).astype(np.int64)  # row 0: background
    width = 2 * per_doc + 64
    parts = []
    for j0 in range(0, m, _PER_DOC_CHUNK):
        c = min(_PER_DOC_CHUNK, m - j0)
        ranks = np.minimum(np.searchsorted(cdf, rng.random((c, width)), side="right"), n - 1)
        src = np.where(rng.random((c, width)) < share, 0, 1 + labels[j0:j0 + c, None].astype(np.int64))
        terms = _first_distinct(perms[src, ranks], per_doc)
        if np.any(terms[:, -1] < 0):
            raise ValueError("per_doc too large for the vocabulary and draw width")
        docs = np.arange(j0, j0 + c, dtype=np.int64)[:, None]
        parts.append((terms * m + docs).ravel())
    keys = np.concatenate(parts)
    keys.sort()
    rows = keys // m
    cols = (keys - rows * m).astype(np.int32)
    counts_per_row = np.bincount(rows, minlength=n).astype(np.int64)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts_per_row, out=indptr[1:])
    counts = rng.lognormal(0.0, 1.0, size=cols.size)
    idf = np.log((1.0 + m) / (1.0 + counts_per_row.astype(np.float64))) + 1.0
    data = counts * np.repeat(idf, counts_per_row)
    data = data.astype(np.float32) if dtype == "f32" else data
    corpus = Corpus(n, m, indptr, cols, data, dtype,
                    meta=dict(seed=seed, alpha=alpha, per_doc=per_doc, n_j=n_j, share=share))
    return corpus, labels


def make_init(n: int, m: int, k: int, *, seed: int, dtype: str = "f64"):
    """U0 = U[0,1)^{n x k}, then V0 = U[0,1)^{m x k}, from PCG64(seed + 1000)."""
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    u0 = rng.random((n, k))
    v0 = rng.random((m, k))
    if dtype == "f32":
        u0 = u0.astype(np.float32)
        v0 = v0.astype(np.float32)
    return u0, v0


# ---------------------------------------------------------------------------
# Named workloads (sizes of the paper-scale runs this library is measured on)
# ---------------------------------------------------------------------------

WORKLOADS: Dict[str, Dict] = {
    # 2,000 terms x 1,000 docs, 1 % dense, FP64 end to end.
    "plain_f64_2000x1000": dict(n=2000, m=1000, nnz=20000, alpha=1.1, k=10, t_u=200, t_v=100,
                                iters=20, dtype="f64", seed=1),
    # 100k terms x 200k docs, 100 distinct terms per doc (20M nnz), FP32.
    "plain_f32_100kx200k": dict(n=100000, m=200000, per_doc=100, alpha=1.1, k=50, t_u=1000,
                                t_v=2000, iters=50, dtype="f32", seed=2),
    # 1M terms x 5M docs, 200 terms per doc (1B nnz), FP32.
    "scale_f32_1Mx5M": dict(n=1000000, m=5000000, per_doc=200, alpha=1.05, k=100, t_u=5000,
                            t_v=20000, iters=30, dtype="f32", seed=3),
}


def _cache_path(name: str) -> Optional[str]:
    root = os.environ.get("NMF_SYNTH_CACHE")
    if not root:
        return None
    os.makedirs(root, exist_ok=True)
    return os.path.join(root, f"{name}.npz")


def make_workload(name: str, *, with_init: bool = True):
    """(Corpus, U0, V0, params) for a named workload; cached to
    ``$NMF_SYNTH_CACHE`` when that is set."""
    p = dict(WORKLOADS[name])
    path = _cache_path(name)
    corpus = None
    if path and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        corpus = Corpus(int(z["n"]), int(z["m"]), z["indptr"], z["indices"], z["data"], p["dtype"])
    if corpus is None:
        corpus = make_corpus(p["n"], p["m"], seed=p["seed"], alpha=p["alpha"], dtype=p["dtype"],
                             nnz=p.get("nnz"), per_doc=p.get("per_doc"))
        if path:
            np.savez(path, n=corpus.n, m=corpus.m, indptr=corpus.indptr,
                     indices=corpus.indices, data=corpus.data)
    u0 = v0 = None
    if with_init:
        u0, v0 = make_init(p["n"], p["m"], p["k"], seed=p["seed"], dtype=p["dtype"])
    return corpus, u0, v0, p


def sparse_factor_init(rows: int, k: int, t: int, *, rng: np.random.Generator,
                       dtype: str = "f32") -> np.ndarray:
    """Dense rows x k array with exactly min(t, rows) nonzeros per column:
    distinct uniformly chosen rows, values U(0,1) (nonzero)."""
    out = np.zeros((rows, k), dtype=np.float64)
    tt = min(t, rows)
    for c in range(k):
        r = rng.choice(rows, size=tt, replace=False)
        v = rng.random(tt)
        v[v == 0.0] = 0.5
        out[r, c] = v
    return out.astype(np.float32) if dtype == "f32" else out


def batched_params(count: int = 256, seed: int = 5):
    """Per-corpus (n, m, density, k, t_u, t_v, seed) for a batch of independent
    corpora: n ~ U{500..50000}, m ~ U{300..20000}, density log-uniform in
    [0.1 %, 2 %], k ~ U{5..64}, t = floor(n/20), floor(m/20)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(rng.integers(500, 50001))
        m = int(rng.integers(300, 20001))
        dens = float(np.exp(rng.uniform(np.log(1e-3), np.log(2e-2))))
        k = int(rng.integers(5, 65))
        out.append(dict(n=n, m=m, density=dens, nnz=int(round(dens * n * m)), k=k,
                        t_u=n // 20, t_v=m // 20, seed=5000 + i))
    return out


def _batch_member(job):
    p, dtype, alpha = job
    c = make_corpus(p["n"], p["m"], seed=p["seed"], alpha=alpha, nnz=max(1, p["nnz"]), dtype=dtype)
    u0, _ = make_init(p["n"], p["m"], p["k"], seed=p["seed"], dtype=dtype)
    return dict(n=p["n"], m=p["m"], k=p["k"], t_u=p["t_u"], t_v=p["t_v"], nnz=c.nnz,
                indptr=c.indptr, indices=c.indices, data=c.data, u0=u0, corpus=c)


def make_batch(params, dtype: str = "f32", alpha: float = 1.1, workers: int = 1):
    """The corpora and initial U of a batch described by ``batched_params``:
    per problem a dict with n, m, k, t_u, t_v, indptr, indices, data, u0
    ("pairs" structure with the problem's nnz, U0 from PCG64(seed + 1000)).

    Each problem depends only on its own seed, so ``workers`` > 1 draws them
    in forked processes (call it before the process touches a GPU)."""
    jobs = [(p, dtype, alpha) for p in params]
    if workers <= 1 or len(jobs) <= 1:
        return [_batch_member(j) for j in jobs]
    import multiprocessing as mp

    # largest first, so the pool's tail is short
    order = sorted(range(len(jobs)), key=lambda i: -jobs[i][0]["nnz"])
    with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
        done = pool.map(_batch_member, [jobs[i] for i in order], chunksize=1)
    out = [None] * len(jobs)
    for i, r in zip(order, done):
        out[i] = r
    return out
