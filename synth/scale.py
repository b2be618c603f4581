"""Seeded generator of the scale corpus (1M terms x 5M docs, 200 distinct
terms per doc, 1B nonzeros), drawn with torch on the GPU: the host recipe of
``make_corpus`` would take many minutes at this size.  Inputs only: no
factorization arithmetic.

Recipe (the same shapes and distributions as ``make_corpus``'s per-doc
structure; only which distinct draws a document keeps differs):
* term ranks ~ Zipf(alpha) over n by inverse-CDF sampling of uniform draws
  from ``torch.Generator(device).manual_seed(seed)``; rank -> term id through
  a seeded permutation, so heavy terms scatter over the id range;
* every document draws ``width`` ranks; of its distinct terms it keeps the
  ``d`` smallest ids (ids are a random permutation of the ranks, so this is
  a random subset of the distinct draws); a document with fewer than ``d``
  distinct draws draws again with twice the width;
* counts lognormal(0, 1) in document order; value = count x (ln((1+m)/(1+df))
  + 1), rounded to float32;
* U0 ~ U[0, 1)^{n x k} from the same generator, after the corpus.
The draws depend on the GPU's random-number streams, so the bytes are fixed
for a (seed, device type), not across devices.
"""

from __future__ import annotations

from dataclasses import dataclass


@dataclass
class ScaleCorpus:
    n: int
    m: int
    d: int
    indptr: "object"     # torch int64 [n + 1], device: CSR over terms
    indices: "object"    # torch int32 [nnz]: doc ids, ascending within a term
    data: "object"       # torch float32 [nnz]
    doc_terms: "object"  # torch int32 [m, d]: each doc's terms, ascending
    doc_vals: "object"   # torch float32 [m, d]: the matching values

    @property
    def nnz(self) -> int:
        return self.m * self.d


def make_scale_corpus(n: int, m: int, d: int, *, seed: int, alpha: float, device="cuda:0",
                      chunk: int = 250_000, width: int = 384) -> ScaleCorpus:
    import torch

    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    w = torch.arange(1, n + 1, device=dev, dtype=torch.float64).pow(-float(alpha))
    cdf = torch.cumsum(w, 0)
    cdf /= cdf[-1].clone()
    del w
    perm = torch.randperm(n, generator=g, device=dev).to(torch.int32)
    doc_terms = torch.empty((m, d), dtype=torch.int32, device=dev)

    def draw(rows: int, wd: int):
        u = torch.rand((rows, wd), generator=g, device=dev, dtype=torch.float64)
        r = torch.searchsorted(cdf, u, right=True).clamp_(max=n - 1)
        del u
        s = torch.sort(perm[r], dim=1).values
        first = torch.ones_like(s, dtype=torch.bool)
        first[:, 1:] = s[:, 1:] != s[:, :-1]
        rank = torch.cumsum(first, dim=1, dtype=torch.int32)
        keep = first & (rank <= d)
        ok = keep.sum(1) == d
        return s, keep, ok

    for j0 in range(0, m, chunk):
        c = min(chunk, m - j0)
        s, keep, ok = draw(c, width)
        out = torch.zeros((c, d), dtype=torch.int32, device=dev)
        good = ok.nonzero().squeeze(1)
        out[good] = s[good][keep[good]].view(-1, d)
        bad = (~ok).nonzero().squeeze(1)
        wd = width
        while bad.numel() > 0:
            wd *= 2
            s2, keep2, ok2 = draw(bad.numel(), wd)
            g2 = ok2.nonzero().squeeze(1)
            out[bad[g2]] = s2[g2][keep2[g2]].view(-1, d)
            bad = bad[(~ok2).nonzero().squeeze(1)]
        doc_terms[j0:j0 + c] = out
        del s, keep, ok, out
    flat_terms = doc_terms.view(-1)
    df = torch.bincount(flat_terms, minlength=n)
    counts = torch.empty(m * d, dtype=torch.float64, device=dev).log_normal_(0.0, 1.0, generator=g)
    idf = torch.log((1.0 + m) / (1.0 + df.to(torch.float64))) + 1.0
    doc_vals = (counts * idf[flat_terms.long()]).to(torch.float32).view(m, d)
    del counts, idf
    # CSR over terms: sort (term, doc) keys
    docs = torch.arange(m, device=dev, dtype=torch.int64).repeat_interleave(d)
    key = flat_terms.to(torch.int64) * m + docs
    del docs
    key, order = torch.sort(key)
    indices = (key % m).to(torch.int32)
    del key
    data = doc_vals.view(-1)[order]
    del order
    indptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    indptr[1:] = torch.cumsum(df, 0)
    return ScaleCorpus(n, m, d, indptr, indices, data, doc_terms, doc_vals)


def make_scale_init(n: int, k: int, *, seed: int, device="cuda:0"):
    """U0 ~ U[0, 1)^{n x k} float32, from its own generator (seed + 1000)."""
    import torch

    g = torch.Generator(device=torch.device(device))
    g.manual_seed(seed + 1000)
    return torch.rand((n, k), generator=g, device=torch.device(device), dtype=torch.float32)
