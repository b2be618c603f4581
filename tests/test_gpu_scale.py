"""GPU parity at the scale size: 1M terms x 5M docs, 200 distinct terms per
doc (1B nonzeros, held in both orientations in HBM), k = 100, t_u = 5000,
t_v = 20000, FP32 with FP64 solves.  The corpus is drawn on the GPU
(synth.scale).  One iteration of half-steps; the FP64 oracle's half-step
recomputes the rows of both pre-selection matrices for sampled documents and
terms (on the row-restricted matrix, from the GPU's own inputs to each
half-step: U0, then the GPU's V), and the top-t rule is
re-applied on the CPU to the GPU's whole pre-selection matrices (the kept
sets must equal the GPU's exactly).  Prints every step before it runs."""

import time

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from tests.parity import check_pre

pytestmark = pytest.mark.gpu

N, M, D, K, T_U, T_V = 1_000_000, 5_000_000, 200, 100, 5000, 20000


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _kept_exact(X, t):
    """Per-column top-t of X (rows x k, float32 values compared exactly):
    the t largest positives, ties at the threshold to the lowest rows."""
    keep = np.zeros(X.shape, dtype=bool)
    for c in range(X.shape[1]):
        col = X[:, c]
        pos = np.flatnonzero(col > 0)
        if pos.size <= t:
            keep[pos, c] = True
            continue
        theta = np.partition(col[pos], pos.size - t)[pos.size - t]  # t-th largest
        above = pos[col[pos] > theta]
        eq = pos[col[pos] == theta]  # ascending rows
        keep[above, c] = True
        keep[eq[: t - above.size], c] = True
    return keep


def test_scale_1Mx5M_sampled():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_05237_amd import NMF
    from synth.scale import make_scale_corpus, make_scale_init

    dev = torch.device("cuda:0")
    _say(f"scale {N}x{M}, {D} terms/doc, k={K}: drawing the corpus on the GPU")
    t0 = time.perf_counter()
    c = make_scale_corpus(N, M, D, seed=3, alpha=1.05, device=dev)
    u0 = make_scale_init(N, K, seed=3, device=dev)
    torch.cuda.synchronize()
    _say(f"  drawn in {time.perf_counter() - t0:.1f}s; nnz={c.nnz}, longest term row {int((c.indptr[1:] - c.indptr[:-1]).max())}")
    t0 = time.perf_counter()
    prob = NMF(N, M, c.indptr, c.indices, c.data, u0, t_u=T_U, t_v=T_V, dtype="f32", device=dev)
    torch.cuda.synchronize()
    _say(f"  handle created in {time.perf_counter() - t0:.1f}s (workspace {prob.ws_bytes / 2**30:.1f} GiB)")
    rng = np.random.default_rng(17)
    docs = np.sort(rng.choice(M, 4096, replace=False))
    terms = np.sort(rng.choice(N, 4096, replace=False))
    dt = c.doc_terms[torch.from_numpy(docs).to(dev)].cpu().numpy()
    dv = c.doc_vals[torch.from_numpy(docs).to(dev)].cpu().numpy().astype(np.float64)
    ip = c.indptr.cpu().numpy()
    rows_idx = np.concatenate([np.arange(ip[i], ip[i + 1]) for i in terms])
    t_docs = c.indices[torch.from_numpy(rows_idx).to(dev)].cpu().numpy()
    t_vals = c.data[torch.from_numpy(rows_idx).to(dev)].cpu().numpy().astype(np.float64)
    t_len = np.array([ip[i + 1] - ip[i] for i in terms])
    del c
    torch.cuda.empty_cache()
    U0 = u0.cpu().numpy().astype(np.float64)

    _say("  V half")
    prob.half_step(0)
    vpre = prob.pre(0)
    # the oracle's half-step on the sampled documents' rows of A^T (its Gram
    # matrix is that of the whole U0)
    A_docs = sp.csr_matrix((dv.ravel(), dt.ravel(), np.arange(0, dt.size + 1, dt.shape[1])), shape=(docs.size, N))
    _, info = oracle.half_step(A_docs, U0, T_V)
    ref = oracle.clamp(info["X_pre"])
    rv = check_pre(vpre[docs].astype(np.float64), ref, 1e-4)
    _say(f"  V_pre sampled rows: worst (whole or column) rel {rv:.2e}")
    _, V = prob.factors()
    keep = _kept_exact(vpre, T_V)
    np.testing.assert_array_equal(V != 0, keep)
    np.testing.assert_array_equal(V[keep], vpre[keep])
    del vpre, keep

    _say("  U half")
    prob.half_step(1)
    upre = prob.pre(1)
    # the oracle's half-step on the sampled terms' rows of A, from the GPU's V
    starts = np.concatenate([[0], np.cumsum(t_len)])
    A_terms = sp.csr_matrix((t_vals, t_docs, starts), shape=(terms.size, M))
    _, info = oracle.half_step(A_terms, V.astype(np.float64), T_U)
    ref = oracle.clamp(info["X_pre"])
    ru = check_pre(upre[terms].astype(np.float64), ref, 1e-4)
    _say(f"  U_pre sampled rows: worst (whole or column) rel {ru:.2e}")
    U, _ = prob.factors()
    keep = _kept_exact(upre, T_U)
    np.testing.assert_array_equal(U != 0, keep)
    np.testing.assert_array_equal(U[keep], upre[keep])

    _say("  3 timed iterations")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.step(3)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / 3
    E = prob.error()
    _say(f"  {ms:.2f} ms/iteration ({1e3 / ms:.1f} it/s) at 1B nonzeros; E {E:.6f}")
    assert 0.0 < E < 1.0
    prob.close()
