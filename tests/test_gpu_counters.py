"""The gathered-entry counters of the history (NMF_HIST_GATHERED_V/U)
against the same sums formed on the CPU from the GPU's own factors: the V
half gathers, for every streamed nonzero (i, j) of A, the stored entries of
U's row i; the U half, for every nonzero, the stored entries of V's row j.
With every term streamed (NMF_FLAG_NO_HOT) the V-half count is the sum over
all nonzeros; by default the terms of the dense hot block (those in at least
1/16 of the documents, at least 16 nonzeros, the 128 densest, ties to the
lower term) are left out.  Every test prints its case before touching the
GPU."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _hot_terms(df, m):
    need = max(16, int(np.ceil(m / 16)))
    cand = np.flatnonzero(df >= need)
    order = cand[np.argsort(-df[cand], kind="stable")]
    return order[:128]


@pytest.mark.parametrize("flags", [0, 2])
def test_gathered_counts_match_the_factors(flags):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_05237_amd import NMF

    n, m, k = 3000, 5000, 16
    c = synth.make_corpus(n, m, seed=41, alpha=1.1, nnz=200000, dtype="f32")
    u0, _ = synth.make_init(n, m, k, seed=41, dtype="f32")
    _say(f"gathered-entry counters fp32 {n}x{m} nnz={c.nnz} k={k} flags={flags}: 4 iterations")
    p = NMF(n, m, c.indptr, c.indices, c.data, u0, t_u=300, t_v=400, dtype="f32", device="cuda:0", flags=flags)
    A = c.scipy()
    df = np.diff(A.indptr)
    dfv = np.diff(A.tocsc().indptr)
    streamed = df.copy()
    if flags == 0:
        streamed[_hot_terms(df, m)] = 0
    U_in = u0
    for it in range(4):
        p.step(1)
        U, V = p.factors()
        gv = p.history_field("gathered_v")[-1]
        gu = p.history_field("gathered_u")[-1]
        want_v = float(np.sum(streamed * np.count_nonzero(U_in, axis=1)))
        want_u = float(np.sum(dfv * np.count_nonzero(V, axis=1)))
        _say(f"  iteration {it + 1}: gathered V half {gv:.0f} (cpu {want_v:.0f}), U half {gu:.0f} (cpu {want_u:.0f})")
        assert gv == want_v and gu == want_u, (it, gv, want_v, gu, want_u)
        U_in = U
    p.close()


def test_conditioning_record_is_the_largest_diagonal_product():
    """NMF_HIST_COND_U/V: the largest G_cc (G^-1)_cc over the live topics of
    the factor's Gram matrix G at the end of the iteration (1 when G is
    diagonal, larger as the columns overlap), against numpy's inverse of the
    Gram matrix of the GPU's own final factors."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_05237_amd import NMF

    c = synth.make_corpus(500, 400, seed=35, alpha=1.1, nnz=5000, dtype="f64")
    u0, _ = synth.make_init(500, 400, 5, seed=35, dtype="f64")
    _say("fp64 500x400 k=5: conditioning record against numpy's inverse of the final Gram matrices")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=30, t_v=20, dtype="f64")
    prob.step(4)
    U, V = prob.factors()
    for F, field in ((U, "cond_u"), (V, "cond_v")):
        G = F.T @ F
        live = np.diag(G) > 0
        Gl = G[np.ix_(live, live)]
        ref = float(np.max(np.diag(Gl) * np.diag(np.linalg.inv(Gl))))
        got = prob.history_field(field)
        assert len(got) == 4, (field, got)
        assert ref > 1.0
        assert got[-1] == pytest.approx(ref, rel=1e-9), (field, got[-1], ref)
    prob.close()
