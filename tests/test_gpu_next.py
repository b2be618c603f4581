"""GPU parity of the comparison baselines (Section 3.2): Algorithm 1 run to
the end with the top-t rule applied once afterwards ("enforce sparsity after
ALS"), per column and over the whole factor, against the FP64 oracle.  Every
test prints its case before touching the GPU."""

import numpy as np
import pytest

import oracle
import synth
from tests.parity import rel_fro

pytestmark = pytest.mark.gpu


def _lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_05237_amd import NMF, NMFError

    return NMF, NMFError


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.mark.parametrize("rule", ["column", "whole"])
def test_enforce_after_algorithm_1(rule):
    NMF, NMFError = _lib()
    c, u0, _, p = synth.make_workload("plain_f64_2000x1000")
    A = c.scipy()
    t_u, t_v = (200, 100) if rule == "column" else (1500, 700)
    _say(f"fp64 2000x1000 k={p['k']}: Algorithm 1 for 6 iterations, then top-t {rule} t_u={t_u} t_v={t_v}")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=1, t_v=1, dtype="f64", mode="none")
    prob.step(6)
    st = oracle.als(A, u0, 1, 1, 6, mode=oracle.MODE_NONE)
    U, V = prob.factors()
    assert rel_fro(U, st.U) < 1e-9 and rel_fro(V, st.V) < 1e-9
    dense_nnz = int(np.count_nonzero(U)) + int(np.count_nonzero(V))
    prob.enforce(t_u, t_v, mode=rule)
    top = oracle.topt_per_column if rule == "column" else oracle.topt_whole
    Uo, Vo = top(st.U, t_u), top(st.V, t_v)
    U, V = prob.factors()
    np.testing.assert_array_equal(U != 0, Uo != 0)
    np.testing.assert_array_equal(V != 0, Vo != 0)
    assert rel_fro(U, Uo) < 1e-9 and rel_fro(V, Vo) < 1e-9
    assert int(np.count_nonzero(U)) + int(np.count_nonzero(V)) < dense_nnz
    assert prob.error() == pytest.approx(oracle.error(A, Uo, Vo), rel=1e-9)
    # the largest storage of the run is the dense one of Algorithm 1
    assert prob.max_nnz() >= dense_nnz
    with pytest.raises(NMFError):
        prob.enforce(0, t_v, mode=rule)
    with pytest.raises(NMFError):
        prob.enforce(t_u, t_v, mode="none")
    prob.close()


def test_enforce_then_continue_column_mode():
    """Sparsified factors are a valid state: a column-mode handle continues
    from them exactly like the oracle started from the same factors."""
    NMF, _ = _lib()
    c = synth.make_corpus(600, 500, seed=81, alpha=1.1, nnz=12000, dtype="f64")
    u0, _ = synth.make_init(600, 500, 7, seed=81, dtype="f64")
    A = c.scipy()
    _say("fp64 600x500 k=7: 3 iterations, enforce(20, 15), 2 more iterations")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=40, t_v=30, dtype="f64")
    prob.step(3)
    prob.enforce(20, 15)
    U1, V1 = prob.factors()
    st0 = oracle.als(A, u0, 40, 30, 3)
    np.testing.assert_array_equal(U1 != 0, oracle.topt_per_column(st0.U, 20) != 0)
    prob.step(2)
    st = oracle.als(A, U1, 40, 30, 2)
    U, V = prob.factors()
    assert rel_fro(U, st.U) < 1e-9 and rel_fro(V, st.V) < 1e-9
    prob.close()


def test_topic_counts_and_accuracy():
    """Eq. (acc) on a corpus with planted journal labels: the GPU's per-topic
    journal counts equal a count over its own V, and the accuracy equals the
    oracle's on the oracle's factors (FP64: identical supports)."""
    NMF, NMFError = _lib()
    import torch

    c, labels = synth.make_labeled_corpus(3000, 1500, 4, 40, seed=83, dtype="f64")
    u0, _ = synth.make_init(3000, 1500, 4, seed=83, dtype="f64")
    _say("fp64 planted labels 3000x1500, 4 journals, k=4, 8 iterations, Eq. (acc)")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=150, t_v=200, dtype="f64")
    prob.step(8)
    counts = prob.topic_counts(labels, 4)
    _, V = prob.factors()
    want = np.stack([np.bincount(labels[V[:, t] != 0], minlength=4) for t in range(4)])
    np.testing.assert_array_equal(counts, want)
    counts_dev = prob.topic_counts(torch.from_numpy(labels).to("cuda:0"), 4)
    np.testing.assert_array_equal(counts_dev, want)
    # Eq. (acc) behind the ABI (device counts, library arithmetic)
    acc = prob.topic_accuracy(labels, 4)
    st = oracle.als(c.scipy(), u0, 150, 200, 8)
    acc_or = [oracle.topic_accuracy(labels[st.V[:, t] != 0], 4) for t in range(4)]
    np.testing.assert_allclose(acc, acc_or, rtol=0, atol=1e-12)
    np.testing.assert_allclose(prob.topic_accuracy(torch.from_numpy(labels).to("cuda:0"), 4), acc_or, rtol=0, atol=1e-12)
    with pytest.raises(NMFError):
        prob.topic_accuracy(labels, 0)
    with pytest.raises(NMFError):
        prob.topic_counts(labels, 0)
    with pytest.raises(NMFError):
        prob.topic_counts(labels, 257)
    prob.close()
