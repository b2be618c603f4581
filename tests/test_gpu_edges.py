"""GPU parity at the degenerate shapes of the method, against the FP64 oracle:

* rank one (k = 1): the Gram matrix is the scalar u^T u and the solve is a
  division (Section 4); the oracle's k = 1 path is pinned to the closed form
  v = A^T u / (u^T u) on the CPU;
* tiny matrices with empty term rows and empty documents, which leave rows of
  the pre-selection matrices at zero, fewer rows than one tile of any kernel,
  and a quota t at or above the number of positive entries of a column;
* a corpus of a single document and one of a single term;
* an all-zero A, which is rejected at creation.

Every test prints its case before touching the GPU.  FP64 cases agree with
the oracle to 1e-9 relative (only the summation order differs) with identical
supports; FP32 cases are teacher-forced (every half-step from the oracle's
state) at the stated 1e-4.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from tests.parity import check_pre, compare_factor, rel_fro

pytestmark = pytest.mark.gpu


def _nmf():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_05237_amd import NMF, NMFError

    return NMF, NMFError


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _corpus(A, dtype):
    A = sp.csr_matrix(A)
    A.sort_indices()
    data = A.data.astype(np.float32 if dtype == "f32" else np.float64)
    return synth.Corpus(A.shape[0], A.shape[1], A.indptr.astype(np.int64), A.indices.astype(np.int32), data, dtype)


def _ragged(n, m, density, seed, empty_rows=(), empty_cols=()):
    """Random non-negative n x m matrix with the given rows and columns empty."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D = rng.random((n, m)) * (rng.random((n, m)) < density)
    D[list(empty_rows), :] = 0.0
    D[:, list(empty_cols)] = 0.0
    return D


def _fp64_run(c, u0, k, t_u, t_v, iters):
    NMF, _ = _nmf()
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=t_u, t_v=t_v, dtype="f64")
    A = c.scipy()
    st = None
    for it in range(iters):
        prob.step(1)
        st = oracle.als(A, u0, t_u, t_v, 1, state=st)
        U, V = prob.factors()
        assert rel_fro(U, st.U) < 1e-9, it
        assert rel_fro(V, st.V) < 1e-9, it
        np.testing.assert_array_equal(U != 0, st.U != 0)
        np.testing.assert_array_equal(V != 0, st.V != 0)
    E, R, nu, nv = prob.history()
    np.testing.assert_allclose(E, st.E, rtol=1e-9)
    np.testing.assert_allclose(R, st.R, rtol=1e-8)
    np.testing.assert_array_equal(nu, st.nnz_u)
    np.testing.assert_array_equal(nv, st.nnz_v)
    prob.close()
    return st


def test_rank_one_fp64():
    """k = 1 over a 700 x 500 corpus: six iterations, every iterate and the
    E / R curves against the oracle."""
    c = synth.make_corpus(700, 500, seed=91, alpha=1.1, nnz=12000, dtype="f64")
    u0, _ = synth.make_init(700, 500, 1, seed=91, dtype="f64")
    _say("fp64 rank one 700x500 nnz=12000 k=1 t_u=60 t_v=50: 6 iterations")
    st = _fp64_run(c, u0, 1, 60, 50, 6)
    assert st.nnz_v[-1] == 50 and st.nnz_u[-1] == 60


def _fp32_forced(c, u0, k, t_u, t_v, iters, tol=1e-4):
    """Each float32 half-step from the oracle's state: pre-selection matrices
    and kept factors within tol."""
    NMF, _ = _nmf()
    A = c.scipy()
    st = oracle.als(A, u0, t_u, t_v, iters, keep_steps=True)
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=t_u, t_v=t_v, dtype="f32")
    for i, s in enumerate(st.steps):
        prob.set_factors(np.ascontiguousarray(s["U_in"], np.float32))
        prob.half_step(0)
        check_pre(prob.pre(0), oracle.clamp(s["V_pre"]), tol)
        dv = compare_factor(prob.factors()[1], s["V"], s["V_pre"], tol)
        prob.set_factors(np.ascontiguousarray(s["U_in"], np.float32), v=np.ascontiguousarray(s["V"], np.float32))
        prob.half_step(1)
        check_pre(prob.pre(1), oracle.clamp(s["U_pre"]), tol)
        du = compare_factor(prob.factors()[0], s["U"], s["U_pre"], tol)
        _say(f"  iter {i}: V {dv} | U {du}")
        assert dv.ok(tol) and du.ok(tol), (i, dv, du)
    prob.close()


def test_rank_one_fp32_teacher_forced():
    """k = 1 in float32 over a 3000 x 2000 corpus."""
    c = synth.make_corpus(3000, 2000, seed=92, alpha=1.1, per_doc=30, dtype="f32")
    u0, _ = synth.make_init(3000, 2000, 1, seed=92, dtype="f32")
    _say("fp32 rank one 3000x2000 k=1 t_u=200 t_v=150: 4 teacher-forced iterations")
    _fp32_forced(c, u0, 1, 200, 150, 4)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("k,t_u,t_v", [(1, 6, 4), (3, 6, 4), (3, 40, 30), (4, 3, 2)])
def test_tiny_with_empty_lines(k, t_u, t_v, dtype):
    """37 terms x 23 documents, terms 0, 5 and 36 and documents 3 and 22
    empty: fewer rows than one tile, zero rows in both pre-selection
    matrices; (3, 40, 30) keeps every positive entry (t above the column
    counts), (4, 3, 2) keeps two documents per topic (one per topic can give
    two topics the same single document, an exactly singular Gram matrix
    that both sides report as not positive definite)."""
    D = _ragged(37, 23, 0.3, seed=93, empty_rows=(0, 5, 36), empty_cols=(3, 22))
    c = _corpus(D, dtype)
    u0, _ = synth.make_init(37, 23, k, seed=93 + k, dtype=dtype)
    _say(f"{dtype} tiny 37x23 nnz={c.nnz} (empty terms 0,5,36; empty docs 3,22) k={k} t_u={t_u} t_v={t_v}: 5 iterations")
    if dtype == "f32":
        _fp32_forced(c, u0, k, t_u, t_v, 5)
        return
    st = _fp64_run(c, u0, k, t_u, t_v, 5)
    assert not st.V[[3, 22], :].any()
    assert not st.U[[0, 5, 36], :].any()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_single_document(dtype):
    """One document (m = 1), k = 1: V is one number per iteration."""
    D = _ragged(9, 1, 0.7, seed=94)
    D[2, 0] = 0.5  # at least one entry
    c = _corpus(D, dtype)
    u0, _ = synth.make_init(9, 1, 1, seed=94, dtype=dtype)
    _say(f"{dtype} single document 9x1 nnz={c.nnz} k=1 t_u=4 t_v=1: 3 iterations")
    (_fp64_run if dtype == "f64" else _fp32_forced)(c, u0, 1, 4, 1, 3)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_single_term(dtype):
    """One term (n = 1), k = 1: U is one number per iteration."""
    D = _ragged(1, 11, 0.7, seed=95)
    D[0, 4] = 0.25
    c = _corpus(D, dtype)
    u0, _ = synth.make_init(1, 11, 1, seed=95, dtype=dtype)
    _say(f"{dtype} single term 1x11 nnz={c.nnz} k=1 t_u=1 t_v=5: 3 iterations")
    (_fp64_run if dtype == "f64" else _fp32_forced)(c, u0, 1, 1, 5, 3)


def test_all_zero_matrix_rejected():
    """||A|| = 0 (no stored entries, or only zeros stored) is refused with
    NMF_ERR_INVALID_INPUT before any kernel runs."""
    NMF, NMFError = _nmf()
    u0, _ = synth.make_init(6, 4, 2, seed=96, dtype="f64")
    _say("fp64 all-zero A (no entries; explicit zeros) -> NMF_ERR_INVALID_INPUT")
    empty = synth.Corpus(6, 4, np.zeros(7, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float64), "f64")
    with pytest.raises(NMFError) as ei:
        NMF(6, 4, empty.indptr, empty.indices, empty.data, u0, t_u=2, t_v=2, dtype="f64")
    assert ei.value.status == -2
    ip = np.array([0, 1, 1, 2, 2, 2, 2], np.int64)
    zeros = synth.Corpus(6, 4, ip, np.array([1, 3], np.int32), np.zeros(2, np.float64), "f64")
    with pytest.raises(NMFError) as ei:
        NMF(6, 4, zeros.indptr, zeros.indices, zeros.data, u0, t_u=2, t_v=2, dtype="f64")
    assert ei.value.status == -2
