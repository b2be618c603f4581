"""GPU parity of sequential ALS (Algorithm 3) against the FP64 oracle.
Every test prints its case before touching the GPU."""

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


@pytest.mark.parametrize("k2,iters", [(1, 4), (2, 3), (10, 5)])
def test_sequential_fp64_trajectory(k2, iters):
    """Blocks of k2 topics on the 2000 x 1000 FP64 workload (k = 10): the
    full factors and every E and R of the eta * iters iterations match the
    oracle; k2 = k is Algorithm 2."""
    NMF, _ = _lib()
    c, u0, _, p = synth.make_workload("plain_f64_2000x1000")
    A = c.scipy()
    eta = p["k"] // k2
    _say(f"fp64 sequential 2000x1000 k={p['k']} k2={k2} eta={eta} iters/block={iters}")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=p["t_u"], t_v=p["t_v"], dtype="f64")
    prob.sequential(k2, iters)
    U, V = prob.factors()
    st = oracle.sequential_als(A, u0[:, :k2], p["t_u"], p["t_v"], k2=k2, eta=eta, iters=iters)
    assert rel_fro(U, st.U) < 1e-9 and rel_fro(V, st.V) < 1e-9
    np.testing.assert_array_equal(U != 0, st.U != 0)
    np.testing.assert_array_equal(V != 0, st.V != 0)
    E, R, nu, nv = prob.history()
    assert len(E) == eta * iters
    np.testing.assert_allclose(E, st.E, rtol=1e-9)
    np.testing.assert_allclose(R, st.R, rtol=1e-8)
    np.testing.assert_array_equal(nu, st.nnz_u)
    np.testing.assert_array_equal(nv, st.nnz_v)
    assert prob.max_nnz() >= st.max_nnz_uv
    if k2 == p["k"]:
        ref = oracle.als(A, u0, p["t_u"], p["t_v"], iters)
        assert rel_fro(U, ref.U) < 1e-9
    prob.close()


@pytest.mark.parametrize("k,k2", [(80, 16), (80, 40)])
def test_sequential_fp64_wide_k(k, k2):
    """k > 64 (two topics per lane in the full-width kernels) with blocks of
    k2 <= 64 topics, whose products run over a column window one topic per
    lane: factors, E and R against the oracle."""
    NMF, _ = _lib()
    c = synth.make_corpus(1500, 1100, seed=51, alpha=1.1, nnz=40000, dtype="f64")
    u0, _ = synth.make_init(1500, 1100, k, seed=51, dtype="f64")
    A = c.scipy()
    eta, iters, t_u, t_v = k // k2, 2, 60, 45
    _say(f"fp64 sequential 1500x1100 k={k} k2={k2} eta={eta} iters/block={iters}")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=t_u, t_v=t_v, dtype="f64")
    prob.sequential(k2, iters)
    U, V = prob.factors()
    st = oracle.sequential_als(A, u0[:, :k2], t_u, t_v, k2=k2, eta=eta, iters=iters)
    assert rel_fro(U, st.U) < 1e-9 and rel_fro(V, st.V) < 1e-9
    np.testing.assert_array_equal(U != 0, st.U != 0)
    np.testing.assert_array_equal(V != 0, st.V != 0)
    E, R, _, _ = prob.history()
    np.testing.assert_allclose(E, st.E, rtol=1e-9)
    np.testing.assert_allclose(R, st.R, rtol=1e-8)
    prob.close()


def test_sequential_then_algorithm_2():
    """After a sequential run the handle continues with Algorithm 2 from the
    factors it found (the full inverse Gram is rebuilt first)."""
    NMF, _ = _lib()
    c = synth.make_corpus(800, 600, seed=91, alpha=1.1, nnz=15000, dtype="f64")
    u0, _ = synth.make_init(800, 600, 6, seed=91, dtype="f64")
    A = c.scipy()
    _say("fp64 800x600 k=6: sequential k2=2 x 3 iterations, then 3 iterations of Algorithm 2")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=60, t_v=50, dtype="f64")
    prob.sequential(2, 3)
    Us, _ = prob.factors()
    prob.step(3)
    U, V = prob.factors()
    st = oracle.als(A, Us, 60, 50, 3)
    assert rel_fro(U, st.U) < 1e-9 and rel_fro(V, st.V) < 1e-9
    np.testing.assert_array_equal(U != 0, st.U != 0)
    prob.close()


def test_sequential_fp32_error_curve():
    """FP32 products with FP64 solves: the E curve within the stated 1e-4."""
    NMF, _ = _lib()
    c = synth.make_corpus(3000, 5000, seed=92, alpha=1.1, per_doc=40, dtype="f32")
    u0, _ = synth.make_init(3000, 5000, 6, seed=92, dtype="f32")
    _say("fp32 sequential 3000x5000 k=6 k2=1 eta=6, 3 iterations per block")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=100, t_v=150, dtype="f32")
    prob.sequential(1, 3)
    E, _, _, _ = prob.history()
    st = oracle.sequential_als(c.scipy(), u0[:, :1], 100, 150, k2=1, eta=6, iters=3)
    _say(f"  E gpu {E[-1]:.6f} oracle {st.E[-1]:.6f}")
    np.testing.assert_allclose(E, st.E, rtol=1e-4)
    U, V = prob.factors()
    assert rel_fro(U, st.U) < 1e-4 and rel_fro(V, st.V) < 1e-4
    prob.close()


@pytest.mark.parametrize("k,k2,t_u", [(2, 1, 150), (6, 3, 60), (12, 4, 30)])
def test_sequential_fp32_small_k_many_rows(k, k2, t_u):
    """Regression: the float32 V half of a block reads a copy of U's block
    columns written into the dense storage of U's other buffer.  At the start
    of every block those columns hold the dense initial guess, so every row of
    U is nonempty; with k <= 12 a copy padded to 16 columns overran that
    storage (for k = 2 into the next factor's arrays).  The copy's pitch is
    now at most U's own.  E curve and factors against the oracle at the
    stated 1e-4."""
    NMF, _ = _lib()
    c = synth.make_corpus(400, 600, seed=97, alpha=1.1, nnz=12000, dtype="f32")
    u0, _ = synth.make_init(400, 600, k, seed=97, dtype="f32")
    eta = k // k2
    _say(f"fp32 sequential 400x600 nnz={c.nnz} k={k} k2={k2} t_u={t_u} t_v=100, 3 iterations per block")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=t_u, t_v=100, dtype="f32")
    prob.sequential(k2, 3)
    E, _, nu, _ = prob.history()
    st = oracle.sequential_als(c.scipy(), u0[:, :k2], t_u, 100, k2=k2, eta=eta, iters=3)
    _say(f"  E gpu {E[-1]:.6f} oracle {st.E[-1]:.6f}, nnz(U) {nu[-1]} over {c.n} rows")
    np.testing.assert_allclose(E, st.E, rtol=1e-4)
    U, V = prob.factors()
    assert rel_fro(U, st.U) < 1e-4 and rel_fro(V, st.V) < 1e-4
    prob.close()


def test_sequential_arguments():
    NMF, NMFError = _lib()
    c = synth.make_corpus(200, 150, seed=93, alpha=1.1, nnz=3000, dtype="f64")
    u0, _ = synth.make_init(200, 150, 6, seed=93, dtype="f64")
    _say("sequential argument checks (k2 not dividing k, iters 0, whole-matrix mode)")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=20, t_v=20, dtype="f64")
    for k2, it in ((4, 2), (0, 2), (2, 0)):
        with pytest.raises(NMFError) as ei:
            prob.sequential(k2, it)
        assert ei.value.status == -1
    prob.close()
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=100, t_v=100, dtype="f64", mode="whole")
    with pytest.raises(NMFError) as ei:
        prob.sequential(2, 2)
    assert ei.value.status == -3
    prob.close()


def test_sequential_on_recycled_memory():
    """Regression: the first block must not read the solved factor's storage
    (V does not exist before the first V half).  The workspace is carved from
    memory that held other data just before."""
    NMF, _ = _lib()
    import torch

    junk = torch.full((64 << 20,), -1, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()
    del junk
    c = synth.make_corpus(700, 500, seed=94, alpha=1.1, nnz=9000, dtype="f64")
    u0, _ = synth.make_init(700, 500, 4, seed=94, dtype="f64")
    _say("fp64 700x500 k=4 sequential k2=1 on a workspace carved from recycled memory")
    prob = NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=40, t_v=30, dtype="f64")
    prob.sequential(1, 2)
    U, V = prob.factors()
    st = oracle.sequential_als(c.scipy(), u0[:, :1], 40, 30, k2=1, eta=4, iters=2)
    assert rel_fro(U, st.U) < 1e-9 and rel_fro(V, st.V) < 1e-9
    prob.close()
