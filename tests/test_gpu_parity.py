"""GPU parity: the HIP library against the FP64 oracle on the same seeded
inputs.  Every test prints the case it runs before touching the GPU.

Tolerances: FP64 workloads agree to 1e-9 relative (only summation order
differs); FP32 workloads to the stated 1e-4 relative (Frobenius) on U, V and
the error curve, with support mismatches allowed only at near-ties (see
tests/parity.py).
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


def _problem(c, u0, k, t_u, t_v, dtype, **kw):
    NMF, _ = _nmf()
    return NMF(c.n, c.m, c.indptr, c.indices, c.data, u0, t_u=t_u, t_v=t_v, dtype=dtype, **kw)


# ------------------------------------------------------------------ FP64


def test_fp64_trajectory_2000x1000():
    """Full 20-iteration run of the 2000 x 1000 FP64 workload: every iterate
    and the E / R curves match the oracle."""
    p = synth.WORKLOADS["plain_f64_2000x1000"]
    c, u0, v0, p = synth.make_workload("plain_f64_2000x1000")
    _say(f"fp64 2000x1000 nnz={c.nnz} k={p['k']} 20 iterations")
    prob = _problem(c, u0, p["k"], p["t_u"], p["t_v"], "f64", v0=v0)
    A = c.scipy()
    e0 = prob.error()
    assert e0 == pytest.approx(oracle.error_direct(A, u0, v0), rel=1e-10)
    st = None
    for it in range(p["iters"]):
        prob.step(1)
        st = oracle.als(A, u0, p["t_u"], p["t_v"], 1, state=st)
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
    assert prob.max_nnz() == max(st.max_nnz_uv, int(np.count_nonzero(u0)) + int(np.count_nonzero(v0)))
    assert prob.error() == pytest.approx(st.E[-1], rel=1e-12)
    assert prob.residual() == pytest.approx(st.R[-1], rel=1e-12)
    # the stored sparse form agrees with the dense export
    rp, tp, vl = prob.sparse(0)
    S = sp.csr_matrix((vl, tp.astype(np.int64), rp.astype(np.int64)), shape=U.shape).toarray()
    np.testing.assert_array_equal(S, U)
    for r in range(U.shape[0]):
        assert np.all(np.diff(tp[rp[r]:rp[r + 1]].astype(int)) > 0)


# ------------------------------------------------------------------ FP32 teacher forced


def _teacher_forced(c, u0, k, t_u, t_v, iters, tol=1e-4):
    A = c.scipy()
    st = oracle.als(A, u0, t_u, t_v, iters, keep_steps=True)
    prob = _problem(c, u0, k, t_u, t_v, "f32")
    report = []
    for i, s in enumerate(st.steps):
        prob.set_factors(np.ascontiguousarray(s["U_in"], np.float32))
        prob.half_step(0)
        vpre = prob.pre(0)
        check_pre(vpre, oracle.clamp(s["V_pre"]), tol)
        _, V = prob.factors()
        dv = compare_factor(V, s["V"], s["V_pre"], tol)
        prob.set_factors(np.ascontiguousarray(s["U_in"], np.float32), v=np.ascontiguousarray(s["V"], np.float32))
        prob.half_step(1)
        upre = prob.pre(1)
        check_pre(upre, oracle.clamp(s["U_pre"]), tol)
        U, _ = prob.factors()
        du = compare_factor(U, s["U"], s["U_pre"], tol)
        report.append((i, dv, du))
        _say(f"  iter {i}: V {dv} | U {du}")
        assert dv.ok(tol) and du.ok(tol), (i, dv, du)
    prob.close()
    return report


def test_fp32_teacher_forced_small():
    c = synth.make_corpus(3000, 5000, seed=31, alpha=1.1, per_doc=40, dtype="f32")
    u0, _ = synth.make_init(3000, 5000, 16, seed=31, dtype="f32")
    _say(f"fp32 teacher-forced 3000x5000 nnz={c.nnz} k=16")
    _teacher_forced(c, u0, 16, t_u=80, t_v=120, iters=4)


def test_fp32_two_topics_per_lane_k80():
    c = synth.make_corpus(1500, 2500, seed=32, alpha=1.1, per_doc=50, dtype="f32")
    u0, _ = synth.make_init(1500, 2500, 80, seed=32, dtype="f32")
    _say(f"fp32 teacher-forced 1500x2500 nnz={c.nnz} k=80 (two topics per lane)")
    _teacher_forced(c, u0, 80, t_u=40, t_v=60, iters=2)


def test_fp32_heavy_rows_split():
    """Term rows longer than one work chunk (1024 nonzeros) are split and
    recombined in chunk order."""
    c = synth.make_corpus(2000, 12000, seed=33, alpha=1.1, per_doc=30, dtype="f32")
    lens = np.diff(c.indptr)
    assert lens.max() > 2 * 4096
    u0, _ = synth.make_init(2000, 12000, 8, seed=33, dtype="f32")
    _say(f"fp32 heavy rows 2000x12000 nnz={c.nnz} max row {lens.max()} k=8")
    _teacher_forced(c, u0, 8, t_u=50, t_v=300, iters=2)


def test_fp32_free_running_error_curve():
    c = synth.make_corpus(3000, 5000, seed=34, alpha=1.1, per_doc=40, dtype="f32")
    u0, _ = synth.make_init(3000, 5000, 12, seed=34, dtype="f32")
    _say(f"fp32 free-running 3000x5000 nnz={c.nnz} k=12, 8 iterations")
    prob = _problem(c, u0, 12, 100, 150, "f32")
    prob.step(8)
    E, R, nu, nv = prob.history()
    st = oracle.als(c.scipy(), u0, 100, 150, 8)
    _say(f"  E gpu {E[-1]:.6f} oracle {st.E[-1]:.6f}; nnz U {nu[-1]} V {nv[-1]}")
    np.testing.assert_allclose(E, st.E, rtol=1e-4)
    np.testing.assert_array_equal(nu, st.nnz_u)
    np.testing.assert_array_equal(nv, st.nnz_v)


# ------------------------------------------------------------------ special cases


def test_forced_ties_lowest_row_wins_gpu():
    """Duplicate documents produce identical rows of V_pre on both sides; the
    kept supports must agree exactly (lowest document index wins)."""
    rng = np.random.default_rng(7)
    n, m_base, k = 300, 200, 4
    base = sp.random(n, m_base, density=0.05, random_state=rng, format="csc",
                     data_rvs=lambda s: rng.uniform(0.1, 2.0, s)).toarray()
    cols = list(range(m_base)) + [5] * 40 + [17] * 40
    perm = rng.permutation(len(cols))
    Ad = base[:, [cols[p] for p in perm]]
    A = sp.csr_matrix(Ad)
    A.sort_indices()
    u0 = rng.uniform(0.1, 1.0, (n, k))
    _say("fp64 forced ties: 80 duplicated documents, t_v=30")
    NMF, _ = _nmf()
    prob = NMF(n, A.shape[1], A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64),
               u0, t_u=40, t_v=30, dtype="f64")
    prob.half_step(0)
    _, V = prob.factors()
    Vo, _ = oracle.half_step(sp.csr_matrix(A.T), u0, 30)
    np.testing.assert_array_equal(V != 0, Vo != 0)
    np.testing.assert_allclose(V, Vo, rtol=1e-10, atol=1e-14)


def test_dead_topic_gpu():
    c = synth.make_corpus(500, 400, seed=35, alpha=1.1, nnz=5000, dtype="f64")
    u0, _ = synth.make_init(500, 400, 5, seed=35, dtype="f64")
    u0[:, 3] = 0.0
    _say("fp64 dead topic (zero column of U0)")
    prob = _problem(c, u0, 5, 30, 20, "f64")
    prob.step(3)
    U, V = prob.factors()
    st = oracle.als(c.scipy(), u0, 30, 20, 3)
    assert not U[:, 3].any() and not V[:, 3].any()
    assert rel_fro(U, st.U) < 1e-9 and rel_fro(V, st.V) < 1e-9


def test_not_spd_surfaces_gpu():
    """Two equal columns of U0 with exact arithmetic (pivot 9 - 3*3 = 0): the
    Gram factorisation fails on the device and the synchronizing create call
    reports NMF_ERR_NOT_SPD."""
    _, NMFError = _nmf()
    u = np.array([[2.0, 2.0], [1.0, 1.0], [2.0, 2.0], [0.0, 0.0]])
    A = sp.csr_matrix(np.ones((4, 3)))
    _say("fp64 exactly singular Gram -> NMF_ERR_NOT_SPD")
    c = synth.Corpus(4, 3, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data, "f64")
    with pytest.raises(NMFError) as ei:
        _problem(c, u, 2, 2, 2, "f64")
    assert ei.value.status == -4


def test_invalid_inputs_gpu():
    NMF, NMFError = _nmf()
    c = synth.make_corpus(50, 40, seed=36, alpha=1.1, nnz=300, dtype="f64")
    u0, _ = synth.make_init(50, 40, 3, seed=36, dtype="f64")
    _say("input validation: negative value, NaN, unsorted columns, bad row pointer, negative U0")
    bad = c.data.copy()
    bad[7] = -1.0
    with pytest.raises(NMFError) as ei:
        NMF(50, 40, c.indptr, c.indices, bad, u0, t_u=5, t_v=5, dtype="f64")
    assert ei.value.status == -2
    bad[7] = np.nan
    with pytest.raises(NMFError) as ei:
        NMF(50, 40, c.indptr, c.indices, bad, u0, t_u=5, t_v=5, dtype="f64")
    assert ei.value.status == -2
    idx = c.indices.copy()
    r = int(np.argmax(np.diff(c.indptr)))
    idx[c.indptr[r]], idx[c.indptr[r] + 1] = idx[c.indptr[r] + 1], idx[c.indptr[r]]
    with pytest.raises(NMFError) as ei:
        NMF(50, 40, c.indptr, idx, c.data, u0, t_u=5, t_v=5, dtype="f64")
    assert ei.value.status == -1
    ip = c.indptr.copy()
    ip[-1] += 1
    with pytest.raises(NMFError) as ei:
        NMF(50, 40, ip, c.indices, c.data, u0, t_u=5, t_v=5, dtype="f64")
    assert ei.value.status == -1
    un = u0.copy()
    un[3, 1] = -0.5
    with pytest.raises(NMFError) as ei:
        NMF(50, 40, c.indptr, c.indices, c.data, un, t_u=5, t_v=5, dtype="f64")
    assert ei.value.status == -2


def test_determinism_and_resume():
    c = synth.make_corpus(3000, 5000, seed=37, alpha=1.1, per_doc=40, dtype="f32")
    u0, _ = synth.make_init(3000, 5000, 16, seed=37, dtype="f32")
    _say("fp32 determinism (two runs bitwise equal) and resume (3 + 3 == 6)")
    a = _problem(c, u0, 16, 80, 120, "f32")
    a.step(6)
    Ua, Va = a.factors()
    Ea, Ra, _, _ = a.history()
    b = _problem(c, u0, 16, 80, 120, "f32")
    b.step(6)
    Ub, Vb = b.factors()
    Eb, Rb, _, _ = b.history()
    np.testing.assert_array_equal(Ua, Ub)
    np.testing.assert_array_equal(Va, Vb)
    np.testing.assert_array_equal(Ea, Eb)
    np.testing.assert_array_equal(Ra, Rb)
    r = _problem(c, u0, 16, 80, 120, "f32")
    r.step(3)
    U3, V3 = r.factors()
    s = _problem(c, u0, 16, 80, 120, "f32")
    s.set_factors(U3, v=V3)
    s.step(3)
    Us, Vs = s.factors()
    np.testing.assert_array_equal(Us, Ua)
    np.testing.assert_array_equal(Vs, Va)


def test_tuning_parameters_fp64():
    """Every SpMM configuration (entry-by-entry threshold 0, 1, 3, 128, both
    step forms and 1 to 16 waves per block, on both halves, changed between
    iterations) reproduces the oracle's FP64 trajectory; out-of-range
    settings are refused."""
    from paper_1510_05237_amd import (NMF_PARAM_SPARSE_ROW_U, NMF_PARAM_SPARSE_ROW_V, NMF_PARAM_WAVES_U,
                                      NMF_PARAM_WAVES_V, NMF_PARAM_WIDE_U, NMF_PARAM_WIDE_V)

    _, NMFError = _nmf()
    c, u0, v0, p = synth.make_workload("plain_f64_2000x1000")
    A = c.scipy()
    settings = [(0, 0, 0, 0, 16, 8), (0, 1, 0, 1, 8, 16), (3, 1, 3, 0, 1, 2), (128, 0, 128, 1, 4, 1),
                (1, 0, 1, 1, 2, 4), (3, 0, 3, 1, 16, 16)]
    _say(f"fp64 2000x1000 k={p['k']}: {len(settings)} tuning settings, one per iteration")
    prob = _problem(c, u0, p["k"], p["t_u"], p["t_v"], "f64")
    st = None
    for it, (srv, wv, sru, wu, nwv, nwu) in enumerate(settings):
        prob.set_param(NMF_PARAM_SPARSE_ROW_V, srv)
        prob.set_param(NMF_PARAM_WIDE_V, wv)
        prob.set_param(NMF_PARAM_SPARSE_ROW_U, sru)
        prob.set_param(NMF_PARAM_WIDE_U, wu)
        prob.set_param(NMF_PARAM_WAVES_V, nwv)
        prob.set_param(NMF_PARAM_WAVES_U, nwu)
        prob.step(1)
        st = oracle.als(A, u0, p["t_u"], p["t_v"], 1, state=st)
        U, V = prob.factors()
        assert rel_fro(U, st.U) < 1e-9, (it, srv, wv, sru, wu, nwv, nwu)
        assert rel_fro(V, st.V) < 1e-9, (it, srv, wv, sru, wu, nwv, nwu)
        np.testing.assert_array_equal(U != 0, st.U != 0)
        np.testing.assert_array_equal(V != 0, st.V != 0)
    E, R, _, _ = prob.history()
    np.testing.assert_allclose(E, st.E, rtol=1e-9)
    for param, bad in ((NMF_PARAM_SPARSE_ROW_V, -1), (NMF_PARAM_SPARSE_ROW_U, 129), (NMF_PARAM_WIDE_V, 2),
                       (NMF_PARAM_WIDE_U, -1), (NMF_PARAM_WAVES_V, 3), (NMF_PARAM_WAVES_U, 32),
                       (NMF_PARAM_WAVES_U, 0), (99, 0)):
        with pytest.raises(NMFError):
            prob.set_param(param, bad)
    prob.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_k128_fits_lds(dtype):
    """k = 128, the largest supported: the float64 W of the SpMM epilogue
    (128 KiB) leaves room for fewer waves per block, which the launch picks;
    three iterations match the oracle."""
    c = synth.make_corpus(700, 500, seed=41, alpha=1.1, nnz=30000, dtype=dtype)
    u0, _ = synth.make_init(700, 500, 128, seed=41, dtype=dtype)
    _say(f"{dtype} 700x500 nnz={c.nnz} k=128, 3 iterations")
    A = c.scipy()
    prob = _problem(c, u0, 128, 40, 30, dtype)
    prob.step(3)
    st = oracle.als(A, u0.astype(np.float64), 40, 30, 3)
    U, V = prob.factors()
    tol = 1e-9 if dtype == "f64" else 1e-4
    if dtype == "f64":
        assert rel_fro(U, st.U) < tol and rel_fro(V, st.V) < tol
        np.testing.assert_array_equal(U != 0, st.U != 0)
    else:
        E, _, _, _ = prob.history()
        np.testing.assert_allclose(E, st.E, rtol=1e-4)
    prob.close()


def test_k128_fp32_half_steps_vs_oracle():
    """k = 128 in float32 (two topics per lane, the stream kernel in both
    halves, the k > 64 defaults): three iterations half-step by half-step
    from the GPU's own state, V against the oracle's V half from the
    previous U and U against the oracle's U half from the GPU's V (whole
    matrix, every column and every kept entry within 1e-4; supports equal
    but for near-ties)."""
    c = synth.make_corpus(700, 500, seed=42, alpha=1.1, nnz=30000, dtype="f32")
    u0, _ = synth.make_init(700, 500, 128, seed=42, dtype="f32")
    _say(f"f32 700x500 nnz={c.nnz} k=128, 3 iterations half-step by half-step")
    A = c.scipy()
    prob = _problem(c, u0, 128, 40, 30, "f32")
    prev = u0.astype(np.float64)
    for it in range(3):
        prob.step(1)
        U, V = prob.factors()
        _, iv = oracle.half_step(sp.csr_matrix(A.T), prev, 30)
        Vo = oracle.topt_per_column(oracle.clamp(iv["X_pre"]), 30)
        dv = compare_factor(V, Vo, iv["X_pre"], 1e-4)
        _, iu = oracle.half_step(A, V.astype(np.float64), 40)
        Uo = oracle.topt_per_column(oracle.clamp(iu["X_pre"]), 40)
        du = compare_factor(U, Uo, iu["X_pre"], 1e-4)
        _say(f"  iteration {it + 1}: V {dv} | U {du}")
        assert dv.ok(1e-4) and du.ok(1e-4), (it, str(dv), dv.elem_at, str(du), du.elem_at)
        prev = U.astype(np.float64)
    prob.close()


@pytest.mark.parametrize("k,dtype,expect", [
    # (wide_v, sparse_row_u, waves_u): float32 k <= 64 (fused V half), float64, k > 64
    (50, "f32", (0, 1, 8)), (50, "f64", (0, 1, 8)), (80, "f32", (1, 3, 16)), (80, "f64", (1, 3, 16))])
def test_parameter_defaults(k, dtype, expect):
    """The SpMM parameters a handle starts with depend on its shape as the
    header states: for k > 64 the V half's stream takes the wide step and the
    U half gathers rows of up to three entries entry by entry in 16-wave
    blocks; otherwise the narrow V step, rows of one entry and 8 waves."""
    from paper_1510_05237_amd import (NMF_PARAM_SPARSE_ROW_U, NMF_PARAM_SPARSE_ROW_V, NMF_PARAM_WAVES_U,
                                      NMF_PARAM_WAVES_V, NMF_PARAM_WIDE_U, NMF_PARAM_WIDE_V)
    c = synth.make_corpus(600, 500, seed=61, alpha=1.1, nnz=12000, dtype=dtype)
    u0, _ = synth.make_init(600, 500, k, seed=61, dtype=dtype)
    _say(f"parameter defaults {dtype} k={k}")
    prob = _problem(c, u0, k, 30, 30, dtype)
    got = (prob.get_param(NMF_PARAM_WIDE_V), prob.get_param(NMF_PARAM_SPARSE_ROW_U), prob.get_param(NMF_PARAM_WAVES_U))
    assert got == expect, got
    assert prob.get_param(NMF_PARAM_SPARSE_ROW_V) == 1 and prob.get_param(NMF_PARAM_WIDE_U) == 1
    assert prob.get_param(NMF_PARAM_WAVES_V) == 16
    prob.close()


def test_power_of_two_scaling_gpu():
    """Scaling A by 2^p leaves U and every support bit-identical and scales V
    by exactly 2^p on the GPU too (rounding commutes with the scaling)."""
    c = synth.make_corpus(3000, 5000, seed=38, alpha=1.1, per_doc=40, dtype="f32")
    u0, _ = synth.make_init(3000, 5000, 10, seed=38, dtype="f32")
    _say("fp32 power-of-two scaling of A")
    a = _problem(c, u0, 10, 60, 90, "f32")
    a.step(3)
    Ua, Va = a.factors()
    Ea, Ra, _, _ = a.history()
    c2 = synth.Corpus(c.n, c.m, c.indptr, c.indices, (c.data * np.float32(8.0)).astype(np.float32), "f32")
    b = _problem(c2, u0, 10, 60, 90, "f32")
    b.step(3)
    Ub, Vb = b.factors()
    Eb, Rb, _, _ = b.history()
    np.testing.assert_array_equal(Ua, Ub)
    np.testing.assert_array_equal(Va * np.float32(8.0), Vb)
    np.testing.assert_allclose(Ea, Eb, rtol=1e-12)
    np.testing.assert_array_equal(Ra, Rb)


def test_mode_none_is_algorithm_1_gpu():
    c = synth.make_corpus(400, 300, seed=39, alpha=1.1, nnz=5000, dtype="f64")
    u0, _ = synth.make_init(400, 300, 6, seed=39, dtype="f64")
    _say("fp64 mode none (Algorithm 1)")
    prob = _problem(c, u0, 6, 1, 1, "f64", mode="none")
    prob.step(4)
    U, V = prob.factors()
    st = oracle.als(c.scipy(), u0, 1, 1, 4, mode=oracle.MODE_NONE)
    assert rel_fro(U, st.U) < 1e-9 and rel_fro(V, st.V) < 1e-9


# ------------------------------------------------------------------ autograd loss


def test_loss_and_gradient_gpu():
    """NMFLoss: L = ||A - U V^T||_F^2 against the FP64 oracle, the
    hand-written backward against the FP64 gradient, and both against
    central differences of the row-restricted FP64 loss
    ||a_r - u_r V^T||^2 = ||a_r||^2 - 2 u_r . (a_r V) + u_r (V^T V) u_r^T,
    which is exactly quadratic in each entry (no truncation error)."""
    import torch
    from paper_1510_05237_amd import NMFLoss

    c = synth.make_corpus(2000, 3000, seed=41, alpha=1.1, per_doc=30, dtype="f32")
    k = 12
    rng = np.random.Generator(np.random.PCG64(4))
    U = synth.sparse_factor_init(2000, k, 100, rng=rng, dtype="f32")
    V = synth.sparse_factor_init(3000, k, 150, rng=rng, dtype="f32")
    _say(f"fp32 loss/gradient 2000x3000 nnz={c.nnz} k={k}")
    prob = _problem(c, U, k, 100, 150, "f32")
    Ut = torch.tensor(U, device="cuda:0", requires_grad=True)
    Vt = torch.tensor(V, device="cuda:0", requires_grad=True)
    L = NMFLoss.apply(prob, Ut, Vt)
    L.backward()
    A = c.scipy()
    L_or = oracle.loss(A, U, V)
    gU_or, gV_or = oracle.loss_grad(A, U, V)
    assert float(L) == pytest.approx(L_or, rel=1e-5)
    gU = Ut.grad.cpu().numpy()
    gV = Vt.grad.cpu().numpy()
    assert rel_fro(gU, gU_or) <= 1e-4
    assert rel_fro(gV, gV_or) <= 1e-4
    # upstream gradient scaling
    Ut.grad = None
    Vt.grad = None
    (3.0 * NMFLoss.apply(prob, Ut, Vt)).backward()
    assert rel_fro(Ut.grad.cpu().numpy(), 3.0 * gU_or) <= 1e-4
    # central differences at 64 entries: 32 of U, 32 of V, half in the support
    Ad = A.toarray()
    U64, V64 = U.astype(np.float64), V.astype(np.float64)

    def pick(M, n_in, n_out, seed):
        r = np.random.default_rng(seed)
        ins = np.argwhere(M != 0)
        outs = np.argwhere(M == 0)
        return [tuple(x) for x in ins[r.choice(len(ins), n_in, replace=False)]] + \
               [tuple(x) for x in outs[r.choice(len(outs), n_out, replace=False)]]

    GV = V64.T @ V64
    GU = U64.T @ U64
    h = 0.25
    for (i, j) in pick(U, 16, 16, 1):
        aV = Ad[i] @ V64

        def Lrow(u):
            return float(Ad[i] @ Ad[i] - 2.0 * u @ aV + u @ GV @ u)

        up, um = U64[i].copy(), U64[i].copy()
        up[j] += h
        um[j] -= h
        fd = (Lrow(up) - Lrow(um)) / (2 * h)
        assert gU[i, j] == pytest.approx(fd, rel=1e-4, abs=1e-4 * np.abs(gU_or).max())
    for (i, j) in pick(V, 16, 16, 2):
        aU = Ad[:, i] @ U64

        def Lcol(v):
            return float(Ad[:, i] @ Ad[:, i] - 2.0 * v @ aU + v @ GU @ v)

        vp, vm = V64[i].copy(), V64[i].copy()
        vp[j] += h
        vm[j] -= h
        fd = (Lcol(vp) - Lcol(vm)) / (2 * h)
        assert gV[i, j] == pytest.approx(fd, rel=1e-4, abs=1e-4 * np.abs(gV_or).max())


def test_profile_stage_marks():
    """Stage timing marks: every stage bracketed, or only the chosen ones
    (the others then record no interval); profiling leaves the iterates
    unchanged."""
    NMF, NMFError = _nmf()
    c = synth.make_corpus(900, 700, seed=8101, alpha=1.1, nnz=12000, dtype="f32")
    u0, _ = synth.make_init(900, 700, 10, seed=8101, dtype="f32")
    _say("profile marks f32 900x700 k=10: all stages, then spmm_v + gram_u only, 3 iterations each")
    ref = _problem(c, u0, 10, 40, 30, "f32")
    ref.step(6)
    a = _problem(c, u0, 10, 40, 30, "f32")
    a.profile(True)
    a.step(3)
    prof = a.profile_read()
    assert all(cnt == 3 and ms > 0 for ms, cnt in prof.values()), prof
    a.profile(True, stages=["spmm_v", "gram_u"])
    a.step(3)
    prof = a.profile_read()
    a.profile(False)
    for name, (ms, cnt) in prof.items():
        if name in ("spmm_v", "gram_u"):
            assert cnt == 3 and ms > 0, (name, prof)
        else:
            assert cnt == 0 and ms == 0, (name, prof)
    U, V = a.factors()
    U2, V2 = ref.factors()
    np.testing.assert_array_equal(U, U2)
    np.testing.assert_array_equal(V, V2)
    # half-steps open their own first stage
    a.profile(True, stages=["spmm_v", "spmm_u"])
    a.half_step(0)
    a.half_step(1)
    prof = a.profile_read()
    a.profile(False)
    assert prof["spmm_v"][1] == 1 and prof["spmm_u"][1] == 1 and prof["gram_v"][1] == 0, prof
    from paper_1510_05237_amd.nmf import load_library

    assert load_library().nmf_profile_stages(a.h, 1 << 9) != 0  # no such stage
    a.close()
    ref.close()


@pytest.mark.parametrize("k", [16, 50])
def test_hot_block_split(k):
    """float32, k <= 64: the densest terms' nonzeros are multiplied as a
    dense block on the matrix cores instead of streamed.  V_pre of a V half,
    plain iterations and the loss gradient agree with the unsplit path
    (NMF_FLAG_NO_HOT) to float32 rounding; V_pre, two further iterations
    (half-step by half-step) and the gradient agree with the oracle."""
    import torch
    from paper_1510_05237_amd import NMF_FLAG_NO_HOT, NMFLoss

    n, m = 2500, 3000
    c = synth.make_corpus(n, m, seed=43, alpha=1.1, per_doc=60, dtype="f32")
    df = np.diff(c.indptr)
    n_hot = int((df >= max(16, int(np.ceil(0.0625 * m)))).sum())
    assert n_hot >= 16, n_hot
    u0, _ = synth.make_init(n, m, k, seed=43, dtype="f32")
    # the three densest terms get empty rows of U: hot columns whose factor
    # row is not stored
    u0[np.argsort(-df, kind="stable")[:3]] = 0.0
    _say(f"hot block split f32 {n}x{m} nnz={c.nnz} k={k}: {n_hot} hot terms "
         f"({df[df >= max(16, int(np.ceil(0.0625 * m)))].sum() / c.nnz:.0%} of nnz)")
    a = _problem(c, u0, k, 60, 80, "f32")
    b = _problem(c, u0, k, 60, 80, "f32", flags=NMF_FLAG_NO_HOT)
    for p in (a, b):
        p.half_step(0)
    va, vb = a.pre(0), b.pre(0)
    _, d = oracle.half_step(sp.csr_matrix(c.scipy().T), u0.astype(np.float64), 80)
    assert rel_fro(va, vb) < 1e-5
    assert rel_fro(va, oracle.clamp(d["X_pre"])) < 1e-4
    for p in (a, b):
        p.half_step(1)
        p.step(2)
    Ea, _, _, _ = a.history()
    Eb, _, _, _ = b.history()
    np.testing.assert_allclose(Ea, Eb, rtol=1e-4)
    # two more iterations of the hot path, half-step by half-step against
    # the oracle from the GPU's own state (every column and kept entry)
    A = c.scipy()
    prev = a.factors()[0].astype(np.float64)
    for it in range(2):
        a.step(1)
        U, V = a.factors()
        _, iv = oracle.half_step(sp.csr_matrix(A.T), prev, 80)
        dv = compare_factor(V, oracle.topt_per_column(oracle.clamp(iv["X_pre"]), 80), iv["X_pre"], 1e-4)
        _, iu = oracle.half_step(A, V.astype(np.float64), 60)
        du = compare_factor(U, oracle.topt_per_column(oracle.clamp(iu["X_pre"]), 60), iu["X_pre"], 1e-4)
        _say(f"  hot path iteration {it + 1} vs oracle: V {dv} | U {du}")
        assert dv.ok(1e-4) and du.ok(1e-4), (it, str(dv), dv.elem_at, str(du), du.elem_at)
        prev = U.astype(np.float64)
    # the loss gradient through the hot block (dense U input)
    rng = np.random.Generator(np.random.PCG64(5))
    U = synth.sparse_factor_init(n, k, 60, rng=rng, dtype="f32")
    V = synth.sparse_factor_init(m, k, 80, rng=rng, dtype="f32")
    grads = []
    for p in (a, b):
        Ut = torch.tensor(U, device="cuda:0", requires_grad=True)
        Vt = torch.tensor(V, device="cuda:0", requires_grad=True)
        NMFLoss.apply(p, Ut, Vt).backward()
        grads.append((Ut.grad.cpu().numpy(), Vt.grad.cpu().numpy()))
    assert rel_fro(grads[0][0], grads[1][0]) < 1e-5 and rel_fro(grads[0][1], grads[1][1]) < 1e-5
    # and the hot path's gradient against the oracle's
    gU, gV = oracle.loss_grad(c.scipy(), U.astype(np.float64), V.astype(np.float64))
    assert rel_fro(grads[0][0], gU) < 1e-4 and rel_fro(grads[0][1], gV) < 1e-4
    a.close()
    b.close()
