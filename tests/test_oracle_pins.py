"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks it against a
closed form, a library routine solving the same problem another way, a brute
force enumeration, an invariant, or a symmetry of the method.
"""

import itertools
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import MODE_COLUMN, MODE_NONE, MODE_WHOLE
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_sparse(n, m, density, rng):
    A = sp.random(n, m, density=density, random_state=rng, format="csr",
                  data_rvs=lambda s: rng.uniform(0.1, 2.0, s))
    return A


# ---------------------------------------------------------------- worked example


def test_rank1_worked_example():
    """Hand-derived rank-1 run (closed forms; k=1 makes the inverse a division)."""
    g = json.load(open(os.path.join(GOLDEN, "rank1_worked.json")))
    A = sp.csr_matrix(np.array(g["A"]))
    U0 = np.array(g["U0"])
    for case in g["cases"]:
        st = oracle.als(A, U0, case["t_u"], case["t_v"], 1)
        np.testing.assert_allclose(st.V, case["V1"], rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(st.U, case["U1"], rtol=1e-15, atol=1e-15)
        assert st.R[0] == pytest.approx(case["R1"], rel=1e-14)
        assert st.E[0] == pytest.approx(case["E1"], rel=1e-14, abs=1e-15)
        if "R2" in case:
            st = oracle.als(A, U0, case["t_u"], case["t_v"], 1, state=st)
            assert st.R[1] == pytest.approx(case["R2"], abs=1e-15)
            assert st.E[1] == pytest.approx(case["E2"], rel=1e-14)


# ---------------------------------------------------------------- least squares


@pytest.mark.parametrize("seed", range(6))
def test_half_step_matches_lstsq_bruteforce(seed):
    """X_pre of a half-step is the least-squares solution of min ||A - U X^T||,
    which numpy.linalg.lstsq solves by SVD (a different route from Cholesky)."""
    rng = np.random.default_rng(seed)
    n, m, k = rng.integers(4, 9), rng.integers(4, 9), rng.integers(1, 4)
    A = _rand_sparse(n, m, 0.6, rng)
    U = rng.uniform(0.1, 1.0, (n, k))
    _, info = oracle.half_step(sp.csr_matrix(A.T), U, t=m, mode=MODE_COLUMN)
    ref = np.linalg.lstsq(U, A.toarray(), rcond=None)[0].T
    np.testing.assert_allclose(info["X_pre"], ref, rtol=1e-10, atol=1e-12)
    # and the U half mirrors it: min ||A^T - V U^T||
    V = rng.uniform(0.1, 1.0, (m, k))
    _, info = oracle.half_step(A, V, t=n, mode=MODE_COLUMN)
    ref = np.linalg.lstsq(V, A.toarray().T, rcond=None)[0].T
    np.testing.assert_allclose(info["X_pre"], ref, rtol=1e-10, atol=1e-12)


def test_normal_equations_hold():
    """V_pre (U^T U) = A^T U to 1e-10 relative at a moderate size."""
    c = synth.make_corpus(400, 300, seed=11, alpha=1.1, nnz=6000)
    A = c.scipy()
    U0, _ = synth.make_init(400, 300, 8, seed=11)
    _, info = oracle.half_step(sp.csr_matrix(A.T), U0, t=50)
    B = np.asarray(A.T @ U0)
    lhs = info["X_pre"] @ (U0.T @ U0)
    assert np.linalg.norm(lhs - B) / np.linalg.norm(B) <= 1e-10


def test_k1_is_division():
    """k = 1: (u^T u)^-1 is a floating-point division (Section 4)."""
    rng = np.random.default_rng(3)
    A = _rand_sparse(30, 20, 0.3, rng)
    u = rng.uniform(0.0, 1.0, (30, 1))
    V, info = oracle.half_step(sp.csr_matrix(A.T), u, t=7)
    v = (A.T @ u)[:, 0] / float(u[:, 0] @ u[:, 0])
    np.testing.assert_allclose(info["X_pre"][:, 0], v, rtol=1e-14)
    # top-7 of the positive entries, by brute force
    order = sorted(range(20), key=lambda r: (-v[r], r))
    keep = [r for r in order if v[r] > 0][:7]
    ref = np.zeros(20)
    ref[keep] = v[keep]
    # the Cholesky route divides by sqrt(u^T u) twice: equal up to rounding
    np.testing.assert_allclose(V[:, 0], ref, rtol=1e-14, atol=0)
    np.testing.assert_array_equal(V[:, 0] != 0, ref != 0)


# ---------------------------------------------------------------- sparsity rule


@pytest.mark.parametrize("seed", range(10))
def test_topt_bruteforce(seed):
    """Per-column top-t against an explicit Python sort with key (-value, row)."""
    rng = np.random.default_rng(100 + seed)
    rows, k = rng.integers(1, 12), rng.integers(1, 5)
    X = rng.integers(-3, 4, (rows, k)).astype(np.float64)  # small ints: many ties
    X = oracle.clamp(X)
    t = int(rng.integers(1, rows + 2))
    got = oracle.topt_per_column(X, t)
    ref = np.zeros_like(X)
    for c in range(k):
        cand = [r for r in range(rows) if X[r, c] > 0]
        cand.sort(key=lambda r: (-X[r, c], r))
        for r in cand[:t]:
            ref[r, c] = X[r, c]
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("seed", range(6))
def test_topt_whole_bruteforce(seed):
    rng = np.random.default_rng(200 + seed)
    rows, k = rng.integers(1, 9), rng.integers(1, 5)
    X = oracle.clamp(rng.integers(-2, 4, (rows, k)).astype(np.float64))
    t = int(rng.integers(1, rows * k + 2))
    got = oracle.topt_whole(X, t)
    cand = [(r, c) for r in range(rows) for c in range(k) if X[r, c] > 0]
    cand.sort(key=lambda rc: (-X[rc], rc[0], rc[1]))
    ref = np.zeros_like(X)
    for rc in cand[:t]:
        ref[rc] = X[rc]
    np.testing.assert_array_equal(got, ref)


def test_clamp_and_topt_invariants():
    """U, V >= 0; nnz per column <= t; kept values equal the pre-selection
    values; no dropped positive exceeds the smallest kept value."""
    c = synth.make_corpus(300, 500, seed=5, alpha=1.1, nnz=8000)
    A = c.scipy()
    U0, _ = synth.make_init(300, 500, 6, seed=5)
    st = oracle.als(A, U0, t_u=40, t_v=60, iters=3, keep_steps=True)
    for s in st.steps:
        for X, Xpre, t in ((s["V"], s["V_pre"], 60), (s["U"], s["U_pre"], 40)):
            assert (X >= 0).all()
            assert ((X != 0).sum(axis=0) <= t).all()
            kept = X != 0
            np.testing.assert_array_equal(X[kept], Xpre[kept])
            for col in range(X.shape[1]):
                if kept[:, col].any():
                    lo = X[kept[:, col], col].min()
                    dropped = (Xpre[:, col] > 0) & ~kept[:, col]
                    assert (Xpre[dropped, col] <= lo).all()


def test_forced_ties_lowest_row_wins():
    """Duplicate document columns give identical rows of V_pre; when the
    threshold falls among them the lowest document indices are kept."""
    rng = np.random.default_rng(7)
    n, m_base, k = 40, 12, 3
    base = _rand_sparse(n, m_base, 0.4, rng).toarray()
    # doc 3 copied into 6 more columns placed at scattered positions
    cols = list(range(m_base)) + [3] * 6
    perm = rng.permutation(len(cols))
    Ad = base[:, [cols[p] for p in perm]]
    A = sp.csr_matrix(Ad)
    U = rng.uniform(0.2, 1.0, (n, k))
    V, info = oracle.half_step(sp.csr_matrix(A.T), U, t=4)
    Xp = oracle.clamp(info["X_pre"])
    dup = [j for j, p in enumerate(perm) if cols[p] == 3]
    # identical rows bitwise
    for j in dup[1:]:
        np.testing.assert_array_equal(info["X_pre"][j], info["X_pre"][dup[0]])
    hit = False
    for c in range(k):
        col = Xp[:, c]
        kept = np.nonzero(V[:, c])[0]
        if col[dup[0]] <= 0:
            continue
        kept_dup = [j for j in dup if j in kept]
        n_above = int((col > col[dup[0]]).sum())
        if 0 < 4 - n_above < len(dup):
            hit = True
            assert kept_dup == sorted(dup)[: 4 - n_above]
    assert hit, "construction should put the threshold inside the tie block"


def test_t_at_least_rows_is_algorithm_1():
    c = synth.make_corpus(200, 150, seed=9, alpha=1.1, nnz=3000)
    A = c.scipy()
    U0, _ = synth.make_init(200, 150, 5, seed=9)
    a = oracle.als(A, U0, t_u=200, t_v=150, iters=4, mode=MODE_COLUMN)
    b = oracle.als(A, U0, t_u=1, t_v=1, iters=4, mode=MODE_NONE)
    np.testing.assert_array_equal(a.U, b.U)
    np.testing.assert_array_equal(a.V, b.V)
    assert a.E == b.E and a.R == b.R


# ---------------------------------------------------------------- exact recovery


def _disjoint_blocks(seed, n=60, m=45, k=3):
    rng = np.random.default_rng(seed)
    rb = np.array_split(rng.permutation(n), k)
    db = np.array_split(rng.permutation(m), k)
    U0 = np.zeros((n, k))
    V0 = np.zeros((m, k))
    for c in range(k):
        U0[rb[c], c] = rng.uniform(0.5, 1.5, rb[c].size)
        V0[db[c], c] = rng.uniform(0.5, 1.5, db[c].size)
    A = sp.csr_matrix(U0 @ V0.T)
    return A, U0, V0, rb, db, rng


def test_exact_recovery_from_truth():
    A, U0, V0, rb, db, _ = _disjoint_blocks(1)
    t_u, t_v = max(len(b) for b in rb), max(len(b) for b in db)
    st = oracle.als(A, U0, t_u, t_v, 1)
    np.testing.assert_allclose(st.V, V0, rtol=1e-12, atol=1e-14)
    assert oracle.error_direct(A, st.U, st.V) <= 1e-12
    assert st.R[0] <= 1e-12


def test_exact_recovery_from_noisy_start():
    """From U0 + 1e-2 U(0,1) noise one iteration gives U V^T = A: the top-t
    with t = |D_c| keeps exactly each block, V = V0 diag(M), U = U0 diag(M)^-1."""
    A, U0, V0, rb, db, rng = _disjoint_blocks(2)
    k = U0.shape[1]
    # per-column t equal to the block sizes (blocks have equal-ish sizes)
    t_u, t_v = min(len(b) for b in rb), min(len(b) for b in db)
    assert all(len(b) == t_u for b in rb) and all(len(b) == t_v for b in db)
    Uin = U0 + 1e-2 * rng.uniform(0.0, 1.0, U0.shape)
    st = oracle.als(A, Uin, t_u, t_v, 1)
    assert oracle.error_direct(A, st.U, st.V) <= 1e-12
    for c in range(k):
        assert set(np.nonzero(st.V[:, c])[0]) == set(db[c])
        assert set(np.nonzero(st.U[:, c])[0]) == set(rb[c])
    # a second iteration is a fixed point: R = 0 up to rounding
    st = oracle.als(A, Uin, t_u, t_v, 1, state=st)
    assert st.R[1] <= 1e-13


# ---------------------------------------------------------------- symmetries


def test_power_of_two_scaling_is_exact():
    """Section 2: the t-largest rule does not depend on the scaling.  Scaling
    A by 2^p commutes with rounding, so U and both supports are bit-identical,
    V scales by exactly 2^p, and E and R are unchanged."""
    c = synth.make_corpus(250, 180, seed=4, alpha=1.1, nnz=4000)
    A = c.scipy()
    U0, _ = synth.make_init(250, 180, 5, seed=4)
    a = oracle.als(A, U0, t_u=30, t_v=25, iters=3)
    for p in (-3, 5):
        b = oracle.als(A * 2.0 ** p, U0, t_u=30, t_v=25, iters=3)
        np.testing.assert_array_equal(a.U, b.U)
        np.testing.assert_array_equal(a.V * 2.0 ** p, b.V)
        assert a.R == b.R
        np.testing.assert_allclose(a.E, b.E, rtol=1e-14)


def test_topic_permutation():
    c = synth.make_corpus(220, 160, seed=6, alpha=1.1, nnz=3500)
    A = c.scipy()
    U0, _ = synth.make_init(220, 160, 5, seed=6)
    perm = np.array([3, 0, 4, 1, 2])
    a = oracle.als(A, U0, t_u=25, t_v=20, iters=3)
    b = oracle.als(A, U0[:, perm], t_u=25, t_v=20, iters=3)
    np.testing.assert_allclose(b.U, a.U[:, perm], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(b.V, a.V[:, perm], rtol=1e-9, atol=1e-12)
    np.testing.assert_array_equal(b.U != 0, (a.U != 0)[:, perm])


def test_term_permutation():
    c = synth.make_corpus(220, 160, seed=8, alpha=1.1, nnz=3500)
    A = c.scipy()
    U0, _ = synth.make_init(220, 160, 4, seed=8)
    perm = np.random.default_rng(0).permutation(220)
    a = oracle.als(A, U0, t_u=25, t_v=20, iters=3)
    b = oracle.als(A[perm], U0[perm], t_u=25, t_v=20, iters=3)
    np.testing.assert_allclose(b.U, a.U[perm], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(b.V, a.V, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------- metrics


def test_error_expansion_matches_dense():
    """The expanded E used at large sizes equals the dense definition."""
    c = synth.make_corpus(300, 400, seed=12, alpha=1.1, nnz=5000)
    A = c.scipy()
    U0, _ = synth.make_init(300, 400, 6, seed=12)
    st = oracle.als(A, U0, t_u=40, t_v=50, iters=2)
    U, V = st.U, st.V
    nA2 = float((A.data ** 2).sum())
    cross = float(np.sum(U * (A @ V)))
    quad = float(np.sum((U.T @ U) * (V.T @ V)))
    e_exp = np.sqrt(nA2 - 2 * cross + quad) / np.sqrt(nA2)
    assert e_exp == pytest.approx(oracle.error_direct(A, U, V), rel=1e-10)
    # dense definition via numpy's own Frobenius norm on the full matrix
    D = A.toarray() - U @ V.T
    assert oracle.error(A, U, V) == pytest.approx(np.sqrt((D * D).sum() / nA2), rel=1e-12)


def test_error_expansion_branch_matches_dense_large():
    """Past n*m = 4e6 the oracle's E switches to the expansion
    ||A||^2 - 2<U, AV> + <U^T U, V^T V> (Section 3.1's E, expanded so that no
    dense n x m matrix is formed).  Drive that branch on a 2100 x 2000 corpus
    and compare it with the dense definition formed explicitly: a dropped
    term, a wrong factor or a transposed Gram product moves E by O(1)."""
    n, m, k = 2100, 2000, 7
    assert n * m > 4_000_000
    c = synth.make_corpus(n, m, seed=31, alpha=1.1, nnz=60_000)
    A = c.scipy()
    U0, _ = synth.make_init(n, m, k, seed=31)
    st = oracle.als(A, U0, t_u=150, t_v=120, iters=2)
    e_branch = oracle.error(A, st.U, st.V)
    e_branch_c = oracle.error(A, st.U, st.V, C=A @ st.V)
    D = A.toarray() - st.U @ st.V.T
    e_dense = float(np.sqrt((D * D).sum()) / np.sqrt((A.data ** 2).sum()))
    assert 0.1 < e_dense < 1.0
    assert e_branch == pytest.approx(e_dense, rel=1e-12)
    assert e_branch_c == pytest.approx(e_dense, rel=1e-12)
    # the history the iteration records goes through the same branch
    assert st.E[-1] == pytest.approx(e_dense, rel=1e-12)


def test_error_expansion_branch_exact_recovery_large():
    """Disjoint-support blocks scaled past n*m = 4e6: A = U0 V0^T is recovered
    in one iteration from U0 (Section 3.1's E is then zero).  Through the
    expansion E is zero up to cancellation: nA2, 2<U,AV> and <G_U,G_V> agree
    to about 1e-15 relative, so E <= 1e-7 (sqrt of the rounding floor), while
    the dense definition reaches 1e-12."""
    rng = np.random.default_rng(33)
    n, m, k = 2400, 1800, 4
    assert n * m > 4_000_000
    rb = np.array_split(rng.permutation(n), k)
    db = np.array_split(rng.permutation(m), k)
    U0 = np.zeros((n, k))
    V0 = np.zeros((m, k))
    for cc in range(k):
        U0[rb[cc], cc] = rng.uniform(0.5, 1.5, rb[cc].size)
        V0[db[cc], cc] = rng.uniform(0.5, 1.5, db[cc].size)
    A = sp.csr_matrix(U0 @ V0.T)
    st = oracle.als(A, U0, max(map(len, rb)), max(map(len, db)), 1)
    assert st.E[0] <= 1e-7
    assert oracle.error_direct(A, st.U, st.V) <= 1e-12
    # a perturbed V moves the expansion exactly as the dense definition
    Vp = st.V.copy()
    Vp[db[0], 0] *= 1.01
    D = A.toarray() - st.U @ Vp.T
    e_dense = float(np.linalg.norm(D) / np.sqrt((A.data ** 2).sum()))
    assert oracle.error(A, st.U, Vp) == pytest.approx(e_dense, rel=1e-7)


def test_residual_definition_is_relative_to_new_iterate():
    U_old = np.array([[1.0, 0.0], [0.0, 2.0]])
    U_new = np.array([[2.0, 0.0], [0.0, 2.0]])
    # ||U_new - U_old|| = 1, ||U_new|| = sqrt(8)
    assert oracle.residual(U_new, U_old) == pytest.approx(1 / np.sqrt(8), rel=1e-15)


# ---------------------------------------------------------------- special inputs


def test_dead_topic_stays_zero():
    c = synth.make_corpus(120, 90, seed=13, alpha=1.1, nnz=2000)
    A = c.scipy()
    U0, _ = synth.make_init(120, 90, 4, seed=13)
    U0[:, 2] = 0.0
    st = oracle.als(A, U0, t_u=20, t_v=15, iters=3)
    assert not st.U[:, 2].any() and not st.V[:, 2].any()
    assert st.dead_u == [1, 1, 1]
    # the other topics equal a k=3 run without the dead column
    st3 = oracle.als(A, np.delete(U0, 2, axis=1), t_u=20, t_v=15, iters=3)
    np.testing.assert_allclose(np.delete(st.U, 2, axis=1), st3.U, rtol=1e-12, atol=1e-14)


def test_exactly_singular_gram_raises():
    """Two equal columns with exact arithmetic: G = [[9,9],[9,9]], the second
    pivot is 9 - 3*3 = 0 exactly."""
    U = np.array([[2.0, 2.0], [1.0, 1.0], [2.0, 2.0], [0.0, 0.0]])
    A = sp.csr_matrix(np.ones((4, 3)))
    with pytest.raises(oracle.NotSPD):
        oracle.half_step(sp.csr_matrix(A.T), U, t=3)


# ---------------------------------------------------------------- loss / gradient


def test_loss_matches_dense_definition():
    c = synth.make_corpus(80, 60, seed=14, alpha=1.1, nnz=900)
    A = c.scipy()
    rng = np.random.default_rng(1)
    U, V = rng.random((80, 5)), rng.random((60, 5))
    D = A.toarray() - U @ V.T
    assert oracle.loss(A, U, V) == pytest.approx(float((D * D).sum()), rel=1e-12)


def test_gradient_central_difference():
    """L is quadratic in every single entry, so a central difference has no
    truncation error: (L(x+h) - L(x-h)) / 2h is the exact partial derivative
    up to rounding.  Evaluated on the dense definition of L."""
    c = synth.make_corpus(30, 25, seed=15, alpha=1.1, nnz=200)
    A = c.scipy()
    Ad = A.toarray()
    rng = np.random.default_rng(2)
    U, V = rng.random((30, 3)), rng.random((25, 3))
    gU, gV = oracle.loss_grad(A, U, V)

    def Ldense(U_, V_):
        D = Ad - U_ @ V_.T
        return float((D * D).sum())

    h = 0.5
    for (i, j) in [(0, 0), (7, 2), (29, 1), (13, 0)]:
        Up, Um = U.copy(), U.copy()
        Up[i, j] += h
        Um[i, j] -= h
        assert (Ldense(Up, V) - Ldense(Um, V)) / (2 * h) == pytest.approx(gU[i, j], rel=1e-10, abs=1e-10)
    for (i, j) in [(0, 0), (24, 2), (11, 1)]:
        Vp, Vm = V.copy(), V.copy()
        Vp[i, j] += h
        Vm[i, j] -= h
        assert (Ldense(U, Vp) - Ldense(U, Vm)) / (2 * h) == pytest.approx(gV[i, j], rel=1e-10, abs=1e-10)


# ---------------------------------------------------------------- accuracy, Eq. (acc)


def test_accuracy_alpha_is_most_uniform_pair_count():
    """alpha equals the same-journal pair count of the most even split of n_D
    docs over n_J journals (brute force over all splits for small sizes)."""
    for n_J in range(2, 5):
        for n_D in range(0, 10):
            best = None
            for split in itertools.product(range(n_D + 1), repeat=n_J):
                if sum(split) != n_D:
                    continue
                pairs = sum(s * (s - 1) // 2 for s in split)
                best = pairs if best is None else min(best, pairs)
            alpha, beta = oracle.alpha_beta(n_D, n_J)
            assert alpha == best
            assert beta == n_D * (n_D - 1) // 2


def test_accuracy_extremes():
    assert oracle.topic_accuracy([2, 2, 2, 2], 5) == 1.0
    assert oracle.topic_accuracy([0, 1, 2, 3, 4], 5) == 0.0
    assert oracle.topic_accuracy([0, 1, 2, 3, 4, 0, 1, 2, 3, 4], 5) == 0.0
    assert oracle.topic_accuracy([3], 5) == 1.0
    assert oracle.topic_accuracy([], 5) == 1.0
    # two journals, 4 docs split 3/1: S = 3, alpha = 2, beta = 6 -> 0.25
    assert oracle.topic_accuracy([0, 0, 0, 1], 2) == pytest.approx(0.25)


# ---------------------------------------------------------------- sequential ALS (Algorithm 3)


def test_sequential_one_block_is_algorithm_2():
    """With a single block Algorithm 3 is its START step, Algorithm 2 itself."""
    c = synth.make_corpus(300, 220, seed=12, alpha=1.1, nnz=5000)
    A = c.scipy()
    U0, _ = synth.make_init(300, 220, 4, seed=12)
    seq = oracle.sequential_als(A, U0, 40, 30, k2=4, eta=1, iters=5)
    ref = oracle.als(A, U0, 40, 30, 5)
    np.testing.assert_array_equal(seq.U, ref.U)
    np.testing.assert_array_equal(seq.V, ref.V)
    np.testing.assert_allclose(seq.E, ref.E, rtol=1e-14)
    np.testing.assert_allclose(seq.R, ref.R, rtol=1e-14)


@pytest.mark.parametrize("k1,k2", [(2, 1), (3, 2), (1, 3)])
def test_sequential_deflation_is_least_squares(k1, k2):
    """The deflated solve equals the least-squares fit of U2 V2^T to the
    residual A - U1 V1^T (numpy's SVD-based lstsq), for both half-steps."""
    rng = np.random.default_rng(20 + k1 * 3 + k2)
    n, m = 9, 7
    A = sp.csr_matrix(rng.uniform(0.0, 2.0, (n, m)) * (rng.random((n, m)) < 0.6))
    U1, V1 = rng.uniform(0.1, 1.0, (n, k1)), rng.uniform(0.1, 1.0, (m, k1))
    U2, V2 = rng.uniform(0.1, 1.0, (n, k2)), rng.uniform(0.1, 1.0, (m, k2))
    Rsd = A.toarray() - U1 @ V1.T
    _, dv = oracle.deflated_half_step(sp.csr_matrix(A.T), U2, U1, V1, 10**6, mode=oracle.MODE_NONE)
    np.testing.assert_allclose(dv["X_pre"], np.linalg.lstsq(U2, Rsd, rcond=None)[0].T, rtol=1e-10, atol=1e-12)
    _, du = oracle.deflated_half_step(A, V2, V1, U1, 10**6, mode=oracle.MODE_NONE)
    np.testing.assert_allclose(du["X_pre"], np.linalg.lstsq(V2, Rsd.T, rcond=None)[0].T, rtol=1e-10, atol=1e-12)


def test_sequential_exact_factors_leave_nothing_to_deflate():
    """A = U* V*^T with disjoint supports.  The first block (Algorithm 2 from
    a noisy U*) recovers A exactly; the second block then fits a zero
    residual, so E stays at rounding level and the first block's columns
    are untouched."""
    A, Us, Vs, rb, db, rng = _disjoint_blocks(2)
    k = Us.shape[1]
    t_u, t_v = min(len(b) for b in rb), min(len(b) for b in db)
    U0 = Us + 1e-2 * rng.uniform(0.0, 1.0, Us.shape)
    st = oracle.sequential_als(A, U0, t_u, t_v, k2=k, eta=2, iters=2)
    assert st.E[1] <= 1e-12
    assert max(st.E[2:]) <= 1e-10
    first = oracle.sequential_als(A, U0, t_u, t_v, k2=k, eta=1, iters=2)
    np.testing.assert_array_equal(st.U[:, :k], first.U)
    np.testing.assert_array_equal(st.V[:, :k], first.V)


def test_sequential_invariants():
    """Blocks already found never change; every column keeps at most t
    positive entries; each block's first iteration restarts from U0."""
    c = synth.make_corpus(400, 300, seed=13, alpha=1.1, nnz=8000)
    A = c.scipy()
    U0, _ = synth.make_init(400, 300, 1, seed=13)
    t_u, t_v = 25, 20
    st = oracle.sequential_als(A, U0, t_u, t_v, k2=1, eta=4, iters=3, keep_steps=True)
    assert len(st.E) == 12
    for i, s in enumerate(st.steps):
        b = s["block"]
        if i % 3 == 0:
            np.testing.assert_array_equal(s["U_in"][:, b], U0[:, 0])
        if i > 0 and b > 0:
            prev = st.steps[i - 1]
            np.testing.assert_array_equal(s["U"][:, :b], prev["U"][:, :b])
            np.testing.assert_array_equal(s["V"][:, :b], prev["V"][:, :b])
        np.testing.assert_array_equal(s["U"][:, b + 1:], 0.0)
    assert np.all(st.U >= 0) and np.all(st.V >= 0)
    assert np.all((st.U > 0).sum(0) <= t_u) and np.all((st.V > 0).sum(0) <= t_v)
