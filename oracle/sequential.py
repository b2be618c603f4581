"""FP64 reference of sequential ALS (Algorithm 3, Section 4).

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the library
imports or calls this module.

The factorization is found block by block: k2 new topics at a time are
solved for while the topics already found (U1, V1) are held fixed.  With
U = [U1 U2] and V = [V1 V2], minimising ||A - U1 V1^T - U2 V2^T|| over one of
U2, V2 with the other fixed gives the deflated least-squares solutions of
Eqs. (seq-V) and (seq-U):

    V2 = (A^T U2 - V1 (U1^T U2)) (U2^T U2)^-1
    U2 = (A V2 - U1 (V1^T V2)) (V2^T V2)^-1

each followed, as in Algorithm 2, by the clamp and the top-t rule.  The first
block (no U1 yet) is Algorithm 2 itself, started from U0; every later block
starts again from the same U0; then its columns are appended.

Readings taken (also in the design notes):
* "until convergence" is a fixed number of iterations per block;
* the top-t rule is applied to every column of the block separately (the
  column-wise rule of Section 4; with one topic per block, the paper's case,
  it is the same as the rule over the whole block);
* the factors are kept at their full width k = eta * k2, the columns of
  blocks not yet started being zero; R and E of Section 3.1 are recorded
  after every iteration on those full factors, R comparing with the factor
  as it stood when the iteration began (at a block's first iteration: the
  finished blocks, U0 in the block's columns, zeros after).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .als import MODE_COLUMN, NotSPD, OracleState, _enforce, clamp, error, gram_dead, residual


def deflated_half_step(A_rows, F2: np.ndarray, F1: np.ndarray, X1: np.ndarray, t: int,
                       mode: str = MODE_COLUMN):
    """One deflated half-step: X2_pre = (A_rows F2 - X1 (F1^T F2)) (F2^T F2)^-1,
    then clamp and top-t.  For the V half A_rows = A^T, F = U, X = V; for the
    U half A_rows = A, F = V, X = U.  Returns (X2, info)."""
    F2 = np.asarray(F2, dtype=np.float64)
    G, dead = gram_dead(F2)
    try:
        cf = sla.cho_factor(G, lower=True, check_finite=True)
    except np.linalg.LinAlgError as e:
        raise NotSPD(str(e)) from None
    B = np.asarray(A_rows @ F2, dtype=np.float64)
    if F1.shape[1] > 0:
        B = B - np.asarray(X1, np.float64) @ (np.asarray(F1, np.float64).T @ F2)
    X_pre = sla.cho_solve(cf, B.T).T
    X = _enforce(clamp(X_pre), t, mode)
    return X, dict(B=B, G=G, dead=dead, X_pre=X_pre)


def sequential_als(A, U0: np.ndarray, t_u: int, t_v: int, k2: int, eta: int, iters: int,
                   keep_steps: bool = False) -> OracleState:
    """Algorithm 3 with ``eta`` blocks of ``k2`` topics, ``iters`` iterations
    per block, from the n x k2 initial guess ``U0``.  The returned state holds
    the full n x (eta k2) and m x (eta k2) factors and one E, R record per
    iteration (eta * iters in all)."""
    A = sp.csr_matrix(A, dtype=np.float64)
    At = sp.csr_matrix(A.T)
    n, m = A.shape
    U0 = np.asarray(U0, dtype=np.float64)
    assert U0.shape == (n, k2)
    k = eta * k2
    U = np.zeros((n, k))
    V = np.zeros((m, k))
    st = OracleState(U=U, V=V, U_prev=U.copy(), max_nnz_uv=int(np.count_nonzero(U0)))
    for b in range(eta):
        k1 = b * k2
        blk = slice(k1, k1 + k2)
        U = U.copy()
        U[:, blk] = U0
        for _ in range(iters):
            U1, U2, V1 = U[:, :k1], U[:, blk], V[:, :k1]
            V2, dv = deflated_half_step(At, U2, U1, V1, t_v)
            V = V.copy()
            V[:, blk] = V2
            U2n, du = deflated_half_step(A, V2, V1, U1, t_u)
            U_new = U.copy()
            U_new[:, blk] = U2n
            st.R.append(residual(U_new, U))
            st.E.append(error(A, U_new, V))
            st.U_prev = U
            U = U_new
            st.U, st.V = U, V
            st.iters += 1
            nu, nv = int(np.count_nonzero(U)), int(np.count_nonzero(V))
            st.nnz_u.append(nu)
            st.nnz_v.append(nv)
            st.max_nnz_uv = max(st.max_nnz_uv, nu + nv)
            if keep_steps:
                st.steps.append(dict(block=b, U_in=st.U_prev, V=V, U=U, V2_pre=dv["X_pre"], U2_pre=du["X_pre"]))
    return st
