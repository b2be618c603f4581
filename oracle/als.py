"""FP64 reference of enforced-sparsity alternating least squares.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the library
imports or calls this module.

What it follows, by passage of the paper (Gavin, Gadepally, Kepner,
"Enforced Sparse Non-Negative Matrix Factorization"):

* The problem (Eqs. (1)-(2)): A ~ U V^T with A (n x m), U (n x k), V (m x k),
  all non-negative; minimise ||A - U V^T||.
* Algorithm 1 (projected ALS): V = A^T U (U^T U)^-1, negatives set to zero;
  then U = A V (V^T V)^-1, negatives set to zero; repeat.
* Algorithm 2 (enforced-sparsity ALS): after each projected half-step, keep
  only the t largest nonzeros (t_v for V, t_u for U).  Section 2 states the
  rule: find the t-th largest magnitude and zero the entries below it.
* Section 4, column-wise enforcement: the same rule applied to every column
  of U and of V separately.  This is the default mode here.
* Section 3.1: residual R = ||U_i - U_{i-1}|| / ||U_i|| and error
  E = ||A - U V^T|| / ||A||.

Readings taken where the paper is silent or loose (each also listed in the
design notes):

* "t largest" is strict: exactly min(t, #positive) entries survive per column;
  among entries equal to the t-th largest value, the lowest row indices win.
* Only strictly positive entries (after clamping) are candidates; a column
  with fewer than t positives keeps all of them.
* Norms are Frobenius norms.
* A topic whose Gram diagonal is zero (an all-zero column of the fixed
  factor) is "dead": its row and column of the Gram matrix are replaced by
  the identity, which keeps that topic at exactly zero.  Any other failure of
  the Cholesky factorisation is reported as NotSPD.
* One iteration is the V half-step followed by the U half-step, starting
  from U0; the initial U0 is used as given (not sparsified first).
* R at iteration 1 compares against U0.

Everything here is float64, with library primitives (sparse products,
Cholesky, sort) used as single steps and no reordering beyond the
algorithm's own.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

MODE_COLUMN = "column"  # Section 4: top-t in every column separately
MODE_NONE = "none"      # Algorithm 1: projection only
MODE_WHOLE = "whole"    # Algorithm 2 as printed: top-t over the whole matrix


class NotSPD(ArithmeticError):
    """The Gram matrix of the fixed factor is not positive definite."""


# ---------------------------------------------------------------------------
# Building blocks
# ---------------------------------------------------------------------------


def gram_dead(F: np.ndarray):
    """G = F^T F (the (U^T U) / (V^T V) of Algorithms 1-2), with dead topics
    (zero diagonal) replaced by identity rows/columns.  Returns (G, dead)."""
    F = np.asarray(F, dtype=np.float64)
    G = F.T @ F
    dead = np.diag(G) == 0.0
    if dead.any():
        G[dead, :] = 0.0
        G[:, dead] = 0.0
        G[dead, dead] = 1.0
    return G, dead


def clamp(X: np.ndarray) -> np.ndarray:
    """Projection of Algorithm 1: negative entries set to zero (and -0.0
    becomes +0.0)."""
    return np.where(X > 0.0, X, 0.0)


def topt_per_column(X: np.ndarray, t: int) -> np.ndarray:
    """Section 4 column-wise enforcement of the Section 2 rule: in each column
    keep the t largest strictly positive entries, ties at the threshold going
    to the lowest row index; every other entry becomes zero."""
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros_like(X)
    rows = np.arange(X.shape[0])
    for c in range(X.shape[1]):
        col = X[:, c]
        pos = np.nonzero(col > 0.0)[0]
        if pos.size <= t:
            out[pos, c] = col[pos]
            continue
        # primary key: value descending; secondary key: row ascending
        order = np.lexsort((rows[pos], -col[pos]))
        keep = pos[order[:t]]
        out[keep, c] = col[keep]
    return out


def topt_whole(X: np.ndarray, t: int) -> np.ndarray:
    """Algorithm 2 as printed: keep the t largest strictly positive entries of
    the whole matrix; ties go to the lowest (row, column) in row-major order."""
    X = np.asarray(X, dtype=np.float64)
    flat = X.ravel()
    pos = np.nonzero(flat > 0.0)[0]
    out = np.zeros_like(flat)
    if pos.size <= t:
        out[pos] = flat[pos]
    else:
        order = np.lexsort((pos, -flat[pos]))
        keep = pos[order[:t]]
        out[keep] = flat[keep]
    return out.reshape(X.shape)


def _enforce(X: np.ndarray, t: int, mode: str) -> np.ndarray:
    if mode == MODE_COLUMN:
        return topt_per_column(X, t)
    if mode == MODE_WHOLE:
        return topt_whole(X, t)
    if mode == MODE_NONE:
        return X
    raise ValueError(mode)


def half_step(A_rows, F: np.ndarray, t: int, mode: str = MODE_COLUMN):
    """One half-step of Algorithm 2.

    ``A_rows`` is the sparse operator whose rows index the factor being
    solved for: A^T (docs x terms) for the V half, A (terms x docs) for the U
    half.  ``F`` is the fixed factor (U for the V half, V for the U half).

    X_pre = (A_rows F) (F^T F)^-1   (least squares, via Cholesky)
    X     = t-largest(clamp(X_pre))

    Returns (X, info) with info = dict(B=A_rows F, G, dead, X_pre).
    """
    F = np.asarray(F, dtype=np.float64)
    G, dead = gram_dead(F)
    try:
        cf = sla.cho_factor(G, lower=True, check_finite=True)
    except np.linalg.LinAlgError as e:  # not positive definite
        raise NotSPD(str(e)) from None
    B = np.asarray(A_rows @ F, dtype=np.float64)
    X_pre = sla.cho_solve(cf, B.T).T
    X = _enforce(clamp(X_pre), t, mode)
    return X, dict(B=B, G=G, dead=dead, X_pre=X_pre)


def error_direct(A, U: np.ndarray, V: np.ndarray) -> float:
    """E = ||A - U V^T||_F / ||A||_F formed densely (small problems only)."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    D = Ad - np.asarray(U, np.float64) @ np.asarray(V, np.float64).T
    return float(np.linalg.norm(D) / np.linalg.norm(Ad))


def error(A, U: np.ndarray, V: np.ndarray, C: Optional[np.ndarray] = None) -> float:
    """E of Section 3.1.  Small problems: the dense definition.  Large ones:
    ||A - UV^T||^2 = ||A||^2 - 2<U, AV> + <U^T U, V^T V>, all in float64
    (``C`` = A V when the caller already has it)."""
    n, m = A.shape
    if n * m <= 4_000_000:
        return error_direct(A, U, V)
    A = sp.csr_matrix(A)
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    nA2 = float(np.dot(A.data.astype(np.float64), A.data.astype(np.float64)))
    if C is None:
        C = A @ V
    cross = float(np.sum(U * C))
    quad = float(np.sum((U.T @ U) * (V.T @ V)))
    return float(np.sqrt(max(0.0, nA2 - 2.0 * cross + quad)) / np.sqrt(nA2))


def residual(U_new: np.ndarray, U_old: np.ndarray) -> float:
    """R = ||U_i - U_{i-1}||_F / ||U_i||_F (Section 3.1), formed directly."""
    U_new = np.asarray(U_new, np.float64)
    num = np.linalg.norm(U_new - np.asarray(U_old, np.float64))
    den = np.linalg.norm(U_new)
    return float(num / den) if den > 0 else float("nan")


# ---------------------------------------------------------------------------
# The iteration
# ---------------------------------------------------------------------------


@dataclass
class OracleState:
    U: np.ndarray
    V: np.ndarray
    U_prev: np.ndarray
    iters: int = 0
    E: List[float] = field(default_factory=list)
    R: List[float] = field(default_factory=list)
    nnz_u: List[int] = field(default_factory=list)
    nnz_v: List[int] = field(default_factory=list)
    max_nnz_uv: int = 0
    dead_u: List[int] = field(default_factory=list)
    dead_v: List[int] = field(default_factory=list)
    steps: List[dict] = field(default_factory=list)


def als(A, U0: np.ndarray, t_u: int, t_v: int, iters: int, mode: str = MODE_COLUMN,
        V0: Optional[np.ndarray] = None, keep_steps: bool = False,
        state: Optional[OracleState] = None) -> OracleState:
    """Run ``iters`` iterations of Algorithm 2 (mode ``column``: the Section 4
    column-wise variant; ``none``: Algorithm 1; ``whole``: Algorithm 2 as
    printed).  Each iteration: V half-step from U, then U half-step from V;
    then R and E of Section 3.1 are recorded.

    ``state`` continues an earlier run (resume).  ``keep_steps`` stores every
    intermediate (for teacher-forced comparisons).
    """
    A = sp.csr_matrix(A, dtype=np.float64)
    At = sp.csr_matrix(A.T)
    if state is None:
        U = np.array(U0, dtype=np.float64, copy=True)
        V = np.zeros((A.shape[1], U.shape[1])) if V0 is None else np.array(V0, np.float64)
        # the initial guess counts toward the storage high-water mark
        state = OracleState(U=U, V=V, U_prev=U.copy(),
                            max_nnz_uv=int(np.count_nonzero(U) + (np.count_nonzero(V) if V0 is not None else 0)))
    U = state.U
    for _ in range(iters):
        V, dv = half_step(At, U, t_v, mode)
        U_new, du = half_step(A, V, t_u, mode)
        R = residual(U_new, U)
        E = error(A, U_new, V, C=du["B"])
        state.U_prev = U
        U = U_new
        state.U, state.V = U, V
        state.iters += 1
        state.E.append(E)
        state.R.append(R)
        nu, nv = int(np.count_nonzero(U)), int(np.count_nonzero(V))
        state.nnz_u.append(nu)
        state.nnz_v.append(nv)
        state.max_nnz_uv = max(state.max_nnz_uv, nu + nv)
        state.dead_u.append(int(dv["dead"].sum()))
        state.dead_v.append(int(du["dead"].sum()))
        if keep_steps:
            state.steps.append(dict(U_in=state.U_prev, V=V, U=U, V_pre=dv["X_pre"], U_pre=du["X_pre"],
                                    B=dv["B"], C=du["B"], G_U=dv["G"], G_V=du["G"]))
    return state


# ---------------------------------------------------------------------------
# Loss and gradient of the squared objective
# ---------------------------------------------------------------------------


def loss(A, U: np.ndarray, V: np.ndarray) -> float:
    """L = ||A - U V^T||_F^2 (the squared form of Eq. (2), as written for the
    block derivation of Section 4), expanded as
    ||A||^2 - 2 tr(U^T A V) + tr(U^T U V^T V) in float64."""
    A = sp.csr_matrix(A, dtype=np.float64)
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    nA2 = float(np.dot(A.data, A.data))
    return nA2 - 2.0 * float(np.sum(U * (A @ V))) + float(np.sum((U.T @ U) * (V.T @ V)))


def loss_grad(A, U: np.ndarray, V: np.ndarray):
    """Gradient of L: dL/dU = -2 A V + 2 U (V^T V), dL/dV = -2 A^T U + 2 V (U^T U)."""
    A = sp.csr_matrix(A, dtype=np.float64)
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    gU = -2.0 * (A @ V) + 2.0 * U @ (V.T @ V)
    gV = -2.0 * (A.T @ U) + 2.0 * V @ (U.T @ U)
    return np.asarray(gU), np.asarray(gV)
