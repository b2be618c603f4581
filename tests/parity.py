"""Comparison helpers for the GPU-vs-oracle parity tests (test code only).

A factor from the GPU and one from the oracle are compared in three parts:
* values, whole factor: relative Frobenius error over the entries both keep,
  normalised by the oracle factor's norm;
* values, per column and per entry: for every column c the relative error
  ||x_gpu,c - x_or,c|| / ||x_or,c|| over the entries both keep, and for every
  entry both keep |x_gpu - x_or| <= tol * max(|x_or|, theta_c, s_r), i.e. an
  element-wise relative bound whose floor is the larger of the column's
  threshold theta_c (the smallest value the oracle keeps in that column) and
  the row's scale s_r (its largest pre-selection value).  The row floor is
  the precision the float32 product allows: a row's raw sums are rounded
  relative to their own magnitude and the solve mixes all of them, so an
  entry that is small through cancellation carries an error of the row's
  size, not of its own.  A column or a few entries far off can no longer
  hide behind the norm of the rest;
* supports: every entry kept by one side only is a mismatch.  It is a
  near-tie when its pre-selection value lies within ``tol * theta_c`` of the
  oracle's threshold theta_c of that column (for the whole-matrix rule, the
  smallest value the oracle keeps anywhere); otherwise it is a non-tie
  mismatch.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class FactorDiff:
    rel: float          # whole-factor relative Frobenius error (entries both keep)
    mismatches: int
    near_ties: int
    non_ties: int
    col_rel: float = 0.0   # worst per-column relative error
    worst_col: int = -1
    elem: float = 0.0      # worst |dx| / max(|x_or|, theta_c, s_r) over entries both keep
    elem_at: tuple = ()    # (row, column, x_gpu, x_or, floor) of that entry

    def ok(self, tol: float) -> bool:
        return self.rel <= tol and self.col_rel <= tol and self.elem <= tol and self.non_ties == 0

    def __str__(self) -> str:
        return (f"rel {self.rel:.2e} worst column {self.worst_col} ({self.col_rel:.2e}) "
                f"worst entry {self.elem:.2e} mismatches {self.mismatches} "
                f"(near-tie {self.near_ties}, non-tie {self.non_ties})")


def compare_factor(X_gpu: np.ndarray, X_or: np.ndarray, Xpre_or: np.ndarray, tol: float = 1e-4,
                   whole: bool = False) -> FactorDiff:
    """``whole``: the factors come from the whole-matrix rule, whose one
    threshold is the smallest value the oracle keeps anywhere."""
    X_gpu = np.asarray(X_gpu, np.float64)
    X_or = np.asarray(X_or, np.float64)
    Xpre = np.where(np.asarray(Xpre_or, np.float64) > 0, Xpre_or, 0.0)
    row_scale = Xpre.max(axis=1) if Xpre.size else np.zeros(X_or.shape[0])
    kg, ko = X_gpu != 0, X_or != 0
    both = kg & ko
    den = np.linalg.norm(X_or)
    rel = float(np.linalg.norm(X_gpu[both] - X_or[both]) / den) if den > 0 else float(np.linalg.norm(X_gpu))
    theta_all = X_or[ko].min() if ko.any() else 0.0
    # per column: relative error of the entries both keep, element-wise bound
    D = np.where(both, X_gpu - X_or, 0.0)
    col_rel, worst_col, elem, elem_at = 0.0, -1, 0.0, ()
    for c in range(X_or.shape[1]):
        kept = X_or[ko[:, c], c]
        theta = theta_all if whole else (kept.min() if kept.size else 0.0)
        dc = D[:, c]
        nc = np.linalg.norm(X_or[:, c])
        r = float(np.linalg.norm(dc) / nc) if nc > 0 else float(np.linalg.norm(dc))
        if worst_col < 0 or r > col_rel:
            col_rel, worst_col = r, c
        sel = both[:, c]
        if sel.any():
            floor = np.maximum(np.maximum(np.abs(X_or[sel, c]), row_scale[sel]), max(theta, 1e-300))
            ratio = np.abs(dc[sel]) / floor
            j = int(np.argmax(ratio))
            if ratio[j] > elem:
                i = int(np.flatnonzero(sel)[j])
                elem, elem_at = float(ratio[j]), (i, int(c), float(X_gpu[i, c]), float(X_or[i, c]), float(floor[j]))
    mism = kg != ko
    near = non = 0
    for c in np.nonzero(mism.any(axis=0))[0]:
        kept = X_or[ko[:, c], c]
        theta = theta_all if whole else (kept.min() if kept.size else 0.0)
        for r in np.nonzero(mism[:, c])[0]:
            v = Xpre[r, c]
            if abs(v - theta) <= tol * max(theta, 1e-300):
                near += 1
            else:
                non += 1
    return FactorDiff(rel, int(mism.sum()), near, non, col_rel, worst_col, elem, elem_at)


def rel_fro(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / d) if d > 0 else float(np.linalg.norm(a))


def col_rel(a, b) -> float:
    """Worst per-column relative Frobenius error of ``a`` against ``b`` (a
    column of ``b`` that is entirely zero contributes ``||a_c||``)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.ndim == 1:
        return rel_fro(a, b)
    worst = 0.0
    for c in range(b.shape[1]):
        worst = max(worst, rel_fro(a[:, c], b[:, c]))
    return worst


def check_pre(a, b, tol: float) -> float:
    """A pre-selection (or raw product) matrix against the oracle's: the whole
    matrix and every column within ``tol`` relative; returns the worst."""
    w = max(rel_fro(a, b), col_rel(a, b))
    assert w <= tol, f"pre-selection matrix off: whole {rel_fro(a, b):.2e}, worst column {col_rel(a, b):.2e}"
    return w


def elem_kept(X_gpu, Xpre_or) -> float:
    """Worst element-wise error of the GPU's kept entries against the oracle's
    pre-selection values at the same positions (both sides took the step from
    the same input): max |x_gpu - x_or| / max(|x_or|, theta_c, s_r), theta_c
    the smallest value the GPU keeps in column c, s_r the row's largest
    pre-selection value (see the module docstring)."""
    X_gpu = np.asarray(X_gpu, np.float64)
    Xp = np.asarray(Xpre_or, np.float64)
    row_scale = np.where(Xp > 0, Xp, 0.0).max(axis=1)
    worst = 0.0
    for c in range(X_gpu.shape[1]):
        sel = X_gpu[:, c] != 0
        if not sel.any():
            continue
        theta = X_gpu[sel, c].min()
        err = np.abs(X_gpu[sel, c] - Xp[sel, c]) / np.maximum(np.maximum(np.abs(Xp[sel, c]), row_scale[sel]), theta)
        worst = max(worst, float(err.max()))
    return worst
