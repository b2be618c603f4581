"""Comparison helpers for the GPU-vs-oracle parity tests (test code only).

A factor from the GPU and one from the oracle are compared in two parts:
* values: relative Frobenius error over the entries both keep, normalised
  by the oracle factor's norm;
* supports: every entry kept by one side only is a mismatch.  It is a
  near-tie when its pre-selection value lies within ``tol * theta_c`` of the
  oracle's threshold theta_c of that column (the smallest value the oracle
  keeps there; for the whole-matrix rule, the smallest it keeps anywhere);
  otherwise it is a non-tie mismatch.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class FactorDiff:
    rel: float
    mismatches: int
    near_ties: int
    non_ties: int

    def ok(self, tol: float) -> bool:
        return self.rel <= tol and self.non_ties == 0


def compare_factor(X_gpu: np.ndarray, X_or: np.ndarray, Xpre_or: np.ndarray, tol: float = 1e-4,
                   whole: bool = False) -> FactorDiff:
    """``whole``: the factors come from the whole-matrix rule, whose one
    threshold is the smallest value the oracle keeps anywhere."""
    X_gpu = np.asarray(X_gpu, np.float64)
    X_or = np.asarray(X_or, np.float64)
    Xpre = np.where(np.asarray(Xpre_or, np.float64) > 0, Xpre_or, 0.0)
    kg, ko = X_gpu != 0, X_or != 0
    both = kg & ko
    den = np.linalg.norm(X_or)
    rel = float(np.linalg.norm(X_gpu[both] - X_or[both]) / den) if den > 0 else float(np.linalg.norm(X_gpu))
    mism = kg != ko
    near = non = 0
    theta_all = X_or[ko].min() if ko.any() else 0.0
    for c in np.nonzero(mism.any(axis=0))[0]:
        kept = X_or[ko[:, c], c]
        theta = theta_all if whole else (kept.min() if kept.size else 0.0)
        for r in np.nonzero(mism[:, c])[0]:
            v = Xpre[r, c]
            if abs(v - theta) <= tol * max(theta, 1e-300):
                near += 1
            else:
                non += 1
    return FactorDiff(rel, int(mism.sum()), near, non)


def rel_fro(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / d) if d > 0 else float(np.linalg.norm(a))
