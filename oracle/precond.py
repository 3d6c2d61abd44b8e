"""Diagonal preconditioners M = C C^dagger of Sec. II.

* identity ("id", no preconditioner);
* Jacobi: M = diag(|a_ii - sigma|), assumes a_ii != sigma;
* row norm (the row-norm preconditioner of Sec. II): M = diag(r_i) with r_i the
  2-norm of row i of A - sigma I.

The row norms are taken straight from the stored sparse rows, as defined.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def shifted(A, sigma: float):
    n = A.shape[0]
    if sp.issparse(A):
        return (A - sigma * sp.identity(n, format="csr")).tocsr()
    return A - sigma * np.eye(n)


def row_norm_diagonal(A, sigma: float) -> np.ndarray:
    """r_i = sqrt(|a_ii - sigma|^2 + sum_{k != i} |a_ik|^2)."""
    B = shifted(A, sigma)
    if sp.issparse(B):
        return np.sqrt(np.asarray(B.multiply(B).sum(axis=1)).ravel())
    return np.sqrt((np.abs(B) ** 2).sum(axis=1))


def jacobi_diagonal(A, sigma: float) -> np.ndarray:
    d = A.diagonal() if sp.issparse(A) else np.diag(A)
    return np.abs(d - sigma)


def preconditioner_diagonal(A, sigma: float, kind: str) -> np.ndarray:
    if kind == "row":
        return row_norm_diagonal(A, sigma)
    if kind == "jacobi":
        return jacobi_diagonal(A, sigma)
    if kind == "id":
        return np.ones(A.shape[0])
    raise ValueError(kind)
