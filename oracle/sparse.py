"""Sparse-matrix helpers of the oracle (test infrastructure only).

The products use SciPy's CSR routines as library primitives: row i of A·v is
summed over the row's stored entries in storage order.  The transpose is the
plain definition of CSC: entries ordered by (column, row).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class CSRError(ValueError):
    pass


def validate_csr(m, n, row_ptr, col_idx, vals):
    """Raise CSRError if (row_ptr, col_idx, vals) is not a well-formed CSR
    matrix of shape m x n with ascending, distinct, in-range column indices
    within each row and finite values."""
    row_ptr = np.asarray(row_ptr)
    col_idx = np.asarray(col_idx)
    vals = np.asarray(vals)
    if m <= 0 or n <= 0:
        raise CSRError("m and n must be positive")
    if row_ptr.shape != (m + 1,):
        raise CSRError("row_ptr must have m+1 entries")
    if row_ptr[0] != 0:
        raise CSRError("row_ptr[0] must be 0")
    if np.any(np.diff(row_ptr) < 0):
        raise CSRError("row_ptr must be non-decreasing")
    nnz = int(row_ptr[-1])
    if col_idx.shape != (nnz,) or vals.shape != (nnz,):
        raise CSRError("col_idx and vals must have row_ptr[m] entries")
    if nnz and (col_idx.min() < 0 or col_idx.max() >= n):
        raise CSRError("column index out of range")
    if not np.all(np.isfinite(vals)):
        raise CSRError("non-finite value")
    # ascending and distinct within each row: consecutive entries of the same
    # row must strictly increase
    if nnz > 1:
        same_row = np.ones(nnz - 1, dtype=bool)
        starts = row_ptr[1:-1]
        starts = starts[(starts > 0) & (starts < nnz)]
        same_row[starts - 1] = False
        if np.any(np.diff(col_idx.astype(np.int64))[same_row] <= 0):
            raise CSRError("column indices must be ascending and distinct within a row")


def as_scipy(m, n, row_ptr, col_idx, vals) -> sp.csr_matrix:
    return sp.csr_matrix((np.asarray(vals, dtype=np.float64), col_idx, row_ptr), shape=(m, n))


def matvec(S: sp.csr_matrix, v: np.ndarray) -> np.ndarray:
    """A·v (float64)."""
    return S @ v


def rmatvec(S: sp.csr_matrix, v: np.ndarray) -> np.ndarray:
    """Aᵀ·v (float64)."""
    return S.T @ v


def residual_pair(S: sp.csr_matrix, p: np.ndarray, r: np.ndarray):
    """The two matrix products of one iteration of Algorithm 1 (Section 5),
    in the algorithm's order: the residual update r <- r - A p, then
    y = Aᵀ r with the updated residual, and the squared norms of both
    (rho = ||r||², phi = yᵀ y, i.e. W = I).  Returns (r, y, rho, phi); the
    input r is not modified."""
    r_new = np.asarray(r, dtype=np.float64) - matvec(S, np.asarray(p, dtype=np.float64))
    y = rmatvec(S, r_new)
    return r_new, y, float(r_new @ r_new), float(y @ y)


def csr_to_csc(m, n, row_ptr, col_idx, vals):
    """Transpose storage: CSC of A with rows ascending inside every column.

    Definition: the CSC lists the stored entries of A sorted by (column, row).
    Since CSR lists them sorted by (row, column), a stable sort on the column
    index alone yields that order.  Returns (col_ptr int64[n+1], row_idx
    int32[nnz], vals[nnz] in the input dtype)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx)
    rows = np.repeat(np.arange(m, dtype=np.int32), np.diff(row_ptr))
    order = np.argsort(col_idx, kind="stable")
    counts = np.bincount(col_idx, minlength=n).astype(np.int64)
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=col_ptr[1:])
    return col_ptr, rows[order], np.asarray(vals)[order]
