"""Helpers of the GPU tests (host side only)."""
import numpy as np

import paper_2207_07615_amd as plss


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def matrix(h, A, storage="f64"):
    return plss.Matrix(h, A.row_ptr, A.col_idx, A.vals, shape=(A.m, A.n), storage=storage)


def csr_from_dense(D):
    import scipy.sparse as sp
    S = sp.csr_matrix(D)
    S.sort_indices()
    return S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.astype(np.float64)
