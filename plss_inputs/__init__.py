"""Seeded synthetic inputs for PLSS (consistent sparse systems A x = b).

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
no arithmetic of the solver: it only draws matrices, solutions and sketch
orders from NumPy's PCG64 generator, and forms the consistent right-hand side
``b = A x*`` with SciPy's sparse product (a library routine, not solver code).

All matrices are CSR with int64 ``row_ptr``, int32 ``col_idx`` (distinct and
ascending within each row) and float64 ``vals``.

Workload recipes (the paper's own test sets are SuiteSparse / LIBSVM matrices
that are not available here; these synthetic recipes stand in for them, with
the shape classes of Tables 1-4 of the paper):

* ``small``      2000 x 1000, exactly 8 nnz per row, N(0,1) values.
* ``large``      2,000,000 x 500,000, row lengths Zipf(1.5) clipped to
                 [2, 2000] (realised mean ~68), N(0,1) values.
* ``underdet``   200,000 x 1,000,000, 30 nnz per row, U(-1,1) values, with a
                 seeded row permutation for identity sketch columns.
* ``batch``      256 systems, m log-uniform in [1e3, 2e5], n = m*U(0.5,1),
                 row lengths uniform in [5, 50]; plus a shared 500,000 x
                 250,000 matrix with 20 nnz per row and 32 right-hand sides.
* ``stream``     served systems, m log-uniform in [1e3, 1e6], n/m in
                 U(0.3, 1), row lengths Zipf(1.5) clipped to [1, 100].
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.sparse as sp

SEED_BASE = 761500


@dataclasses.dataclass
class CSR:
    """A sparse matrix in CSR form (host arrays)."""

    m: int
    n: int
    row_ptr: np.ndarray  # int64, m+1
    col_idx: np.ndarray  # int32, nnz
    vals: np.ndarray     # float64 (or float32 for reduced storage), nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.vals.astype(np.float64), self.col_idx, self.row_ptr),
                             shape=(self.m, self.n))

    def dense(self) -> np.ndarray:
        return self.scipy().toarray()

    def astype(self, dtype) -> "CSR":
        return CSR(self.m, self.n, self.row_ptr, self.col_idx, self.vals.astype(dtype))


@dataclasses.dataclass
class System:
    """A consistent system: A, b = A x*, the generating x* and a row order."""

    A: CSR
    b: np.ndarray
    xstar: np.ndarray
    perm: Optional[np.ndarray] = None  # int32 row permutation for identity sketches
    tol: float = 1e-8


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def distinct_sorted_columns(rng: np.random.Generator, row_len: np.ndarray, n: int):
    """Draw, per row, ``row_len[i]`` distinct column indices uniform in [0, n),
    returned ascending within each row.  Returns (row_ptr int64, col_idx int32).

    Duplicates inside a row are redrawn until none remain (sampling without
    replacement)."""
    row_len = np.asarray(row_len, dtype=np.int64)
    if np.any(row_len > n):
        raise ValueError("row length exceeds the number of columns")
    m = row_len.shape[0]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(row_len, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    rows = np.repeat(np.arange(m, dtype=np.int64), row_len)
    key = rows * n + rng.integers(0, n, size=nnz, dtype=np.int64)
    while True:
        key.sort()
        dup = np.zeros(nnz, dtype=bool)
        if nnz > 1:
            dup[1:] = key[1:] == key[:-1]
        nd = int(dup.sum())
        if nd == 0:
            break
        key[dup] = rows[dup] * n + rng.integers(0, n, size=nd, dtype=np.int64)
    col = (key - rows * n).astype(np.int32)
    return row_ptr, col


def make_csr(rng, m, n, row_len, value_dist="normal") -> CSR:
    row_ptr, col = distinct_sorted_columns(rng, row_len, n)
    nnz = int(row_ptr[-1])
    if value_dist == "normal":
        vals = rng.standard_normal(nnz)
    elif value_dist == "uniform":
        vals = rng.uniform(-1.0, 1.0, nnz)
    elif value_dist == "int":
        # nonzero integers in {-3..-1, 1..3}
        mag = rng.integers(1, 4, size=nnz)
        sgn = rng.integers(0, 2, size=nnz) * 2 - 1
        vals = (mag * sgn).astype(np.float64)
    else:
        raise ValueError(value_dist)
    return CSR(m, n, row_ptr, col, vals.astype(np.float64))


def rhs(A: CSR, xstar: np.ndarray) -> np.ndarray:
    """b = A x* in float64 (library sparse product; A's stored values are
    widened to float64 first, so a float32-stored A gives b in range(A))."""
    return A.scipy() @ np.asarray(xstar, dtype=np.float64)


def zipf_lengths(rng, m, s, lo, hi, n):
    L = rng.zipf(s, size=m).astype(np.int64)
    return np.clip(L, lo, min(hi, n))


def consistent(rng, A: CSR, tol=1e-8, perm=False) -> System:
    xstar = rng.standard_normal(A.n)
    b = rhs(A, xstar)
    p = rng.permutation(A.m).astype(np.int32) if perm else None
    return System(A, b, xstar, p, tol)


# --------------------------------------------------------------------------
# Workload recipes
# --------------------------------------------------------------------------

def small(seed: int = SEED_BASE + 1, m: int = 2000, n: int = 1000, L: int = 8,
          storage=np.float64) -> System:
    """2000 x 1000, exactly 8 nnz per row, N(0,1) values, x* ~ N(0,1)."""
    rng = rng_for(seed)
    A = make_csr(rng, m, n, np.full(m, L, dtype=np.int64), "normal")
    A = A.astype(storage)
    return consistent(rng, A, 1e-8)


def large(seed: int = SEED_BASE + 2, m: int = 2_000_000, n: int = 500_000,
          storage=np.float64) -> System:
    """Zipf(1.5) row lengths clipped to [2, 2000], N(0,1), columns uniform."""
    rng = rng_for(seed)
    L = zipf_lengths(rng, m, 1.5, 2, 2000, n)
    A = make_csr(rng, m, n, L, "normal").astype(storage)
    return consistent(rng, A, 1e-8)


def underdet(seed: int = SEED_BASE + 3, m: int = 200_000, n: int = 1_000_000,
             L: int = 30) -> System:
    """Underdetermined, 30 nnz per row, U(-1,1) values, seeded row order."""
    rng = rng_for(seed)
    A = make_csr(rng, m, n, np.full(m, min(L, n), dtype=np.int64), "uniform")
    return consistent(rng, A, 1e-8, perm=True)


def batch_systems(count: int = 256, seed: int = SEED_BASE + 4, m_lo=1e3, m_hi=2e5,
                  storage=np.float64, first: int = 0):
    """Independent uneven systems (each from its own spawned stream)."""
    ss = np.random.SeedSequence(seed).spawn(first + count)[first:]
    out = []
    for s in ss:
        rng = np.random.Generator(np.random.PCG64(s))
        m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        n = max(1, int(round(m * rng.uniform(0.5, 1.0))))
        L = rng.integers(5, 51, size=m)
        L = np.minimum(L, n)
        A = make_csr(rng, m, n, L, "normal").astype(storage)
        out.append(consistent(rng, A, 1e-8))
    return out


def shared_multi_rhs(seed: int = SEED_BASE + 5, m: int = 500_000, n: int = 250_000,
                     L: int = 20, nrhs: int = 32, storage=np.float64):
    """One matrix with an (n x nrhs) N(0,1) solution block; B = A X*
    (column-major: column j is contiguous)."""
    rng = rng_for(seed)
    A = make_csr(rng, m, n, np.full(m, L, dtype=np.int64), "normal").astype(storage)
    X = rng.standard_normal((nrhs, n))          # row j = solution j
    S = A.scipy()
    B = np.stack([S @ X[j] for j in range(nrhs)])  # nrhs x m
    return A, B, X


def stream_systems(count: int = 10_000, seed: int = SEED_BASE + 6, first: int = 0,
                   m_lo=1e3, m_hi=1e6, storage=np.float64):
    """Served request stream: log-uniform rows, n/m in U(0.3,1), Zipf rows,
    per-request tolerance 1e-6 or 1e-10 with equal probability."""
    ss = np.random.SeedSequence(seed).spawn(first + count)[first:]
    out = []
    for s in ss:
        rng = np.random.Generator(np.random.PCG64(s))
        m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        n = max(1, int(round(m * rng.uniform(0.3, 1.0))))
        L = zipf_lengths(rng, m, 1.5, 1, 100, n)
        A = make_csr(rng, m, n, L, "normal").astype(storage)
        tol = 1e-6 if rng.random() < 0.5 else 1e-10
        out.append(consistent(rng, A, tol))
    return out


def poisson_arrivals(count: int, rate: float, seed: int = SEED_BASE + 7) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = rng_for(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def tiny(seed: int, m: int, n: int, L: int, value_dist="normal") -> System:
    """Small consistent systems for pins and edge cases."""
    rng = rng_for(seed)
    A = make_csr(rng, m, n, np.full(m, min(L, n), dtype=np.int64), value_dist)
    return consistent(rng, A, 1e-12, perm=True)


def tiny_integer(seed: int, m: int, n: int, L: int):
    """Small integer-valued A and integer x* (for exact rational runs)."""
    rng = rng_for(seed)
    A = make_csr(rng, m, n, np.full(m, min(L, n), dtype=np.int64), "int")
    xstar = rng.integers(-3, 4, size=n).astype(np.float64)
    b = rhs(A, xstar)
    return System(A, b, xstar, rng.permutation(m).astype(np.int32), 0.0)
