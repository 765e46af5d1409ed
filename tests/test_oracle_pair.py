"""Pins of the oracle's residual pair (the two products of one iteration of
Algorithm 1: r <- r - A p, then y = Aᵀ r with the updated r, and their squared
norms), independent of the SciPy routines it calls:

* a hand-worked 2 x 3 example with every intermediate written out;
* exact rational arithmetic (Fractions, plain loops) on small integer systems,
  where float64 is exact, so the oracle must match bit for bit;
* the closed form y_new = y_old - AᵀA p on dense copies (NumPy dense products,
  not the sparse routines), which fails if y is formed from the old residual.
"""
from fractions import Fraction

import numpy as np
import pytest

import plss_inputs as gen
from oracle import sparse as osp


def test_hand_worked_2x3():
    # A = [[1, 0, 2], [0, -3, 1]], p = (1, 1, 1), r = (4, 1)
    #   A p     = (3, -2)          r_new = r - A p = (1, 3)
    #   y       = Aᵀ r_new = (1*1 + 0*3, 0*1 - 3*3, 2*1 + 1*3) = (1, -9, 5)
    #   rho     = 1 + 9 = 10       phi = 1 + 81 + 25 = 107
    S = osp.as_scipy(2, 3, np.array([0, 2, 4]), np.array([0, 2, 1, 2]), np.array([1.0, 2.0, -3.0, 1.0]))
    r_in = np.array([4.0, 1.0])
    r, y, rho, phi = osp.residual_pair(S, np.ones(3), r_in)
    np.testing.assert_array_equal(r, [1.0, 3.0])
    np.testing.assert_array_equal(y, [1.0, -9.0, 5.0])
    assert rho == 10.0 and phi == 107.0
    np.testing.assert_array_equal(r_in, [4.0, 1.0])  # the input is left alone


def _exact(m, n, row_ptr, col_idx, vals, p, r):
    """Plain-loop rational evaluation of the same definition."""
    rn = [Fraction(int(r[i])) for i in range(m)]
    for i in range(m):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            rn[i] -= Fraction(int(vals[e])) * Fraction(int(p[col_idx[e]]))
    y = [Fraction(0)] * n
    for i in range(m):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            y[col_idx[e]] += Fraction(int(vals[e])) * rn[i]
    return rn, y, sum(v * v for v in rn), sum(v * v for v in y)


@pytest.mark.parametrize("seed,m,n", [(1, 7, 5), (2, 5, 9), (3, 12, 12), (4, 1, 6), (5, 6, 1)])
def test_exact_rational(seed, m, n):
    rng = np.random.default_rng(seed)
    L = rng.integers(0, n + 1, size=m)
    L[0] = 0  # an empty row
    row_ptr = np.concatenate([[0], np.cumsum(L)])
    col_idx = np.concatenate([np.sort(rng.choice(n, size=k, replace=False)) for k in L]).astype(np.int64) \
        if row_ptr[-1] else np.zeros(0, dtype=np.int64)
    vals = rng.integers(-5, 6, size=row_ptr[-1]).astype(np.float64)
    p = rng.integers(-4, 5, size=n).astype(np.float64)
    r0 = rng.integers(-9, 10, size=m).astype(np.float64)
    S = osp.as_scipy(m, n, row_ptr, col_idx, vals)
    r, y, rho, phi = osp.residual_pair(S, p, r0)
    er, ey, erho, ephi = _exact(m, n, row_ptr, col_idx, vals, p, r0)
    assert [Fraction(v) for v in r] == er
    assert [Fraction(v) for v in y] == ey
    assert Fraction(rho) == erho and Fraction(phi) == ephi


def test_closed_form_gram_update():
    """y_new = Aᵀ r_new = Aᵀ r - AᵀA p (dense NumPy on both sides)."""
    A = gen.small(m=300, n=120).A
    S = A.scipy()
    D = S.toarray()
    rng = np.random.default_rng(7)
    p = rng.standard_normal(A.n)
    r0 = rng.standard_normal(A.m)
    r, y, rho, phi = osp.residual_pair(S, p, r0)
    y_old = D.T @ r0
    want = y_old - D.T @ (D @ p)
    assert np.max(np.abs(y - want)) <= 1e-12 * np.max(np.abs(D).T @ (np.abs(r0) + np.abs(D) @ np.abs(p)))
    assert abs(rho - float(np.dot(r0 - D @ p, r0 - D @ p))) <= 1e-12 * rho
    assert abs(phi - float(np.dot(want, want))) <= 1e-11 * phi
