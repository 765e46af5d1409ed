"""PLSS oracle: Algorithm 1 and the general one-column sketch step, float64.

Test infrastructure only.  Written from the paper:

* ``plss_residual`` follows Algorithm 1 (Section 5) line by line in the
  paper's notation (r, y, rho, WIy, phi, beta, gamma, p, theta, x), with the
  stopping rule stated after the algorithm (sqrt(rho)/||b|| below tau).
* ``plss_columns`` is the general update for a sketch grown by one column per
  step: with S_{k-1}ᵀ r_{k-1} = 0 (eq. orthSr) the update of eq. (pkLong) is
  p_k = sigma * Y_k (Y_kᵀY_k)^{-1} e_k, sigma = s_kᵀ r_{k-1}, and by the
  orthogonality of the updates (Section 2.5) and their representation as a
  combination of previous updates and y_k (Section 2.6) this is
  p_k = (sigma/delta) (y_k - P Θ^{-1} Pᵀ y_k),
  delta = (||y_k|| - ||d||)(||y_k|| + ||d||), d = Θ^{-1/2} Pᵀ y_k.
  Pᵀ y_k = (A P)ᵀ s_k is read from the stored products A p_j (Section 7's
  storage scheme).  For identity columns s_k = e_i this is eq. (pkKacz).

Readings (where the paper is silent or inconsistent):

* gamma: Algorithm 1's gamma = (theta/rho)*beta, i.e. theta*rho/(theta*phi -
  rho^2).  The closed forms printed with Theorem 2 and with the W-variant
  lack a factor rho; only Algorithm 1's form keeps successive residuals and
  updates orthogonal (checked exactly in rationals by the tests).
* k counts applied updates; k = 1 after the initial step; at most maxit
  updates are applied.
* The stop test is ``sqrt(rho) <= tol * ||b||`` (or ``<= tol`` when
  absolute), taken right after each rho is formed, including before the
  first step; b = 0 returns x0 after 0 updates.
* x0 = 0 unless given (the experiments' choice).
* Breakdown: phi == 0 or not (sqrt(theta*phi)/rho > 1) returns the last
  iterate with status BREAKDOWN (only possible when b is not in range(A) in
  exact arithmetic).
* The residual is updated recursively as in Algorithm 1 and the stop test
  uses it; the true relative residual ||b - A x||/||b|| is reported once at
  exit.
* Identity columns: sampled without replacement from a given row order; the
  order is reused cyclically.  After every full pass through the m rows the
  stored history (P, AP, Θ) is cleared.  A column with r_i == 0 or
  delta <= 1e-14 * ||a_i||^2 is skipped (left out of the sketch); a skipped
  column is not an update.
* Mixed sketch: the columns r_{k-1}, e_{π0}, r, e_{π1}, ... alternate, one
  row per residual column; every column is one step of ``plss_columns``.
* The history is also cleared when it holds ``hist_cap`` updates (a memory
  bound; default min(m, n)).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterable, List, Optional

import numpy as np
import scipy.sparse as sp

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


@dataclasses.dataclass
class Result:
    x: np.ndarray
    iters: int
    hist: List[float]          # sqrt(rho_k)/||b|| for k = 0..iters (recursive residual)
    status: int
    relres_true: float
    xs: Optional[list] = None  # iterates x_0..x_k when recorded
    ps: Optional[list] = None  # updates p_1..p_k when recorded
    rs: Optional[list] = None  # residuals r_0..r_k when recorded
    columns: Optional[list] = None  # sketch columns actually used, ('r',) or ('e', i)


def _as_sparse(A) -> sp.csr_matrix:
    if sp.issparse(A):
        return sp.csr_matrix(A, dtype=np.float64)
    if hasattr(A, "scipy"):
        return A.scipy()
    return sp.csr_matrix(np.asarray(A, dtype=np.float64))


def _relres_true(S, x, b, nb):
    res = np.linalg.norm(b - S @ x)
    return res / nb if nb > 0 else res


def plss_residual(A, b, tol=1e-8, maxit=1000, x0=None, wi=None, tol_absolute=False,
                  record=False, dot=None) -> Result:
    """Algorithm 1 (PLSS) with residual sketch S_k = [r_0 ... r_{k-1}] (eq. S).

    ``wi`` is the diagonal of the optional parameter matrix BᵀB (the inverse of
    W); None means W = I.  ``dot`` replaces the inner product (default
    ``numpy.dot``): runs that differ only in its summation order measure how
    far two equally valid float64 evaluations of Algorithm 1 drift apart."""
    dot = dot or (lambda a, c: float(a @ c))
    S = _as_sparse(A)
    m, n = S.shape
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    thr = tol if tol_absolute else tol * nb
    scale = 1.0 if tol_absolute or nb == 0 else 1.0 / nb
    WI = np.ones(n) if wi is None else np.asarray(wi, dtype=np.float64)

    # Initialisation (Algorithm 1, before the loop)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - S @ x
    rho = dot(r, r)
    hist = [math.sqrt(rho) * scale]
    xs = [x.copy()] if record else None
    ps = [] if record else None
    rs = [r.copy()] if record else None

    def done(status, k):
        return Result(x, k, hist, status, _relres_true(S, x, b, nb), xs, ps, rs)

    if math.sqrt(rho) <= thr:
        return done(OK, 0)
    y = S.T @ r
    WIy = y / WI
    phi = dot(y, WIy)
    if not (phi > 0.0):
        return done(BREAKDOWN, 0)
    p = (rho / phi) * WIy
    theta = dot(p, WI * p)
    x = x + p
    k = 1
    if record:
        xs.append(x.copy()); ps.append(p.copy())

    while True:
        r = r - S @ p
        rho = dot(r, r)
        hist.append(math.sqrt(rho) * scale)
        if record:
            rs.append(r.copy())
        if math.sqrt(rho) <= thr:
            return done(OK, k)
        if k >= maxit:
            return done(NOT_CONVERGED, k)
        y = S.T @ r
        WIy = y / WI
        phi = dot(y, WIy)
        s = math.sqrt(theta * phi) / rho
        if not (s > 1.0):
            return done(BREAKDOWN, k)
        beta = 1.0 / ((s - 1.0) * (s + 1.0))
        gamma = (theta / rho) * beta
        p = beta * p + gamma * WIy
        theta = dot(p, WI * p)
        x = x + p
        k += 1
        if record:
            xs.append(x.copy()); ps.append(p.copy())


def column_sequence(kind: str, m: int, perm=None) -> Iterable[tuple]:
    """Sketch columns: 'residual' -> r, r, ...; 'identity' -> e_{π0}, e_{π1},
    ... cycling through ``perm``; 'mixed' -> r, e_{π0}, r, e_{π1}, ..."""
    if perm is None:
        perm = np.arange(m)
    perm = [int(i) for i in perm]
    if sorted(perm) != list(range(m)):
        raise ValueError("row order must be a permutation of 0..m-1")
    t = 0
    while True:
        i = perm[t % m]
        if kind == "residual":
            yield ("r",)
        elif kind == "identity":
            yield ("e", i, (t % m) == m - 1)
        elif kind == "mixed":
            yield ("r",)
            yield ("e", i, (t % m) == m - 1)
        else:
            raise ValueError(kind)
        t += 1


def plss_columns(A, b, sketch="identity", perm=None, tol=1e-8, maxit=1000,
                 tol_absolute=False, hist_cap=None, max_columns=None,
                 record=False, dot=None) -> Result:
    """PLSS with a sketch grown by one column per step (identity, mixed or
    residual columns), storing P = [p_1..p_k], AP = [A p_1..A p_k] and
    Θ = diag(p_jᵀ p_j) as in Section 7.  W = I.

    ``maxit`` bounds applied updates; ``max_columns`` (default 4*maxit + 4*m)
    bounds columns examined, including skipped ones.  ``dot`` replaces the
    inner product (default ``numpy.dot``), as in ``plss_residual``."""
    dot = dot or (lambda a, c: float(a @ c))
    S = _as_sparse(A)
    m, n = S.shape
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    thr = tol if tol_absolute else tol * nb
    scale = 1.0 if tol_absolute or nb == 0 else 1.0 / nb
    cap = min(m, n) if hist_cap is None else int(hist_cap)
    if max_columns is None:
        max_columns = 4 * maxit + 4 * m

    x = np.zeros(n)
    r = b.copy()
    rho = dot(r, r)
    hist = [math.sqrt(rho) * scale]
    P: List[np.ndarray] = []
    AP: List[np.ndarray] = []
    Theta: List[float] = []
    xs = [x.copy()] if record else None
    ps = [] if record else None
    rs = [r.copy()] if record else None
    used = [] if record else None
    k = 0

    def done(status):
        return Result(x, k, hist, status, _relres_true(S, x, b, nb), xs, ps, rs, used)

    if math.sqrt(rho) <= thr:
        return done(OK)

    for t, col in enumerate(column_sequence(sketch, m, perm)):
        if t >= max_columns:
            return done(NOT_CONVERGED)
        th = np.array(Theta)
        if col[0] == "r":
            y = S.T @ r                                   # y = Aᵀ r
            w = np.array([dot(ap, r) for ap in AP])      # (AP)ᵀ r = Pᵀ y
            sigma = rho                                   # r_{k-1}ᵀ r_{k-1}
        else:
            i = col[1]
            lo, hi = S.indptr[i], S.indptr[i + 1]
            y = np.zeros(n)
            y[S.indices[lo:hi]] = S.data[lo:hi]          # y = Aᵀ e_i = a_i
            w = np.array([ap[i] for ap in AP])           # row i of AP = Pᵀ a_i
            sigma = float(r[i])                          # e_iᵀ r_{k-1}
        c = w / th if len(Theta) else np.zeros(0)
        q = y - (np.column_stack(P) @ c if P else 0.0)
        yy = dot(y, y)
        na = math.sqrt(yy)
        nd = math.sqrt(float(np.sum(w * w / th))) if len(Theta) else 0.0
        delta = (na - nd) * (na + nd)
        bad = sigma == 0.0 or not (delta > 1e-14 * yy)
        if bad:
            if col[0] == "r":
                return done(BREAKDOWN)
            if col[2]:
                P.clear(); AP.clear(); Theta.clear()
            continue
        p = (sigma / delta) * q
        Ap = S @ p
        r = r - Ap
        x = x + p
        P.append(p); AP.append(Ap); Theta.append(dot(p, p))
        k += 1
        rho = dot(r, r)
        hist.append(math.sqrt(rho) * scale)
        if record:
            xs.append(x.copy()); ps.append(p.copy()); rs.append(r.copy()); used.append(col[:2])
        if math.sqrt(rho) <= thr:
            return done(OK)
        if k >= maxit:
            return done(NOT_CONVERGED)
        if (col[0] == "e" and col[2]) or len(Theta) >= cap:
            P.clear(); AP.clear(); Theta.clear()


def plss(A, b, sketch="residual", **kw) -> Result:
    if sketch == "residual":
        kw.pop("perm", None)
        kw.pop("hist_cap", None)
        return plss_residual(A, b, **kw)
    return plss_columns(A, b, sketch=sketch, **kw)
