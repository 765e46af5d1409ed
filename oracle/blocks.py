"""Block sketches: PLSS with a sketch grown by several columns per step.

Test infrastructure only.  Written from Section 2.4 of the paper (the
triangular factorization: Theorem "simplified inverse" and its Corollary),
taken one block of columns at a time instead of one column.

Notation as in the paper: Y_k = Aᵀ S_k collects y_j = Aᵀ s_j (eq. yk), and
N_k = (Y_kᵀ Y_k)^{-1}.  A step appends a block S_new = [s_1 .. s_w] (m x w)
to the sketch, Y_new = Aᵀ S_new (n x w), and with S_{k-1}ᵀ r_{k-1} = 0
(eq. orthSr) eq. (pkLong) becomes

    T_hat = N_{k-1} Y_{k-1}ᵀ Y_new                      (K x w)
    Delta = Y_newᵀ Y_new - Y_newᵀ Y_{k-1} T_hat          (w x w, Schur complement)
    p_k   = (Y_new - Y_{k-1} T_hat) Delta^{-1} S_newᵀ r_{k-1}
    N_k   = [[N_{k-1} + T_hat Delta^{-1} T_hatᵀ, -T_hat Delta^{-1}],
             [-Delta^{-1} T_hatᵀ,                  Delta^{-1}     ]]

which for w = 1 are the Theorem's t_hat, delta_k and eq. (Nkrec), and the
Corollary's eq. (compute-pk-alpha1).  Then x_k = x_{k-1} + p_k (eq. xko) and
r_k = r_{k-1} - A p_k.

Readings (the paper grows the sketch by one column per step and states no
block rule):

* Block columns: ``residual=True`` puts r_{k-1} first, then ``block``
  identity columns e_i in the given row order (cycled); ``residual=False``
  takes identity columns only.  A block never crosses the end of a pass
  through the rows (the last block of a pass is shorter when block does not
  divide m); the history (Y, N) is cleared after the block that ends a pass,
  as for one-column identity steps.
* A column is kept when its pivot in block order - the Schur complement of
  Delta after the history and the block's earlier kept columns - exceeds
  1e-14 * ||y_j||^2 (the one-column threshold); otherwise it is left out of
  the sketch (it lies in the span already held).  A left-out residual column
  is a breakdown.  sigma_j = e_iᵀ r_{k-1} = 0 alone does not leave a column
  out: in a block it still constrains the update.  A step with no kept
  column is not an update.
* ``iters`` counts updates (block steps with at least one kept column);
  ``maxit`` bounds them.  The history holds at most ``hist_cap`` columns: it
  is cleared before a block that would exceed it (default min(m, n)).
* The stop test is that of Algorithm 1 on the recursive residual, taken
  after every update and before the first step.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from .plss import BREAKDOWN, NOT_CONVERGED, OK, Result, _as_sparse, _relres_true

SKIP_REL = 1e-14


def block_columns(m, block, residual, perm=None):
    """The sketch blocks in order: lists of ('r',) / ('e', i), with a flag
    telling whether the block ends a pass through the rows."""
    if perm is None:
        perm = np.arange(m)
    perm = [int(i) for i in perm]
    if sorted(perm) != list(range(m)):
        raise ValueError("row order must be a permutation of 0..m-1")
    if block < (0 if residual else 1):
        raise ValueError("block size")
    pos = 0
    while True:
        rows = perm[pos:min(pos + block, m)] if block > 0 else []
        pos += len(rows)
        end = pos >= m
        if end:
            pos = 0
        cols = ([("r",)] if residual else []) + [("e", i) for i in rows]
        yield cols, end and block > 0


def plss_blocks(A, b, block=4, residual=False, perm=None, tol=1e-8, maxit=1000,
                tol_absolute=False, hist_cap=None, max_steps=None, record=False, dot=None) -> Result:
    """Block-sketch PLSS (W = I, x0 = 0).  ``dot`` replaces the inner product
    of the Gram entries and rho (default numpy.dot)."""
    dot = dot or (lambda a, c: float(a @ c))
    S = _as_sparse(A)
    m, n = S.shape
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    thr = tol if tol_absolute else tol * nb
    scale = 1.0 if tol_absolute or nb == 0 else 1.0 / nb
    cap = min(m, n) if hist_cap is None else int(hist_cap)
    if max_steps is None:
        max_steps = 4 * maxit + 4 * m
    x = np.zeros(n)
    r = b.copy()
    rho = dot(r, r)
    hist = [math.sqrt(rho) * scale]
    Y = np.zeros((n, 0))
    N = np.zeros((0, 0))
    xs = [x.copy()] if record else None
    ps = [] if record else None
    rs = [r.copy()] if record else None
    used: List = [] if record else None
    k = 0

    def done(status):
        return Result(x, k, hist, status, _relres_true(S, x, b, nb), xs, ps, rs, used)

    if math.sqrt(rho) <= thr:
        return done(OK)
    for t, (cols, pass_end) in enumerate(block_columns(m, block, residual, perm)):
        if t >= max_steps:
            return done(NOT_CONVERGED)
        w = len(cols)
        if Y.shape[1] + w > cap:
            Y = np.zeros((n, 0))
            N = np.zeros((0, 0))
        # Y_new = Aᵀ S_new and sigma = S_newᵀ r_{k-1}
        Ynew = np.zeros((n, w))
        sigma = np.zeros(w)
        for j, c in enumerate(cols):
            if c[0] == "r":
                Ynew[:, j] = S.T @ r
                sigma[j] = rho
            else:
                i = c[1]
                lo, hi = S.indptr[i], S.indptr[i + 1]
                Ynew[S.indices[lo:hi], j] = S.data[lo:hi]
                sigma[j] = r[i]
        K = Y.shape[1]
        G = np.array([[dot(Y[:, a], Ynew[:, j]) for j in range(w)] for a in range(K)]).reshape(K, w)
        That = N @ G
        Delta = np.array([[dot(Ynew[:, a], Ynew[:, j]) for j in range(w)] for a in range(w)]) - G.T @ That
        # columns kept in block order (pivot of the Schur complement)
        keep = []
        for j in range(w):
            yy = Delta[j, j] + (G[:, j] @ That[:, j] if K else 0.0)   # = y_jᵀ y_j
            if keep:
                Dk = Delta[np.ix_(keep, keep)]
                piv = Delta[j, j] - Delta[j, keep] @ np.linalg.solve(Dk, Delta[keep, j])
            else:
                piv = Delta[j, j]
            if piv > SKIP_REL * yy:
                keep.append(j)
            elif cols[j][0] == "r":
                return done(BREAKDOWN)
        if not keep:
            if pass_end:
                Y = np.zeros((n, 0))
                N = np.zeros((0, 0))
            continue
        Dk = Delta[np.ix_(keep, keep)]
        Tk = That[:, keep]
        Yk = Ynew[:, keep]
        c = np.linalg.solve(Dk, sigma[keep])
        p = (Yk - Y @ Tk) @ c
        Ap = S @ p
        r = r - Ap
        x = x + p
        Dinv = np.linalg.inv(Dk)
        N = np.block([[N + Tk @ Dinv @ Tk.T, -Tk @ Dinv], [-Dinv @ Tk.T, Dinv]])
        Y = np.hstack([Y, Yk])
        k += 1
        rho = dot(r, r)
        hist.append(math.sqrt(rho) * scale)
        if record:
            xs.append(x.copy()); ps.append(p.copy()); rs.append(r.copy())
            used.append([cols[j] for j in keep])
        if math.sqrt(rho) <= thr:
            return done(OK)
        if k >= maxit:
            return done(NOT_CONVERGED)
        if pass_end:
            Y = np.zeros((n, 0))
            N = np.zeros((0, 0))
