"""Rational-arithmetic twin of the oracle (test infrastructure only).

Runs Algorithm 1 and the one-column sketch step in exact arithmetic
(``fractions.Fraction``) on small dense integer systems, so the finite
termination of Theorem 1 / Corollaries 1-2 and the orthogonality of residuals
and updates (Sections 2.1, 2.5, 4) can be checked as exact equalities.

Algorithm 1's beta and gamma involve sqrt(theta*phi); their product forms
need no square root:
  beta  = 1/((s-1)(s+1)) with s^2 = theta*phi/rho^2  ->  rho^2/(theta*phi - rho^2)
  gamma = (theta/rho)*beta                           ->  theta*rho/(theta*phi - rho^2)
Likewise the column step's delta = (||y||-||d||)(||y||+||d||) = yᵀy - dᵀd.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence

Vec = List[Fraction]
Mat = List[List[Fraction]]


def F(x) -> Fraction:
    return Fraction(int(x)) if float(x).is_integer() else Fraction(x)


def mat(A) -> Mat:
    return [[F(v) for v in row] for row in A]


def vec(v) -> Vec:
    return [F(x) for x in v]


def dot(a: Sequence[Fraction], b: Sequence[Fraction]) -> Fraction:
    return sum((x * y for x, y in zip(a, b)), Fraction(0))


def mv(A: Mat, v: Vec) -> Vec:
    return [dot(row, v) for row in A]


def mtv(A: Mat, v: Vec) -> Vec:
    n = len(A[0])
    return [sum((A[i][j] * v[i] for i in range(len(A))), Fraction(0)) for j in range(n)]


def axpy(a: Fraction, x: Vec, y: Vec) -> Vec:
    return [a * xi + yi for xi, yi in zip(x, y)]


def plss_residual_exact(A, b, maxit=None):
    """Algorithm 1 with W = I in rationals, run until r = 0 exactly.
    Returns (x, residuals r_0.., updates p_1..)."""
    A = mat(A); b = vec(b)
    m, n = len(A), len(A[0])
    maxit = maxit or (min(m, n) + 1)
    x = [Fraction(0)] * n
    r = list(b)
    rs, ps = [list(r)], []
    rho = dot(r, r)
    if rho == 0:
        return x, rs, ps
    y = mtv(A, r)
    phi = dot(y, y)
    p = [(rho / phi) * yi for yi in y]
    theta = dot(p, p)
    x = axpy(Fraction(1), p, x)
    ps.append(p)
    for _ in range(maxit):
        r = axpy(Fraction(-1), mv(A, p), r)
        rs.append(r)
        rho = dot(r, r)
        if rho == 0:
            break
        y = mtv(A, r)
        phi = dot(y, y)
        den = theta * phi - rho * rho
        beta = rho * rho / den
        gamma = theta * rho / den
        p = [beta * pi + gamma * yi for pi, yi in zip(p, y)]
        theta = dot(p, p)
        x = axpy(Fraction(1), p, x)
        ps.append(p)
    return x, rs, ps


def plss_columns_exact(A, b, columns, used=None):
    """One-column sketch steps in rationals.  ``columns`` is a list of
    ('r',) or ('e', i).  A column with sigma == 0 (the update would be zero)
    or delta == 0 (y_k in the span of the stored updates, so appending it
    would leave Y_k rank deficient, against eq. seqS) is skipped.  Returns
    (x, residuals, updates); the columns that produced an update are appended
    to ``used`` when given."""
    A = mat(A); b = vec(b)
    m, n = len(A), len(A[0])
    x = [Fraction(0)] * n
    r = list(b)
    P: List[Vec] = []
    AP: List[Vec] = []
    Th: List[Fraction] = []
    rs, ps = [list(r)], []
    for col in columns:
        if dot(r, r) == 0:
            break
        if col[0] == "r":
            y = mtv(A, r)
            w = [dot(ap, r) for ap in AP]
            sigma = dot(r, r)
        else:
            i = col[1]
            y = list(A[i])
            w = [ap[i] for ap in AP]
            sigma = r[i]
        c = [wj / tj for wj, tj in zip(w, Th)]
        q = list(y)
        for cj, pj in zip(c, P):
            q = axpy(-cj, pj, q)
        delta = dot(y, y) - sum((wj * wj / tj for wj, tj in zip(w, Th)), Fraction(0))
        if sigma == 0 or delta == 0:
            continue
        p = [(sigma / delta) * qi for qi in q]
        Ap = mv(A, p)
        r = axpy(Fraction(-1), Ap, r)
        x = axpy(Fraction(1), p, x)
        P.append(p); AP.append(Ap); Th.append(dot(p, p))
        rs.append(r); ps.append(p)
        if used is not None:
            used.append(tuple(col))
    return x, rs, ps


def solve_exact(M: Mat, rhs: Vec) -> Vec:
    """Gauss-Jordan elimination in rationals for a nonsingular square M."""
    k = len(M)
    aug = [list(M[i]) + [rhs[i]] for i in range(k)]
    for c in range(k):
        piv = next(i for i in range(c, k) if aug[i][c] != 0)
        aug[c], aug[piv] = aug[piv], aug[c]
        pv = aug[c][c]
        aug[c] = [v / pv for v in aug[c]]
        for i in range(k):
            if i != c and aug[i][c] != 0:
                f = aug[i][c]
                aug[i] = [vi - f * vc for vi, vc in zip(aug[i], aug[c])]
    return [aug[i][k] for i in range(k)]


def min_norm_exact(A, b) -> Vec:
    """A†b in rationals for a full-row-rank A (m <= n): Aᵀ (A Aᵀ)^{-1} b;
    for a full-column-rank A (m >= n) with consistent b: (AᵀA)^{-1} Aᵀ b."""
    A = mat(A); b = vec(b)
    m, n = len(A), len(A[0])
    if m <= n:
        AAt = [[dot(A[i], A[j]) for j in range(m)] for i in range(m)]
        z = solve_exact(AAt, b)
        return mtv(A, z)
    AtA = [[sum((A[i][a] * A[i][c] for i in range(m)), Fraction(0)) for c in range(n)]
           for a in range(n)]
    return solve_exact(AtA, mtv(A, b))


def plss_blocks_exact(A, b, blocks, used=None):
    """Block sketch steps in rationals (the block form of the triangular
    update of Section 2.4, as ``oracle.blocks``).  ``blocks`` is a list of
    lists of columns ('r',) / ('e', i), or ('clear',) to empty the history.
    In block order, a column whose Schur-complement pivot is exactly zero
    (y_j in the span of the history and the block's earlier kept columns) is
    left out; a step with no kept column is not an update.  Returns (x,
    residuals, updates); the kept columns of each update go to ``used``."""
    A = mat(A); b = vec(b)
    m, n = len(A), len(A[0])
    x = [Fraction(0)] * n
    r = list(b)
    Y: List[Vec] = []          # history columns y_j (each length n)
    N: Mat = []                # (Yᵀ Y)^{-1}
    rs, ps = [list(r)], []
    for blk in blocks:
        if blk == ("clear",):
            Y, N = [], []
            continue
        if dot(r, r) == 0:
            break
        ynew, sig = [], []
        for col in blk:
            if col[0] == "r":
                ynew.append(mtv(A, r)); sig.append(dot(r, r))
            else:
                ynew.append(list(A[col[1]])); sig.append(r[col[1]])
        w, K = len(blk), len(Y)
        G = [[dot(Y[a], ynew[j]) for j in range(w)] for a in range(K)]          # Yᵀ Y_new
        T = [[sum((N[a][c] * G[c][j] for c in range(K)), Fraction(0)) for j in range(w)] for a in range(K)]
        D = [[dot(ynew[a], ynew[j]) - sum((G[c][a] * T[c][j] for c in range(K)), Fraction(0))
              for j in range(w)] for a in range(w)]
        keep = []
        for j in range(w):
            if keep:
                Dk = [[D[a][c] for c in keep] for a in keep]
                z = solve_exact(Dk, [D[a][j] for a in keep])
                piv = D[j][j] - sum((D[j][a] * za for a, za in zip(keep, z)), Fraction(0))
            else:
                piv = D[j][j]
            if piv != 0:
                keep.append(j)
        if not keep:
            continue
        kw = len(keep)
        Dk = [[D[a][c] for c in keep] for a in keep]
        # Delta^{-1} column by column
        Dinv_cols = [solve_exact(Dk, [Fraction(int(i == j)) for i in range(kw)]) for j in range(kw)]
        Dinv = [[Dinv_cols[c][a] for c in range(kw)] for a in range(kw)]
        c = [sum((Dinv[a][q] * sig[keep[q]] for q in range(kw)), Fraction(0)) for a in range(kw)]
        Tk = [[T[a][j] for j in keep] for a in range(K)]
        # q_j = y_j - Y T_hat_j, p = Σ_j c_j q_j
        p = [Fraction(0)] * n
        for q_i, j in enumerate(keep):
            qv = list(ynew[j])
            for a in range(K):
                qv = axpy(-Tk[a][q_i], Y[a], qv)
            p = axpy(c[q_i], qv, p)
        r = axpy(Fraction(-1), mv(A, p), r)
        x = axpy(Fraction(1), p, x)
        # N_k = [[N + T D^-1 Tᵀ, -T D^-1], [-D^-1 Tᵀ, D^-1]]
        TD = [[sum((Tk[a][q] * Dinv[q][j] for q in range(kw)), Fraction(0)) for j in range(kw)] for a in range(K)]
        newN = [[N[a][c2] + sum((TD[a][q] * Tk[c2][q] for q in range(kw)), Fraction(0)) for c2 in range(K)]
                + [-TD[a][j] for j in range(kw)] for a in range(K)]
        for q in range(kw):
            newN.append([-TD[c2][q] for c2 in range(K)] + [Dinv[q][j] for j in range(kw)])
        N = newN
        Y = Y + [ynew[j] for j in keep]
        rs.append(r); ps.append(p)
        if used is not None:
            used.append([tuple(blk[j]) for j in keep])
    return x, rs, ps
