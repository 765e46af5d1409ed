"""Independent reference routines the oracle is pinned to (test
infrastructure only).  None of them shares code with ``oracle.plss``.

* ``pk_bruteforce``  eq. (pkLong) evaluated densely for an explicit sketch.
* ``craig``          Craig's method via Golub-Kahan bidiagonalisation, in the
                     form given in Section 6 (eqs. bidiag1-2, craigRes):
                     beta_1 u_1 = b, alpha_1 v_1 = Aᵀu_1,
                     beta_{k+1} u_{k+1} = A v_k - alpha_k u_k,
                     alpha_{k+1} v_{k+1} = Aᵀu_{k+1} - beta_{k+1} v_k,
                     zeta_k = -(beta_k/alpha_k) zeta_{k-1} (zeta_0 = -1),
                     x_k = x_{k-1} + zeta_k v_k.
* ``kaczmarz``       textbook Kaczmarz projections
                     x <- x + (b_i - a_iᵀx)/||a_i||^2 a_i (Section 7).
* ``min_norm``       the dense minimum-norm solution A†b (SVD based lstsq).
"""
from __future__ import annotations

import numpy as np


def pk_bruteforce(A, S, r, W=None):
    """p = W Aᵀ S (Sᵀ A W Aᵀ S)^† Sᵀ r  (eq. pkLong; pseudo-inverse as the
    paper prescribes when the inverse does not exist)."""
    A = np.asarray(A, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    if S.ndim == 1:
        S = S[:, None]
    n = A.shape[1]
    W = np.eye(n) if W is None else np.asarray(W, dtype=np.float64)
    Y = A.T @ S
    G = Y.T @ W @ Y
    return W @ Y @ (np.linalg.pinv(G) @ (S.T @ r))


def x_bruteforce(A, S, b, x0=None):
    """Closed form of the iterate after the sketch S (W = I): since the
    iterates are nested projections, x_k = x0 + Aᵀ S (Sᵀ A Aᵀ S)^† Sᵀ (b - A x0)."""
    A = np.asarray(A, dtype=np.float64)
    x0 = np.zeros(A.shape[1]) if x0 is None else x0
    return x0 + pk_bruteforce(A, S, b - A @ x0)


def craig(A, b, iters):
    """Iterates x_1..x_iters of Craig's method (no reorthogonalisation)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    beta = np.linalg.norm(b)
    u = b / beta
    v = A.T @ u
    alpha = np.linalg.norm(v)
    v = v / alpha
    zeta = beta / alpha          # zeta_1 = -(beta_1/alpha_1) * zeta_0, zeta_0 = -1
    x = zeta * v
    xs = [x.copy()]
    for _ in range(iters - 1):
        uu = A @ v - alpha * u
        beta = np.linalg.norm(uu)
        u = uu / beta
        vv = A.T @ u - beta * v
        alpha = np.linalg.norm(vv)
        v = vv / alpha
        zeta = -(beta / alpha) * zeta
        x = x + zeta * v
        xs.append(x.copy())
    return xs


def kaczmarz(A, b, order, x0=None):
    """One Kaczmarz projection per entry of ``order``; returns all iterates."""
    A = np.asarray(A, dtype=np.float64)
    x = np.zeros(A.shape[1]) if x0 is None else np.array(x0, dtype=np.float64)
    xs = []
    for i in order:
        a = A[i]
        x = x + ((b[i] - a @ x) / (a @ a)) * a
        xs.append(x.copy())
    return xs


def min_norm(A, b):
    A = np.asarray(A, dtype=np.float64)
    return np.linalg.lstsq(A, b, rcond=None)[0]
