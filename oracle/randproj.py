"""Randomized projection: the paper's self-contained comparison method.

Test infrastructure only.  Section 8 (Experiments I and III, and the
'Randomized projection' comparison) runs update eq. (pkLong) with W = I and
a sketch S_k in R^{m x r} drawn afresh at every iteration with standard
normal entries: p_k = Aᵀ S_k (S_kᵀ A Aᵀ S_k)^{-1} S_kᵀ r_{k-1}, recomputing
Y_k = Aᵀ S_k, Y_kᵀ Y_k and a solve with it each iteration.

The random numbers come from a counter-based generator written from its
published definition, so that the GPU path can draw the same matrix:

* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
  as easy as 1, 2, 3", SC 2011): a 128-bit counter and a 64-bit key, ten
  rounds; each round multiplies counter words 0 and 2 by the constants
  0xD2511F53 and 0xCD9E8D57 (64-bit products split in high and low words),
  and mixes: (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2),
  hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key is bumped by the Weyl constants
  (0x9E3779B9, 0xBB67AE85) between rounds.
* Uniforms u = (w + 1/2) 2^-32 in (0, 1) from 32-bit words w.
* Box-Muller (1958): z0 = sqrt(-2 ln u0) cos(2 pi u1),
  z1 = sqrt(-2 ln u0) sin(2 pi u1).

Readings: entry S_k[i, 4q + t] (t = 0..3) is normal t of the block drawn
with counter (i, k, q, 0) and key (seed low word, seed high word): words
0, 1 give normals 0, 1 and words 2, 3 normals 2, 3.  k counts iterations
from 1.  The residual is updated recursively (r <- r - A p) and the stop
test is Algorithm 1's, as for the other sketches.  A column of Y_k whose
pivot in column order (the Schur complement of Y_kᵀ Y_k after the earlier
kept columns) is at most 1e-14 ||y_j||^2 is left out (the pseudo-inverse the
paper prescribes when the inverse does not exist, restricted to a basis of
the span); an iteration with no kept column is a breakdown.
"""
from __future__ import annotations

import math

import numpy as np

from .plss import BREAKDOWN, NOT_CONVERGED, OK, Result, _as_sparse, _relres_true

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 of counters ``ctr`` (array (..., 4), uint32 values) with
    key ``key`` (two 32-bit words).  Returns an array (..., 4) of uint32."""
    c = [np.asarray(ctr[..., j], dtype=np.uint64) for j in range(4)]
    k0, k1 = np.uint64(key[0] & MASK), np.uint64(key[1] & MASK)
    m0, m1, mask = np.uint64(M0), np.uint64(M1), np.uint64(MASK)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + np.uint64(W0)) & mask
            k1 = (k1 + np.uint64(W1)) & mask
        p0 = m0 * c[0]
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [(hi1 ^ c[1] ^ k0) & mask, lo1, (hi0 ^ c[3] ^ k1) & mask, lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def uniforms(words):
    return (np.asarray(words, dtype=np.float64) + 0.5) * 2.0 ** -32


def box_muller(u0, u1):
    rad = np.sqrt(-2.0 * np.log(u0))
    ang = 2.0 * math.pi * u1
    return rad * np.cos(ang), rad * np.sin(ang)


def sketch(m, r, it, seed):
    """S_it (m x r): entry [i, 4q + t] from Philox counter (i, it, q, 0)."""
    nq = (r + 3) // 4
    i = np.repeat(np.arange(m, dtype=np.uint64), nq)
    q = np.tile(np.arange(nq, dtype=np.uint64), m)
    ctr = np.stack([i, np.full_like(i, it), q, np.zeros_like(i)], axis=-1)
    w = philox4x32_10(ctr, (seed & MASK, (seed >> 32) & MASK))
    u = uniforms(w)
    z0, z1 = box_muller(u[:, 0], u[:, 1])
    z2, z3 = box_muller(u[:, 2], u[:, 3])
    z = np.stack([z0, z1, z2, z3], axis=-1).reshape(m, nq * 4)
    return z[:, :r]


def randproj(A, b, r=10, seed=0, tol=1e-8, maxit=1000, tol_absolute=False, record=False, dot=None) -> Result:
    """Randomized projection with fresh Gaussian sketches (W = I, x0 = 0)."""
    dot = dot or (lambda a, c: float(a @ c))
    S_ = _as_sparse(A)
    m, n = S_.shape
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    thr = tol if tol_absolute else tol * nb
    scale = 1.0 if tol_absolute or nb == 0 else 1.0 / nb
    x = np.zeros(n)
    res = b.copy()
    rho = dot(res, res)
    hist = [math.sqrt(rho) * scale]
    xs = [x.copy()] if record else None
    ps = [] if record else None
    rs = [res.copy()] if record else None
    k = 0

    def done(status):
        return Result(x, k, hist, status, _relres_true(S_, x, b, nb), xs, ps, rs, None)

    if math.sqrt(rho) <= thr:
        return done(OK)
    while True:
        S = sketch(m, r, k + 1, seed)
        Y = S_.T @ S                                   # Y_k = Aᵀ S_k
        G = np.array([[dot(Y[:, a], Y[:, c]) for c in range(r)] for a in range(r)])
        sig = np.array([dot(S[:, a], res) for a in range(r)])
        keep = []
        for j in range(r):
            if keep:
                Gk = G[np.ix_(keep, keep)]
                piv = G[j, j] - G[j, keep] @ np.linalg.solve(Gk, G[keep, j])
            else:
                piv = G[j, j]
            if piv > 1e-14 * G[j, j]:
                keep.append(j)
        if not keep:
            return done(BREAKDOWN)
        c = np.linalg.solve(G[np.ix_(keep, keep)], sig[keep])
        p = Y[:, keep] @ c
        res = res - S_ @ p
        x = x + p
        k += 1
        rho = dot(res, res)
        hist.append(math.sqrt(rho) * scale)
        if record:
            xs.append(x.copy()); ps.append(p.copy()); rs.append(res.copy())
        if math.sqrt(rho) <= thr:
            return done(OK)
        if k >= maxit:
            return done(NOT_CONVERGED)
