"""Helpers of the GPU tests (host side only)."""
import json
import os

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


def fsum_dot(a, b):
    import math
    return math.fsum(a * b)


def rev_dot(a, b):
    return float(a[::-1] @ b[::-1])


def chunk_dot(a, b):
    c = a * b
    n = len(c)
    k = max(1, n // 97)
    return float(sum(float(c[i:i + k].sum()) for i in range(0, n, k)))


# Relative residual both sides are run to before their solutions are compared
# at the flat float64 tolerance: near convergence the iterates of any
# summation order approach the same limit (x* or A†b), so two converged runs
# differ by about kappa * CONVERGED_TOL, far below PARITY_TOL.
CONVERGED_TOL = 1e-13
PARITY_TOL = 1e-10
# Margin of the equal-iteration-count check over the order spread (see
# order_bound).
SPREAD_MARGIN = 4.0


def log_parity(**kw):
    """Append one record of a parity check to $PLSS_PARITY_LOG (JSON lines),
    when set: the measured errors, spreads and their ratio per case."""
    path = os.environ.get("PLSS_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(kw) + "\n")


def order_bound(err, spread, case):
    """Equal-iteration-count check: the GPU run is one more float64
    evaluation of the same recurrence with another summation order, so its
    distance from the oracle is of the size of the spread between the
    oracle's own reorderings.  The spread is the largest of three samples;
    the bound is SPREAD_MARGIN times it (never below PARITY_TOL).  The ratio
    err/spread is logged per case; the largest measured is recorded beside
    the margin in the project's design notes.  This check is a trajectory
    check; the stated 1e-10 is asserted on converged solutions
    (converged_check)."""
    log_parity(case=case, kind="equal_count", err=err, spread=spread,
               ratio=(err / spread if spread > 0 else None))
    assert err <= max(PARITY_TOL, SPREAD_MARGIN * spread), (case, err, spread)


def converged_check(x_gpu, x_ref, case, tol=PARITY_TOL):
    """Flat float64 parity of two solutions both run to CONVERGED_TOL."""
    err = rel(x_gpu, x_ref)
    log_parity(case=case, kind="converged", err=err)
    print(f"  {case}: converged err_vs_oracle={err:.3e}", flush=True)
    assert err <= tol, (case, err)
    return err


def order_spread(A, b, k, wi=None, x0=None):
    """Largest distance, after k iterations, between the oracle's iterate and
    three reruns that change only the summation order of inner products."""
    from oracle import plss as O
    ref = O.plss_residual(A, b, tol=1e-300, maxit=k, wi=wi, x0=x0)
    spread = 0.0
    for dot in (fsum_dot, rev_dot, chunk_dot):
        alt = O.plss_residual(A, b, tol=1e-300, maxit=k, wi=wi, x0=x0, dot=dot)
        spread = max(spread, rel(alt.x, ref.x))
    return ref, spread


def fp64_parity(h, sysm, tol=1e-8, maxit=5000, wi=None, storage="f64", layout=None,
                case="fp64", **kw):
    """Check a float64 solve against Algorithm 1 (oracle):

    * the GPU meets the stop test and its iteration count is within one of
      the oracle's own count;
    * solved to relative residual 1e-13 on both sides, the solutions agree
      within the stated 1e-10 (converged_check);
    * at the GPU's iteration count the two iterates agree within the
      trajectory bound of order_bound: the finite-precision Craig/Lanczos
      process amplifies rounding differences, so the spread between
      equally valid float64 runs of the oracle (not machine epsilon) is the
      floor there;
    * the first 15 iterates agree to 1e-12 (before the amplification).
    Returns the GPU's (x, info)."""
    import paper_2207_07615_amd as plss
    from oracle import plss as O
    M = matrix(h, sysm.A, storage)
    if layout is not None:
        M.layout(**layout)
    x, info, hist = plss.solve(h, M, sysm.b, tol=tol, maxit=maxit, wi=wi, **kw)
    assert info["status"] == 0, info
    k = info["iters"]
    ref, floor = order_spread(sysm.A, sysm.b, k, wi=wi)
    err = rel(x, ref.x)
    print(f"  iters={k} err_vs_oracle={err:.3e} oracle_order_spread={floor:.3e}", flush=True)
    order_bound(err, floor, case)
    full = O.plss_residual(sysm.A, sysm.b, tol=tol, maxit=maxit, wi=wi)
    assert abs(full.iters - k) <= 1
    xc, ic, _ = plss.solve(h, M, sysm.b, tol=CONVERGED_TOL, maxit=20 * maxit, wi=wi, **kw)
    assert ic["status"] == 0, ic
    refc = O.plss_residual(sysm.A, sysm.b, tol=CONVERGED_TOL, maxit=20 * maxit, wi=wi)
    assert refc.status == O.OK
    converged_check(xc, refc.x, case)
    k15 = min(15, k)
    x15, i15, _ = plss.solve(h, M, sysm.b, tol=1e-300, maxit=k15, wi=wi, **kw)
    r15 = O.plss_residual(sysm.A, sysm.b, tol=1e-300, maxit=k15, wi=wi)
    assert rel(x15, r15.x) <= 1e-12
    return x, info, M
