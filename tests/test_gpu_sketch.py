"""GPU parity of the identity (Section 7) and mixed sketches against the
oracle's one-column step, at equal update counts (see gpu_common)."""
import sys

import numpy as np
import pytest

import plss_inputs as gen
from oracle import pins
from oracle import plss as O

from gpu_common import CONVERGED_TOL, chunk_dot, converged_check, fsum_dot, matrix, order_bound, rel, rev_dot

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2207_07615_amd as plss
    return plss.Handle(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def column_parity(h, sysm, sketch, tol, maxit, cap):
    import paper_2207_07615_amd as plss
    M = matrix(h, sysm.A)
    x, info, hist = plss.solve(h, M, sysm.b, sketch=sketch, tol=tol, maxit=maxit,
                               row_perm=sysm.perm, hist_cap=cap)
    k = info["iters"]
    ref = O.plss_columns(sysm.A, sysm.b, sketch, perm=sysm.perm, tol=1e-300, maxit=k, hist_cap=cap)
    spread = 0.0
    for dot in (fsum_dot, rev_dot, chunk_dot):
        alt = O.plss_columns(sysm.A, sysm.b, sketch, perm=sysm.perm, tol=1e-300, maxit=k,
                             hist_cap=cap, dot=dot)
        spread = max(spread, rel(alt.x, ref.x))
    err = rel(x, ref.x)
    say(f"  {sketch}: updates={k} columns={info['outer_iters']} err={err:.3e} spread={spread:.3e}")
    assert ref.iters == k
    order_bound(err, spread, f"{sketch}_{sysm.A.m}x{sysm.A.n}_cap{cap}")
    # converged (relres 1e-13) against the oracle at the flat 1e-10
    xc, ic, _ = plss.solve(h, M, sysm.b, sketch=sketch, tol=CONVERGED_TOL, maxit=20 * maxit,
                           row_perm=sysm.perm, hist_cap=cap)
    assert ic["status"] == 0, ic
    refc = O.plss_columns(sysm.A, sysm.b, sketch, perm=sysm.perm, tol=CONVERGED_TOL,
                          maxit=20 * maxit, hist_cap=cap)
    assert refc.status == O.OK
    converged_check(xc, refc.x, f"{sketch}_{sysm.A.m}x{sysm.A.n}_cap{cap}")
    return x, info, hist, ref


@pytest.mark.parametrize("sketch", ["identity", "mixed"])
def test_tiny_sketch_matches_oracle(h, sketch):
    say("tiny", sketch)
    sysm = gen.tiny(31, 60, 150, 8, "uniform")
    x, info, hist, ref = column_parity(h, sysm, sketch, 1e-10, 4000, 60)
    assert info["status"] == 0
    np.testing.assert_allclose(hist[:5], ref.hist[:5], rtol=1e-9)


def test_identity_underdetermined_reaches_min_norm(h):
    """Corollary 2: a full pass of identity columns on a full-row-rank
    64 x 256 system gives A†b."""
    import paper_2207_07615_amd as plss
    say("cor2")
    sysm = gen.tiny(77, 64, 256, 30, "uniform")
    M = matrix(h, sysm.A)
    x, info, _ = plss.solve(h, M, sysm.b, sketch="identity", tol=1e-12, maxit=64,
                            row_perm=sysm.perm, hist_cap=64)
    xm = pins.min_norm(sysm.A.dense(), sysm.b)
    assert info["iters"] <= 64
    assert rel(x, xm) <= 1e-10


def test_identity_orthogonal_rows_is_kaczmarz(h):
    """Rows with disjoint supports: each step is the Kaczmarz step."""
    import paper_2207_07615_amd as plss
    from gpu_common import csr_from_dense
    say("kaczmarz")
    m, n = 6, 18
    rng = np.random.default_rng(5)
    D = np.zeros((m, n))
    cols = rng.permutation(n)
    for i in range(m):
        D[i, cols[3 * i:3 * i + 3]] = rng.standard_normal(3)
    b = D @ rng.standard_normal(n)
    order = rng.permutation(m).astype(np.int32)
    rp, ci, va = csr_from_dense(D)
    M = plss.Matrix(h, rp, ci, va, shape=(m, n))
    kz = pins.kaczmarz(D, b, order)
    for k in range(1, m + 1):
        x, info, _ = plss.solve(h, M, b, sketch="identity", tol=1e-300, maxit=k, row_perm=order)
        assert rel(x, kz[k - 1]) <= 1e-13


@pytest.mark.parametrize("cap", [3, 7])
def test_history_cap_matches_oracle(h, cap):
    """A small history capacity clears P, AP, Θ periodically on both sides."""
    say("cap", cap)
    sysm = gen.tiny(41, 80, 200, 10, "uniform")
    column_parity(h, sysm, "mixed", 1e-9, 3000, cap)


def test_history_block_reuse_leaves_no_trace():
    """A handle keeps the sketch history block between calls: a solve after
    a larger one (block filled with its columns) and after a smaller one is
    bit-identical to the same solve on a fresh handle."""
    import paper_2207_07615_amd as plss
    say("history block reuse")
    big = gen.underdet(m=3000, n=12000)
    mid = gen.tiny(43, 900, 2500, 12, "uniform")
    small = gen.tiny(44, 60, 150, 8, "uniform")
    kw = dict(sketch="mixed", tol=1e-10, maxit=400, hist_cap=48)

    def solve(hd, sysm):
        M = matrix(hd, sysm.A)
        return plss.solve(hd, M, sysm.b, row_perm=sysm.perm, **kw)

    fresh = plss.Handle(0)
    x_ref, i_ref, _ = solve(fresh, mid)
    reused = plss.Handle(0)
    solve(reused, big)
    x1, i1, _ = solve(reused, mid)
    solve(reused, small)
    x2, i2, _ = solve(reused, mid)
    assert i1["iters"] == i2["iters"] == i_ref["iters"] > 0
    np.testing.assert_array_equal(x1, x_ref)
    np.testing.assert_array_equal(x2, x_ref)


def test_release_workspace_keeps_results():
    """plss_release_workspace frees a handle's scratch; the calls after it
    (a mixed-sketch solve, a batch and a residual-sketch solve) allocate
    afresh and give the same bits as before it; releasing twice is fine."""
    import paper_2207_07615_amd as plss
    say("release workspace")
    hd = plss.Handle(0)
    mid = gen.tiny(43, 900, 2500, 12, "uniform")
    sq = gen.small(m=600, n=300)
    Mm, Ms = matrix(hd, mid.A), matrix(hd, sq.A)
    kw = dict(sketch="mixed", tol=1e-10, maxit=400, hist_cap=48, row_perm=mid.perm)

    def run():
        xm, im, _ = plss.solve(hd, Mm, mid.b, **kw)
        xb, ib = plss.solve_batch(hd, [Ms, Ms], [sq.b, 2.0 * sq.b], tol=1e-10, maxit=2000)
        xr, ir, _ = plss.solve(hd, Ms, sq.b, tol=1e-10, maxit=2000, engine="multi")
        return [xm, xb[0], xb[1], xr], [im["iters"], ib[0]["iters"], ib[1]["iters"], ir["iters"]]

    xs0, its0 = run()
    hd.release_workspace()
    hd.release_workspace()
    xs1, its1 = run()
    assert its0 == its1 and min(its0) > 0
    for a, b in zip(xs0, xs1):
        np.testing.assert_array_equal(a, b)


def test_mixed_underdetermined_medium(h):
    """The underdetermined recipe (30 nnz per row, U(-1,1)) at 20,000 x
    100,000, mixed sketch, tol 1e-8, against the oracle and A†b-consistency."""
    say("mixed medium")
    sysm = gen.underdet(m=20000, n=100000)
    x, info, hist, ref = column_parity(h, sysm, "mixed", 1e-8, 2000, 64)
    assert info["status"] == 0
    assert info["relres_true"] <= 1.5e-8
    # x lies in range(Aᵀ) (x0 = 0), so it is the minimum-norm solution up to
    # the residual: compare with the oracle's converged iterate
    full = O.plss_columns(sysm.A, sysm.b, "mixed", perm=sysm.perm, tol=1e-8, maxit=2000, hist_cap=64)
    assert abs(full.iters - info["iters"]) <= 1


def test_mixed_column_blocks(h):
    """A wide underdetermined system (8,000 x 500,000: the new column of P,
    4 MB, does not fit one XCD's L2), so the product A p runs over column
    blocks of A (one per XCD) and their fixed-order sum; against the oracle
    at equal update counts and converged."""
    import paper_2207_07615_amd as plss
    say("mixed column blocks")
    sysm = gen.underdet(m=8000, n=500000)
    M = matrix(h, sysm.A)
    before = M.info()["device_bytes"]
    plss.solve(h, M, sysm.b, sketch="mixed", tol=1e-300, maxit=2, row_perm=sysm.perm, hist_cap=32)
    # the column-blocked copy of A was built by the first sketch solve
    assert M.info()["device_bytes"] - before >= 12 * sysm.A.nnz
    x, info, hist, ref = column_parity(h, sysm, "mixed", 1e-8, 2000, 32)
    assert info["status"] == 0


def dependent_rows_system(seed=61):
    """Identity-sketch system whose row order meets every branch of the skip
    rule (Section 7, eq. pkKacz; reading C7): 20 row pairs (u, u) with u =
    (1,1,1,1) on 4 own columns (dyadic, so the residual at the repeat is an
    exact zero: sigma == 0); 20 triples (u, v, u + v) of N(0,1) rows on
    disjoint supports (the sum is exact, the residual at it a rounding
    remainder: delta ~ 1e-16 ||a||^2); 10 triples (w, z, w + z + 0.01 e_c)
    (nearly dependent: an update); then 30 rows of 20 N(0,1) entries over all
    columns, which overlap everything before them.  x* has entries in
    {1, 2, 3}, so no row's right-hand side is zero by accident."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    n = 500
    cols = list(rng.permutation(n))
    rows = []
    for _ in range(20):
        c = [cols.pop() for _ in range(4)]
        rows += [(c, [1.0] * 4)] * 2
    for _ in range(20):
        cu = [cols.pop() for _ in range(5)]
        cv = [cols.pop() for _ in range(5)]
        u, v = rng.standard_normal(5), rng.standard_normal(5)
        rows += [(cu, list(u)), (cv, list(v)), (cu + cv, list(u) + list(v))]
    for _ in range(10):
        cw = [cols.pop() for _ in range(5)]
        cz = [cols.pop() for _ in range(5)]
        ce = [cols.pop()]
        w, z = rng.standard_normal(5), rng.standard_normal(5)
        rows += [(cw, list(w)), (cz, list(z)), (cw + cz + ce, list(w) + list(z) + [0.01])]
    for _ in range(30):
        c = list(rng.choice(n, 20, replace=False))
        rows += [(c, list(rng.standard_normal(20)))]
    m = len(rows)
    D = np.zeros((m, n))
    for i, (c, v) in enumerate(rows):
        D[i, c] = v
    xs = rng.integers(1, 4, n).astype(np.float64)
    S = sp.csr_matrix(D)
    S.sort_indices()
    return D, S, S @ xs


def test_identity_skip_rule_matches_oracle(h):
    """Repeated, dependent and nearly dependent rows: the GPU skips the
    columns the oracle skips (same update count, same number of columns
    examined), its iterate after the pass agrees with the oracle's to 1e-10,
    and it is A†b (Corollary 2 on the independent rows)."""
    import paper_2207_07615_amd as plss
    say("skip rule")
    D, S, b = dependent_rows_system()
    m, n = D.shape
    M = plss.Matrix(h, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data, shape=(m, n))
    order = np.arange(m, dtype=np.int32)
    ref = O.plss_columns(D, b, "identity", perm=order, tol=1e-300, maxit=m, max_columns=m,
                         record=True)
    used = [c[1] for c in ref.columns]
    skipped = sorted(set(range(m)) - set(used))
    # the 20 repeats and the 20 exact sums, nothing else
    assert len(skipped) == 40 and ref.iters == m - 40
    x, info, _ = plss.solve(h, M, b, sketch="identity", tol=1e-300, maxit=ref.iters, row_perm=order)
    err = rel(x, ref.x)
    say(f"  updates={info['iters']} columns={info['outer_iters']} err={err:.3e}")
    assert info["iters"] == ref.iters
    assert info["outer_iters"] == m
    assert err <= 1e-10
    assert rel(x, pins.min_norm(D, b)) <= 1e-9
    # converged solve: same updates as the oracle's own
    x2, i2, _ = plss.solve(h, M, b, sketch="identity", tol=1e-12, maxit=10 * m, row_perm=order)
    r2 = O.plss_columns(D, b, "identity", perm=order, tol=1e-12, maxit=10 * m)
    assert i2["status"] == 0 and i2["iters"] == r2.iters
    assert rel(x2, r2.x) <= 1e-10


def test_mixed_skip_rule_matches_oracle(h):
    """The same system under the mixed sketch: equal update counts and
    iterates at every checked count."""
    import paper_2207_07615_amd as plss
    say("skip rule, mixed")
    D, S, b = dependent_rows_system(seed=62)
    m, n = D.shape
    M = plss.Matrix(h, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data, shape=(m, n))
    order = np.arange(m, dtype=np.int32)
    for k in (10, 40, 90):
        x, info, _ = plss.solve(h, M, b, sketch="mixed", tol=1e-300, maxit=k, row_perm=order)
        ref = O.plss_columns(D, b, "mixed", perm=order, tol=1e-300, maxit=k)
        assert info["iters"] == ref.iters == k
        assert rel(x, ref.x) <= 1e-10, (k, rel(x, ref.x))


def test_sketch_edge_cases(h):
    import paper_2207_07615_amd as plss
    say("sketch edges")
    sysm = gen.tiny(55, 40, 90, 6)
    M = matrix(h, sysm.A)
    x, info, _ = plss.solve(h, M, np.zeros(40), sketch="mixed", tol=1e-8, maxit=10, row_perm=sysm.perm)
    assert info["iters"] == 0 and not np.any(x)
    x, info, _ = plss.solve(h, M, sysm.b, sketch="identity", tol=1e-14, maxit=1, row_perm=sysm.perm)
    ref = O.plss_columns(sysm.A, sysm.b, "identity", perm=sysm.perm, tol=1e-14, maxit=1)
    assert info["iters"] == 1 and rel(x, ref.x) <= 1e-13
    bad = np.arange(40, dtype=np.int32)
    bad[3] = 4
    with pytest.raises(plss.PlssError):
        plss.solve(h, M, sysm.b, sketch="identity", tol=1e-8, maxit=10, row_perm=bad)
    M32 = matrix(h, sysm.A, "f32")
    with pytest.raises(plss.PlssError):
        plss.solve(h, M32, sysm.b, sketch="identity", tol=1e-8, maxit=10)
