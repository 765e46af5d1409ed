"""GPU parity of the residual-sketch path against the CPU oracle.

Structure (CSC copy) is compared bit for bit; products entry by entry; solves
at equal iteration counts (the oracle is rerun with maxit = the GPU's count,
since a stop one iteration apart differs by ||p_k||)."""
import sys

import numpy as np
import pytest

import plss_inputs as gen
from oracle import plss as O
from oracle import sparse as osp

from gpu_common import (CONVERGED_TOL, converged_check, csr_from_dense, fp64_parity, matrix,
                        order_bound, order_spread, rel)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2207_07615_amd as plss
    return plss.Handle(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ragged_matrix(seed, m, n):
    """Rows of very different lengths: empty rows, short rows, and rows longer
    than any tile (4096 entries), so tiles of every kind appear."""
    rng = gen.rng_for(seed)
    L = rng.integers(0, 12, size=m)
    L[rng.random(m) < 0.1] = 0
    L[:: max(1, m // 3)] = min(n, 4500)
    L[5] = min(n, 2048)
    L = np.minimum(L, n)
    return gen.make_csr(rng, m, n, L, "normal")


def long_columns_matrix(seed=6, m=100_000, n=3000):
    """Column 0 in every row (10^5 entries), column 1 in 513 rows, column 2
    in 4097 rows and column 3 in 12,293 rows (columns longer than a wave's
    in-LDS sort, in one or several 4096-entry tiles of the long-column
    sort), plus 3 random columns per row."""
    import scipy.sparse as sp
    rng = gen.rng_for(seed)
    rows, cols = [], []
    for c, cnt in ((0, m), (1, 513), (2, 4097), (3, 12293)):
        rr = np.sort(rng.choice(m, cnt, replace=False))
        rows.append(rr)
        cols.append(np.full(cnt, c))
    rr = np.repeat(np.arange(m), 3)
    rows.append(rr)
    cols.append(rng.integers(4, n, size=rr.size))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    S = sp.csr_matrix((rng.standard_normal(rows.size), (rows, cols)), shape=(m, n))
    S.sum_duplicates()
    S.sort_indices()
    return gen.CSR(m, n, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.astype(np.float64))


@pytest.mark.parametrize("case", ["small", "ragged", "wide", "single", "long_columns"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_csc_bit_exact(h, case, storage):
    say("csc", case, storage)
    if case == "long_columns":
        A = long_columns_matrix()
    elif case == "small":
        A = gen.small(m=3000, n=1500).A
    elif case == "ragged":
        A = ragged_matrix(3, 9000, 6000)
    elif case == "wide":
        A = gen.tiny(4, 300, 20000, 30).A
    else:
        A = gen.make_csr(gen.rng_for(5), 1, 10, np.array([3]), "normal")
    M = matrix(h, A, storage)
    cp, ri, va = M.csc()
    ocp, ori, ova = osp.csr_to_csc(A.m, A.n, A.row_ptr, A.col_idx, A.vals)
    np.testing.assert_array_equal(cp, ocp)
    np.testing.assert_array_equal(ri, ori)
    want = ova if storage == "f64" else ova.astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(va, want)


@pytest.mark.parametrize("case", ["small", "ragged"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_spmv_entrywise(h, case, storage):
    import paper_2207_07615_amd as plss
    say("spmv", case, storage)
    A = gen.small(m=3000, n=1500).A if case == "small" else ragged_matrix(7, 9000, 6000)
    M = matrix(h, A, storage)
    S = A.astype(np.float32).scipy() if storage == "f32" else A.scipy()
    rng = np.random.default_rng(1)
    x = rng.standard_normal(A.n)
    u = rng.standard_normal(A.m)
    y = plss.spmv(h, M, x)
    yt = plss.spmv(h, M, u, transpose=True)
    absA = abs(S)
    tol_y = 1e-14 * (absA @ abs(x)) + 1e-300
    tol_t = 1e-14 * (absA.T @ abs(u)) + 1e-300
    assert np.all(abs(y - S @ x) <= tol_y)
    assert np.all(abs(yt - S.T @ u) <= tol_t)


def test_small_workload_fp64_matches_oracle(h):
    """2000 x 1000, 8 nnz per row, FP64, tol 1e-8 (see fp64_parity)."""
    import paper_2207_07615_amd as plss
    say("small fp64")
    sysm = gen.small()
    x, info, M = fp64_parity(h, sysm, case="small")
    assert info["relres_true"] <= 1.5e-8
    # the converged solution (relres 1e-13) is also x* (full column rank)
    xt, it, _ = plss.solve(h, M, sysm.b, tol=CONVERGED_TOL, maxit=5000)
    assert it["status"] == 0
    assert rel(xt, sysm.xstar) <= 1e-10


def test_solve_deterministic(h):
    import paper_2207_07615_amd as plss
    say("determinism")
    sysm = gen.large(m=60000, n=15000)
    M = matrix(h, sysm.A)
    x1, i1, h1 = plss.solve(h, M, sysm.b, tol=1e-8, maxit=2000)
    x2, i2, h2 = plss.solve(h, M, sysm.b, tol=1e-8, maxit=2000)
    assert i1["iters"] == i2["iters"]
    np.testing.assert_array_equal(x1, x2)
    np.testing.assert_array_equal(h1, h2)


def test_zipf_rows_fp64_matches_oracle(h):
    """Heavy-tailed rows (Zipf(1.5) clipped to [2, 2000]) at a size the
    oracle runs in seconds, spanning many tiles of every kind."""
    say("zipf fp64")
    sysm = gen.large(m=60000, n=15000)
    x, info, M = fp64_parity(h, sysm, case="zipf_60000x15000_tiles")
    assert info["relres_true"] <= 1.5e-8


@pytest.mark.parametrize("engine", ["auto", "multi"])
def test_weighted_W(h, engine):
    """PLSS W (Section 4.1): W = diag(1/||A_{:,j}||) through wi_diag, in the
    single-workgroup solver (auto at this size) and in the per-phase
    launches (the block sum's phi and the update's p, theta weighted)."""
    say("W", engine)
    sysm = gen.small(m=3000, n=1500)
    wi = np.sqrt(np.asarray(sysm.A.scipy().multiply(sysm.A.scipy()).sum(axis=0)).ravel())
    kw = {} if engine == "auto" else {"engine": engine}
    fp64_parity(h, sysm, wi=wi, case=f"W_3000x1500_{engine}", **kw)


def test_edge_cases(h):
    import paper_2207_07615_amd as plss
    say("edges")
    sysm = gen.small(m=400, n=200)
    M = matrix(h, sysm.A)
    # b = 0: x0 returned after 0 updates
    x, info, hist = plss.solve(h, M, np.zeros(400), tol=1e-8, maxit=10)
    assert info["iters"] == 0 and info["status"] == 0 and not np.any(x)
    # maxit = 1
    x, info, hist = plss.solve(h, M, sysm.b, tol=1e-12, maxit=1)
    assert info["iters"] == 1 and info["status"] == 1
    ref = O.plss_residual(sysm.A, sysm.b, tol=1e-12, maxit=1)
    assert rel(x, ref.x) <= 1e-13
    # inconsistent b: breakdown or no convergence, never a false OK
    b = sysm.b + np.random.default_rng(0).standard_normal(400)
    x, info, hist = plss.solve(h, M, b, tol=1e-12, maxit=300)
    assert info["status"] in (1, 2)
    # x0 given: same as starting the oracle there
    x0 = np.random.default_rng(2).standard_normal(200)
    x, info, hist = plss.solve(h, M, sysm.b, tol=1e-10, maxit=500, x0=x0)
    ref = O.plss_residual(sysm.A, sysm.b, tol=1e-300, maxit=info["iters"], x0=x0)
    assert rel(x, ref.x) <= 1e-10
    # malformed input is rejected
    with pytest.raises(plss.PlssError):
        plss.solve(h, M, np.full(400, np.nan), tol=1e-8, maxit=10)
    with pytest.raises(plss.PlssError):
        plss.solve(h, M, sysm.b, tol=-1.0, maxit=10)
    bad_col = sysm.A.col_idx.copy()
    bad_col[3] = 10**6
    with pytest.raises(plss.PlssError):
        plss.Matrix(h, sysm.A.row_ptr, bad_col, sysm.A.vals, shape=(400, 200))
    unsorted = sysm.A.col_idx.copy()
    unsorted[0], unsorted[1] = unsorted[1], unsorted[0]
    with pytest.raises(plss.PlssError):
        plss.Matrix(h, sysm.A.row_ptr, unsorted, sysm.A.vals, shape=(400, 200))


def test_tiny_dense_systems(h):
    """Over- and under-determined tiny systems reach A†b."""
    import paper_2207_07615_amd as plss
    from oracle import pins
    say("tiny")
    for m, n in [(20, 8), (8, 20), (64, 256)]:
        sysm = gen.tiny(500 + m + n, m, n, min(n, 30), "uniform")
        M = matrix(h, sysm.A)
        x, info, _ = plss.solve(h, M, sysm.b, tol=1e-13, maxit=4000)
        assert info["status"] == 0
        xm = pins.min_norm(sysm.A.dense(), sysm.b)
        assert rel(x, xm) <= 1e-9


def test_fp32_storage_with_refinement(h):
    """float32 storage (Â = fl32(A)) + float64 refinement reaches the float64
    tolerance; the reference is Algorithm 1 on Â in float64."""
    import paper_2207_07615_amd as plss
    say("fp32 refine")
    sysm = gen.small(storage=np.float32)
    M = matrix(h, sysm.A, "f32")
    x, info, _ = plss.solve(h, M, sysm.b, tol=1e-12, maxit=5000, refine=True, inner_tol=1e-4)
    assert info["status"] == 0, info
    assert info["relres_true"] <= 1e-12
    assert info["outer_iters"] >= 2
    ref = O.plss_residual(sysm.A, sysm.b, tol=1e-13, maxit=5000)
    assert rel(x, ref.x) <= 1e-10
    assert rel(x, sysm.xstar) <= 1e-10
    # one inner solve without refinement: float32-level accuracy only
    x1, i1, _ = plss.solve(h, M, sysm.b, tol=1e-6, maxit=5000, refine=False)
    assert 1e-9 < rel(x1, sysm.xstar) <= 1e-5


def test_batch_equals_alone(h):
    """Systems solved together give bit-identical results to each alone."""
    import paper_2207_07615_amd as plss
    say("batch")
    systems = gen.batch_systems(6, m_lo=1e3, m_hi=2e4)
    mats = [matrix(h, s.A) for s in systems]
    xs, infos = plss.solve_batch(h, mats, [s.b for s in systems], tol=1e-8, maxit=5000)
    for s, M, x, inf in zip(systems, mats, xs, infos):
        xa, ia, _ = plss.solve(h, M, s.b, tol=1e-8, maxit=5000)
        assert inf["iters"] == ia["iters"]
        np.testing.assert_array_equal(x, xa)
        assert inf["status"] == 0
        ref, spread = order_spread(s.A, s.b, inf["iters"])
        order_bound(rel(x, ref.x), spread, f"batch_{s.A.m}x{s.A.n}")
    # converged batch (relres 1e-13) against the oracle at the flat 1e-10
    xs, infos = plss.solve_batch(h, mats, [s.b for s in systems], tol=CONVERGED_TOL, maxit=50000)
    for s, x, inf in zip(systems, xs, infos):
        assert inf["status"] == 0, inf
        ref = O.plss_residual(s.A, s.b, tol=CONVERGED_TOL, maxit=50000)
        assert ref.status == O.OK
        converged_check(x, ref.x, f"batch_{s.A.m}x{s.A.n}")


@pytest.mark.parametrize("storage,m", [("f64", 500_000), ("f32", 800_000)])
def test_row_blocked_transpose(h, storage, m):
    """Past ~3 MB of r the product with Aᵀ runs on a row-blocked copy of the
    transpose (one block per XCD); the first iterates match the oracle and
    the full solve meets the tolerance."""
    import paper_2207_07615_amd as plss
    say("row-blocked", storage, m)
    dt = np.float32 if storage == "f32" else np.float64
    sysm = gen.large(m=m, n=m // 4, storage=dt)
    M = matrix(h, sysm.A, storage)
    assert M.info()["device_bytes"] > 3 * sysm.A.nnz * (8 if storage == "f32" else 12)
    if storage == "f64":
        x, info, _ = plss.solve(h, M, sysm.b, tol=1e-300, maxit=12)
        ref = O.plss_residual(sysm.A, sysm.b, tol=1e-300, maxit=12)
        assert rel(x, ref.x) <= 1e-12
        x, info, _ = plss.solve(h, M, sysm.b, tol=1e-8, maxit=1000)
        assert info["status"] == 0 and info["relres_true"] <= 1.5e-8
    else:
        x, info, _ = plss.solve(h, M, sysm.b, tol=1e-8, maxit=4000, refine=True)
        assert info["status"] == 0 and info["relres_true"] <= 1e-8
        assert rel(x, sysm.xstar) <= 1e-6
    cp, ri, va = M.csc()
    ocp, ori, ova = osp.csr_to_csc(sysm.A.m, sysm.A.n, sysm.A.row_ptr, sysm.A.col_idx, sysm.A.vals)
    np.testing.assert_array_equal(cp, ocp)
    np.testing.assert_array_equal(ri, ori)


def test_autotune_keeps_parity(h):
    """The tile autotuner (plss_matrix_autotune) times the plain product for
    each tile width and keeps the fastest per direction; products and the
    first iterates after it are the oracle's, and the solve still meets the
    stop test."""
    import paper_2207_07615_amd as plss
    say("autotune")
    sysm = gen.large(m=60000, n=15000)
    M = matrix(h, sysm.A)
    a, t = M.autotune()
    say(f"  widths: A {a}, A^T {t}")
    assert a in (4, 8, 16) and t in (4, 8, 16)
    S = sysm.A.scipy()
    rng = np.random.default_rng(8)
    v = rng.standard_normal(sysm.A.n)
    u = rng.standard_normal(sysm.A.m)
    assert np.all(abs(plss.spmv(h, M, v) - S @ v) <= 1e-14 * (abs(S) @ abs(v)) + 1e-300)
    assert np.all(abs(plss.spmv(h, M, u, transpose=True) - S.T @ u) <= 1e-14 * (abs(S).T @ abs(u)) + 1e-300)
    x, info, _ = plss.solve(h, M, sysm.b, tol=1e-300, maxit=15)
    ref = O.plss_residual(sysm.A, sysm.b, tol=1e-300, maxit=15)
    assert rel(x, ref.x) <= 1e-12
    x, info, _ = plss.solve(h, M, sysm.b, tol=1e-8, maxit=2000)
    assert info["status"] == 0 and info["relres_true"] <= 1.5e-8
