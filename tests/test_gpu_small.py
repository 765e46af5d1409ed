"""Single-workgroup engine (one workgroup runs a whole small solve, vectors
in LDS) against the oracle and against the one-launch-per-phase engine.

Both engines take the same decisions (stop test, breakdown, iteration
limit, refinement restarts) with sums in different orders, so they stop at
the same iteration and their iterates agree within the float64 trajectory
spread that the oracle itself shows under reordered inner products."""
import sys

import numpy as np
import pytest

import plss_inputs as gen
from oracle import plss as O

from gpu_common import CONVERGED_TOL, converged_check, fp64_parity, matrix, order_bound, order_spread, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2207_07615_amd as plss
    return plss.Handle(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def long_rows_system(seed=31, m=1500, n=1200):
    """Rows and columns longer than 64 entries (summed by whole waves)
    beside short ones, rows scaled to unit norm."""
    rng = gen.rng_for(seed)
    L = rng.integers(2, 12, size=m)
    L[::97] = 400
    L[3] = n
    A = gen.make_csr(rng, m, n, np.minimum(L, n), "normal")
    nrm = np.sqrt(np.add.reduceat(A.vals ** 2, A.row_ptr[:-1]))
    A.vals = A.vals / np.repeat(nrm, np.diff(A.row_ptr))
    return gen.consistent(rng, A)


def long_cols_system(seed=33):
    """The transpose of a long-row matrix: columns of 300 and 1000 entries
    (summed by whole waves in the product with Aᵀ) beside short ones."""
    import scipy.sparse as sp
    B = long_rows_system(seed, m=1200, n=1500).A
    T = sp.csr_matrix(B.scipy().T)
    T.sort_indices()
    A = gen.CSR(T.shape[0], T.shape[1], T.indptr.astype(np.int64), T.indices.astype(np.int32),
                T.data.astype(np.float64))
    return gen.consistent(gen.rng_for(seed + 1), A)


def row_mix_system(seed=35, m=1063, n=1500):
    """Row lengths 0..64 mixed inside each slice of 64 rows (rows of exactly
    64 entries, the longest read from the slice layout; rows of 65 and 70,
    the shortest summed by whole waves), a last slice of 39 rows, rows scaled
    to unit norm; columns of every length up to about 60."""
    rng = gen.rng_for(seed)
    L = rng.integers(0, 65, size=m)
    L[::7] = 64
    L[5::11] = 65
    L[9::13] = 70
    L[2::17] = 0
    A = gen.make_csr(rng, m, n, L, "normal")
    nrm = np.sqrt(np.add.reduceat(A.vals ** 2, A.row_ptr[:-1]))
    nrm[np.diff(A.row_ptr) == 0] = 1.0
    A.vals = A.vals / np.repeat(nrm, np.diff(A.row_ptr))
    return gen.consistent(rng, A)


def test_small_engine_small_workload(h):
    """2000 x 1000, 8 entries per row, FP64, tol 1e-8: the oracle protocol."""
    say("single engine: small workload")
    sysm = gen.small()
    x, info, M = fp64_parity(h, sysm, engine="single", case="small_single_engine")
    assert info["relres_true"] <= 1.5e-8


@pytest.mark.parametrize("case", ["small", "wide", "long_rows", "long_cols", "row_mix", "W"])
def test_engines_agree(h, case):
    import paper_2207_07615_amd as plss
    say("engines agree", case)
    wi = None
    if case == "small":
        sysm = gen.small(m=3000, n=1500)
    elif case == "wide":
        sysm = gen.tiny(41, 400, 5000, 25)
    elif case == "long_rows":
        sysm = long_rows_system()
    elif case == "long_cols":
        sysm = long_cols_system()
    elif case == "row_mix":
        sysm = row_mix_system()
    else:
        sysm = gen.small(m=3000, n=1500)
        wi = np.sqrt(np.asarray(sysm.A.scipy().multiply(sysm.A.scipy()).sum(axis=0)).ravel())
    M = matrix(h, sysm.A)
    xs, i_s, hs = plss.solve(h, M, sysm.b, tol=1e-8, maxit=20000, wi=wi, engine="single")
    xm, i_m, hm = plss.solve(h, M, sysm.b, tol=1e-8, maxit=20000, wi=wi, engine="multi")
    assert i_s["status"] == 0 and i_m["status"] == 0, (i_s, i_m)
    assert abs(i_s["iters"] - i_m["iters"]) <= 1
    k = min(i_s["iters"], i_m["iters"])
    ref, spread = order_spread(sysm.A, sysm.b, k, wi=wi)
    xs_k, _, _ = plss.solve(h, M, sysm.b, tol=1e-300, maxit=k, wi=wi, engine="single")
    xm_k, _, _ = plss.solve(h, M, sysm.b, tol=1e-300, maxit=k, wi=wi, engine="multi")
    order_bound(rel(xs_k, ref.x), spread, f"engines_{case}_single")
    order_bound(rel(xm_k, ref.x), spread, f"engines_{case}_multi")
    # converged (relres 1e-13): both engines against the oracle at the flat 1e-10
    refc = O.plss_residual(sysm.A, sysm.b, tol=CONVERGED_TOL, maxit=200000, wi=wi)
    assert refc.status == O.OK
    for eng in ("single", "multi"):
        xc, ic, _ = plss.solve(h, M, sysm.b, tol=CONVERGED_TOL, maxit=200000, wi=wi, engine=eng)
        assert ic["status"] == 0, ic
        converged_check(xc, refc.x, f"engines_{case}_{eng}")
    # the first iterates (before rounding differences are amplified)
    x5, _, h5 = plss.solve(h, M, sysm.b, tol=1e-300, maxit=5, wi=wi, engine="single")
    r5 = O.plss_residual(sysm.A, sysm.b, tol=1e-300, maxit=5, wi=wi)
    assert rel(x5, r5.x) <= 1e-12
    np.testing.assert_allclose(h5[:6], r5.hist[:6], rtol=1e-10)


def test_small_engine_edge_cases(h):
    import paper_2207_07615_amd as plss
    say("single engine: edges")
    sysm = gen.small(m=400, n=200)
    M = matrix(h, sysm.A)
    kw = dict(engine="single")
    x, info, hist = plss.solve(h, M, np.zeros(400), tol=1e-8, maxit=10, **kw)
    assert info["iters"] == 0 and info["status"] == 0 and not np.any(x)
    x, info, hist = plss.solve(h, M, sysm.b, tol=1e-12, maxit=1, **kw)
    assert info["iters"] == 1 and info["status"] == 1
    ref = O.plss_residual(sysm.A, sysm.b, tol=1e-12, maxit=1)
    assert rel(x, ref.x) <= 1e-13
    np.testing.assert_allclose(hist[:2], ref.hist[:2], rtol=1e-12)
    b = sysm.b + np.random.default_rng(0).standard_normal(400)
    x, info, hist = plss.solve(h, M, b, tol=1e-12, maxit=300, **kw)
    assert info["status"] in (1, 2)
    x0 = np.random.default_rng(2).standard_normal(200)
    x, info, hist = plss.solve(h, M, sysm.b, tol=1e-10, maxit=500, x0=x0, **kw)
    ref = O.plss_residual(sysm.A, sysm.b, tol=1e-300, maxit=info["iters"], x0=x0)
    assert rel(x, ref.x) <= 1e-10
    # tiny over- and under-determined systems reach the minimum-norm solution
    from oracle import pins
    for m, n in [(20, 8), (8, 20), (64, 256)]:
        s2 = gen.tiny(500 + m + n, m, n, min(n, 30), "uniform")
        M2 = matrix(h, s2.A)
        x, info, _ = plss.solve(h, M2, s2.b, tol=1e-13, maxit=4000, **kw)
        assert info["status"] == 0
        assert rel(x, pins.min_norm(s2.A.dense(), s2.b)) <= 1e-9


def test_small_engine_fp32_refinement(h):
    import paper_2207_07615_amd as plss
    say("single engine: fp32 refine")
    sysm = gen.small(storage=np.float32)
    M = matrix(h, sysm.A, "f32")
    x, info, _ = plss.solve(h, M, sysm.b, tol=1e-12, maxit=5000, refine=True, inner_tol=1e-4,
                            engine="single")
    assert info["status"] == 0, info
    assert info["relres_true"] <= 1e-12
    assert info["outer_iters"] >= 2
    ref = O.plss_residual(sysm.A, sysm.b, tol=1e-13, maxit=5000)
    assert rel(x, ref.x) <= 1e-10
    xm, im, _ = plss.solve(h, M, sysm.b, tol=1e-12, maxit=5000, refine=True, inner_tol=1e-4,
                           engine="multi")
    assert im["outer_iters"] == info["outer_iters"]
    assert abs(im["iters"] - info["iters"]) <= 2
    x1, i1, _ = plss.solve(h, M, sysm.b, tol=1e-6, maxit=5000, refine=False, engine="single")
    assert 1e-9 < rel(x1, sysm.xstar) <= 1e-5


def test_small_engine_batch(h):
    """Small systems of a batch run as one persistent launch (one workgroup
    each) beside larger ones on the launch lists; every result equals the
    system's own solve bit for bit."""
    import paper_2207_07615_amd as plss
    say("single engine: batch")
    systems = gen.batch_systems(7, m_lo=1e3, m_hi=6e4)
    mats = [matrix(h, s.A) for s in systems]
    xs, infos = plss.solve_batch(h, mats, [s.b for s in systems], tol=1e-8, maxit=5000)
    for s, M, x, inf in zip(systems, mats, xs, infos):
        xa, ia, _ = plss.solve(h, M, s.b, tol=1e-8, maxit=5000)
        assert inf["status"] == 0
        assert inf["iters"] == ia["iters"]
        np.testing.assert_array_equal(x, xa)
        ref, spread = order_spread(s.A, s.b, inf["iters"])
        order_bound(rel(x, ref.x), spread, f"small_engine_batch_{s.A.m}x{s.A.n}")
    # converged batch (relres 1e-13) against the oracle at the flat 1e-10
    xs, infos = plss.solve_batch(h, mats, [s.b for s in systems], tol=CONVERGED_TOL, maxit=50000)
    for s, x, inf in zip(systems, xs, infos):
        assert inf["status"] == 0, inf
        ref = O.plss_residual(s.A, s.b, tol=CONVERGED_TOL, maxit=50000)
        assert ref.status == O.OK
        converged_check(x, ref.x, f"small_engine_batch_{s.A.m}x{s.A.n}")


def test_small_engine_deterministic(h):
    import paper_2207_07615_amd as plss
    say("single engine: determinism")
    sysm = gen.small()
    M = matrix(h, sysm.A)
    x1, i1, h1 = plss.solve(h, M, sysm.b, tol=1e-8, maxit=2000, engine="single")
    x2, i2, h2 = plss.solve(h, M, sysm.b, tol=1e-8, maxit=2000, engine="single")
    assert i1["iters"] == i2["iters"]
    np.testing.assert_array_equal(x1, x2)
    np.testing.assert_array_equal(h1, h2)


def test_engine_choice_errors(h):
    import paper_2207_07615_amd as plss
    say("engine errors")
    big = gen.tiny(7, 20000, 8000, 4)  # m + 2n = 36,000 float64 entries: beyond LDS
    M = matrix(h, big.A)
    with pytest.raises(plss.PlssError):
        plss.solve(h, M, big.b, tol=1e-8, maxit=10, engine="single")
    x, info, _ = plss.solve(h, M, big.b, tol=1e-8, maxit=10, engine="auto")
    assert info["iters"] == 10
    sysm = gen.small(m=400, n=200)
    M2 = matrix(h, sysm.A)
    with pytest.raises(plss.PlssError):
        plss.solve(h, M2, sysm.b, tol=1e-8, maxit=10, sketch="identity", engine="single")
