"""Striped layout of the two products of Algorithm 1 (row sums in LDS, the
gathered vector in stripes through LDS), against the oracle.

Products are checked entry by entry (float64 accumulation, tolerance a
small multiple of eps * (|A| |x|)); solves at equal iteration counts as in
the tile layout; unit sizes are forced small so that many units, ragged
last stripes, rows longer than a wave's window, empty rows and empty row
blocks all occur at sizes the oracle runs in seconds."""
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


def ragged(seed, m, n):
    """Empty rows, short rows, and rows of 4500 and 2048 entries (longer than
    a wave's 512-entry window inside one stripe)."""
    rng = gen.rng_for(seed)
    L = rng.integers(0, 12, size=m)
    L[rng.random(m) < 0.1] = 0
    L[:: max(1, m // 3)] = min(n, 4500)
    L[5] = min(n, 2048)
    return gen.make_csr(rng, m, n, np.minimum(L, n), "normal")


CASES = {
    # name: (matrix builder, unit_rows); units above 8192 rows apply to the
    # row-block stores of Aᵀ only (those of A hold at most 8192 rows)
    "ragged": (lambda: ragged(11, 9000, 13000), 37),
    "wide": (lambda: gen.tiny(4, 300, 20000, 30).A, 7),
    "dense_row": (lambda: gen.make_csr(gen.rng_for(9), 1, 9000, np.array([8000]), "normal"), 1),
    "zipf": (lambda: gen.large(m=60000, n=15000).A, 0),
    "one_unit": (lambda: gen.small(m=3000, n=1500).A, 8192),
    "big_t_units": (lambda: gen.tiny(6, 2000, 40000, 40).A, 16384),
    # vectors shorter than one staging load (the product with A gathers from
    # a vector of 1 or 3 entries; the transposed one scatters into it)
    "one_col": (lambda: gen.make_csr(gen.rng_for(12), 5000, 1, np.ones(5000, dtype=np.int64), "normal"), 64),
    "three_cols": (lambda: gen.make_csr(gen.rng_for(13), 7000, 3, np.full(7000, 2, dtype=np.int64), "normal"), 0),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_stripe_spmv_entrywise(h, case, storage):
    import paper_2207_07615_amd as plss
    say("stripe spmv", case, storage)
    build, R = CASES[case]
    A = build()
    M = matrix(h, A, storage)
    lay = M.layout(a_stripes=True, t_stripes=True, unit_rows=R)
    assert lay["a_stripes"] and lay["t_stripes"]
    if R:
        assert lay["unit_rows"] == min(R, 8192)
    S = A.astype(np.float32).scipy() if storage == "f32" else A.scipy()
    rng = np.random.default_rng(3)
    x = rng.standard_normal(A.n)
    u = rng.standard_normal(A.m)
    y = plss.spmv(h, M, x)
    yt = plss.spmv(h, M, u, transpose=True)
    absA = abs(S)
    assert np.all(abs(y - S @ x) <= 1e-14 * (absA @ abs(x)) + 1e-300)
    assert np.all(abs(yt - S.T @ u) <= 1e-14 * (absA.T @ abs(u)) + 1e-300)
    # the same products again: bit-identical (fixed summation order)
    np.testing.assert_array_equal(plss.spmv(h, M, x), y)
    np.testing.assert_array_equal(plss.spmv(h, M, u, transpose=True), yt)


def test_stripe_layout_control(h):
    import paper_2207_07615_amd as plss
    say("stripe layout")
    A = gen.small(m=3000, n=1500).A
    M = matrix(h, A)
    lay = M.layout()
    assert lay == {"a_stripes": False, "t_stripes": False, "unit_rows": 0}
    b0 = M.info()["device_bytes"]
    lay = M.layout(a_stripes=True, unit_rows=100)
    assert lay == {"a_stripes": True, "t_stripes": False, "unit_rows": 100}
    b1 = M.info()["device_bytes"]
    # the store of A holds at most 8192 rows per unit
    assert M.layout(a_stripes=True, unit_rows=12000)["unit_rows"] == 8192
    M.layout(a_stripes=True, unit_rows=100)
    assert b1 >= b0 + A.nnz * 12
    lay = M.layout(t_stripes=True, unit_rows=100)
    assert lay["a_stripes"] and lay["t_stripes"]
    b2 = M.info()["device_bytes"]
    with pytest.raises(plss.PlssError):
        M.layout(a_stripes=True, unit_rows=16385)
    with pytest.raises(plss.PlssError):
        M.layout(a_stripes=True, unit_rows=-1)
    lay = M.layout(a_stripes=False, t_stripes=False)
    assert not lay["a_stripes"] and not lay["t_stripes"]
    # the row blocks built for the transposed stripes stay; both striped
    # stores (at least 12 bytes per entry each) go
    assert M.info()["device_bytes"] <= b2 - 2 * A.nnz * 12
    # the tile path after the switch still gives the oracle's products
    x = np.random.default_rng(0).standard_normal(A.n)
    S = A.scipy()
    assert np.all(abs(plss.spmv(h, M, x) - S @ x) <= 1e-14 * (abs(S) @ abs(x)))


@pytest.mark.parametrize("R", [0, 64, 16384])
def test_stripe_solve_matches_oracle(h, R):
    """Zipf rows, 60000 x 15000: striped products in both directions."""
    say("stripe solve zipf", R)
    sysm = gen.large(m=60000, n=15000)
    x, info, M = fp64_parity(h, sysm, layout={"a_stripes": True, "t_stripes": True, "unit_rows": R},
                             case=f"zipf_60000x15000_stripes_R{R}")
    assert info["relres_true"] <= 1.5e-8


def test_stripe_solve_weighted_W(h):
    """PLSS W (Section 4.1) on the striped products: Zipf rows, 60000 x 15000,
    W = diag(1/||A_{:,j}||) (column norms spread by the heavy rows)."""
    say("stripe solve W")
    sysm = gen.large(m=60000, n=15000)
    S = sysm.A.scipy()
    wi = np.sqrt(np.asarray(S.multiply(S).sum(axis=0)).ravel())
    x, info, M = fp64_parity(h, sysm, wi=wi, layout={"a_stripes": True, "t_stripes": True},
                             case="zipf_60000x15000_stripes_W")
    assert info["relres_true"] <= 1.5e-8


def test_stripe_solve_ragged_matches_oracle(h):
    """Underdetermined ragged system (empty rows, rows of 4500 entries), rows
    scaled to unit norm (with N(0,1) values the long rows make the system so
    ill-conditioned that two float64 runs of the oracle differing only in
    summation order already part by 5e-4 after 15 iterations): the iterates
    follow the oracle's."""
    import paper_2207_07615_amd as plss
    say("stripe solve ragged")
    A = ragged(21, 3000, 9000)
    L = np.diff(A.row_ptr)
    norms = np.sqrt(np.add.reduceat(A.vals ** 2, A.row_ptr[:-1])) if A.nnz else np.ones(A.m)
    norms = np.where(L > 0, norms, 1.0)
    A.vals = A.vals / np.repeat(norms, L)
    rng = gen.rng_for(22)
    xstar = rng.standard_normal(A.n)
    b = gen.rhs(A, xstar)
    M = matrix(h, A)
    M.layout(a_stripes=True, t_stripes=True, unit_rows=37)
    x, info, _ = plss.solve(h, M, b, tol=1e-300, maxit=15)
    ref = O.plss_residual(A, b, tol=1e-300, maxit=15)
    assert rel(x, ref.x) <= 1e-12
    x, info, _ = plss.solve(h, M, b, tol=1e-8, maxit=20000)
    assert info["status"] == 0, info
    ref, spread = order_spread(A, b, info["iters"])
    order_bound(rel(x, ref.x), spread, "ragged_3000x9000_stripes")
    x, info, _ = plss.solve(h, M, b, tol=CONVERGED_TOL, maxit=50000)
    assert info["status"] == 0, info
    ref = O.plss_residual(A, b, tol=CONVERGED_TOL, maxit=50000)
    assert ref.status == O.OK
    converged_check(x, ref.x, "ragged_3000x9000_stripes")


def test_stripe_equals_tiles_first_iterates(h):
    """Both layouts compute the same iterates up to rounding."""
    import paper_2207_07615_amd as plss
    say("stripe vs tiles")
    sysm = gen.large(m=60000, n=15000)
    M = matrix(h, sysm.A)
    xt, it, ht = plss.solve(h, M, sysm.b, tol=1e-300, maxit=15)
    M.layout(a_stripes=True, t_stripes=True)
    xs, is_, hs = plss.solve(h, M, sysm.b, tol=1e-300, maxit=15)
    assert rel(xs, xt) <= 1e-12
    np.testing.assert_allclose(hs, ht, rtol=1e-10)


def test_stripe_fp32_refinement(h):
    """float32 striped store + float64 refinement reaches the float64 tolerance."""
    import paper_2207_07615_amd as plss
    say("stripe fp32 refine")
    sysm = gen.small(storage=np.float32)
    M = matrix(h, sysm.A, "f32")
    M.layout(a_stripes=True, t_stripes=True, unit_rows=64)
    x, info, _ = plss.solve(h, M, sysm.b, tol=1e-12, maxit=5000, refine=True, inner_tol=1e-4)
    assert info["status"] == 0, info
    assert info["relres_true"] <= 1e-12
    assert info["outer_iters"] >= 2
    ref = O.plss_residual(sysm.A, sysm.b, tol=1e-13, maxit=5000)
    assert rel(x, ref.x) <= 1e-10


def test_stripe_batch_mixed_layouts(h):
    """A batch of striped and tiled systems gives each system's own result
    bit for bit, as when solved alone."""
    import paper_2207_07615_amd as plss
    say("stripe batch")
    systems = gen.batch_systems(5, m_lo=1e3, m_hi=2e4)
    mats = [matrix(h, s.A) for s in systems]
    for i, M in enumerate(mats):
        if i % 2 == 0:
            M.layout(a_stripes=True, t_stripes=(i % 4 == 0), unit_rows=50 + i)
    xs, infos = plss.solve_batch(h, mats, [s.b for s in systems], tol=1e-8, maxit=5000)
    for s, M, x, inf in zip(systems, mats, xs, infos):
        xa, ia, _ = plss.solve(h, M, s.b, tol=1e-8, maxit=5000)
        assert inf["status"] == 0
        assert inf["iters"] == ia["iters"]
        np.testing.assert_array_equal(x, xa)


def test_stripe_deterministic(h):
    import paper_2207_07615_amd as plss
    say("stripe determinism")
    sysm = gen.large(m=60000, n=15000)
    M = matrix(h, sysm.A)
    M.layout(a_stripes=True, t_stripes=True, unit_rows=500)
    x1, i1, h1 = plss.solve(h, M, sysm.b, tol=1e-8, maxit=2000)
    x2, i2, h2 = plss.solve(h, M, sysm.b, tol=1e-8, maxit=2000)
    assert i1["iters"] == i2["iters"]
    np.testing.assert_array_equal(x1, x2)
    np.testing.assert_array_equal(h1, h2)


@pytest.mark.slow
def test_large_workload_first_iterates(h):
    """The 2,000,000 x 500,000 Zipf workload at full size, in the layout the
    benchmark runs (chosen at creation: striped in both directions): the first
    12 iterates match the oracle's, and sampled rows of A x match the oracle's
    row products computed one by one."""
    import paper_2207_07615_amd as plss
    say("large workload: generating")
    sysm = gen.large()
    M = matrix(h, sysm.A)
    lay = M.layout()
    say("large workload layout", lay)
    assert lay["a_stripes"] and lay["t_stripes"]
    x, info, hist = plss.solve(h, M, sysm.b, tol=1e-300, maxit=12)
    say("large workload: oracle")
    ref = O.plss_residual(sysm.A, sysm.b, tol=1e-300, maxit=12)
    assert rel(x, ref.x) <= 1e-12
    np.testing.assert_allclose(hist[:13], ref.hist[:13], rtol=1e-10)
    v = np.random.default_rng(4).standard_normal(sysm.A.n)
    y = plss.spmv(h, M, v)
    A = sysm.A
    for i in np.random.default_rng(5).choice(A.m, 200, replace=False):
        lo, hi = A.row_ptr[i], A.row_ptr[i + 1]
        want = float(np.dot(A.vals[lo:hi], v[A.col_idx[lo:hi]]))
        bound = 1e-14 * float(np.abs(A.vals[lo:hi]) @ np.abs(v[A.col_idx[lo:hi]]))
        assert abs(y[i] - want) <= bound
