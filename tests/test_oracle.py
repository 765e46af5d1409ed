"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own formulas: hand-worked
exact iterates, exact rational termination and orthogonality, the dense
brute-force update of eq. (pkLong), Craig's method (Section 6), textbook
Kaczmarz (Section 7) and the dense minimum-norm solution.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import plss_inputs as gen
from oracle import exact, pins
from oracle import plss as O
from oracle import sparse as osp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out[key] = [Fraction(v) for v in vals]
    return out


def to_f(v):
    return np.array([float(x) for x in v])


# ---------------------------------------------------------------- worked examples

def test_alg1_hand_worked_example_exact():
    g = load_golden("alg1_diag12.txt")
    A = np.array(to_f(g["A"])).reshape(2, 2)
    b = to_f(g["b"])
    x, rs, ps = exact.plss_residual_exact(A, b)
    assert ps[0] == g["p1"] and ps[1] == g["p2"]
    assert rs[1] == g["r1"] and rs[2] == g["r2"]
    assert x == g["x2"]


def test_alg1_hand_worked_example_float():
    g = load_golden("alg1_diag12.txt")
    A = np.array(to_f(g["A"])).reshape(2, 2)
    b = to_f(g["b"])
    res = O.plss_residual(A, b, tol=1e-14, maxit=10, record=True)
    assert res.status == O.OK and res.iters == 2
    np.testing.assert_allclose(res.ps[0], to_f(g["p1"]), rtol=1e-15)
    np.testing.assert_allclose(res.ps[1], to_f(g["p2"]), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(res.x, to_f(g["x2"]), rtol=1e-14)
    assert res.hist[0] == 1.0
    assert abs(res.hist[1] - math.sqrt(float(g["rho1"][0])) / math.sqrt(5)) < 1e-15


def test_kaczmarz_hand_worked_example():
    g = load_golden("kaczmarz_2x3.txt")
    A = to_f(g["A"]).reshape(2, 3)
    b = to_f(g["b"])
    order = [int(v) for v in g["order"]]
    x, rs, ps = exact.plss_columns_exact(A, b, [("e", i) for i in order])
    assert ps[0] == g["p1"] and ps[1] == g["p2"] and x == g["x2"]
    assert x == exact.min_norm_exact(A, b)
    res = O.plss_columns(A, b, "identity", perm=np.array(order), tol=1e-15, maxit=2,
                         record=True)
    np.testing.assert_allclose(res.xs[1], to_f(g["x1"]), rtol=1e-15)
    np.testing.assert_allclose(res.x, to_f(g["x2"]), rtol=1e-15)
    kz = pins.kaczmarz(A, b, order)
    np.testing.assert_allclose(kz[0], to_f(g["x1"]), rtol=1e-15)
    np.testing.assert_allclose(kz[1], to_f(g["kaczmarz_x2"]), rtol=1e-15)


# ---------------------------------------------------------------- exact termination

@pytest.mark.parametrize("m,n,seed", [(7, 4, 1), (5, 5, 2), (4, 8, 3), (9, 3, 4)])
def test_exact_termination_and_orthogonality(m, n, seed):
    """Theorem 1 / Corollary 2 and eq. (orthogonal-updates): in exact
    arithmetic r reaches 0 after at most min(m, n) updates, x = A†b, and all
    residuals and all updates are mutually orthogonal."""
    sysm = gen.tiny_integer(seed, m, n, min(n, 3))
    A = sysm.A.dense()
    x, rs, ps = exact.plss_residual_exact(A, sysm.b)
    assert all(v == 0 for v in rs[-1])
    assert len(ps) <= min(m, n)
    if np.linalg.matrix_rank(A) == min(m, n):
        assert x == exact.min_norm_exact(A, sysm.b)
    for i in range(len(rs)):
        for j in range(i):
            assert exact.dot(rs[i], rs[j]) == 0
    for i in range(len(ps)):
        for j in range(i):
            assert exact.dot(ps[i], ps[j]) == 0


def test_gamma_reading_is_the_only_orthogonal_one():
    """The gamma printed with Theorem 2 (eq. pkShort) equals Algorithm 1's
    gamma divided by rho.  Planting that form breaks residual orthogonality,
    which confirms Algorithm 1's gamma = (theta/rho)*beta."""
    sysm = gen.tiny_integer(11, 6, 4, 3)
    A = exact.mat(sysm.A.dense()); b = exact.vec(sysm.b)
    r = list(b); rho = exact.dot(r, r)
    y = exact.mtv(A, r); phi = exact.dot(y, y)
    p = [(rho / phi) * v for v in y]; theta = exact.dot(p, p)
    r1 = exact.axpy(Fraction(-1), exact.mv(A, p), r)
    rho1 = exact.dot(r1, r1)
    assert exact.dot(r1, r) == 0
    y = exact.mtv(A, r1); phi = exact.dot(y, y)
    den = theta * phi - rho1 * rho1
    beta = rho1 * rho1 / den
    for gamma, ok in ((theta * rho1 / den, True), (theta / den, False)):
        p2 = [beta * a + gamma * c for a, c in zip(p, y)]
        r2 = exact.axpy(Fraction(-1), exact.mv(A, p2), r1)
        assert (exact.dot(r2, r1) == 0) == ok
        assert (exact.dot(p2, p) == 0) == ok


def test_float_oracle_matches_exact_run():
    sysm = gen.tiny_integer(5, 12, 6, 3)
    A = sysm.A.dense()
    x, rs, ps = exact.plss_residual_exact(A, sysm.b)
    res = O.plss_residual(A, sysm.b, tol=0.0, maxit=len(ps), record=True)
    for k, p in enumerate(ps):
        np.testing.assert_allclose(res.ps[k], to_f(p), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(res.x, to_f(x), rtol=1e-11)


@pytest.mark.parametrize("m,n,seed", [(4, 7, 21), (5, 9, 22), (3, 3, 23)])
def test_identity_sketch_exact_corollary2(m, n, seed):
    """Corollary 2: with m <= n, full row rank and a full pass of identity
    columns, x_m = A†b exactly (x0 = 0 keeps x in range(Aᵀ))."""
    sysm = gen.tiny_integer(seed, m, n, min(n, 3))
    A = sysm.A.dense()
    if np.linalg.matrix_rank(A) < m:
        pytest.skip("rank deficient draw")
    cols = [("e", int(i)) for i in sysm.perm]
    x, rs, ps = exact.plss_columns_exact(A, sysm.b, cols)
    assert x == exact.min_norm_exact(A, sysm.b)
    for i in range(len(ps)):
        for j in range(i):
            assert exact.dot(ps[i], ps[j]) == 0


def test_mixed_sketch_exact_termination():
    """Mixed sketch (residual and identity columns interleaved): exact
    termination within rank(A) updates and orthogonal updates."""
    sysm = gen.tiny_integer(31, 8, 5, 3)
    A = sysm.A.dense()
    cols = []
    for i in sysm.perm:
        cols += [("r",), ("e", int(i))]
    x, rs, ps = exact.plss_columns_exact(A, sysm.b, cols)
    assert all(v == 0 for v in rs[-1])
    assert len(ps) <= np.linalg.matrix_rank(A)
    for i in range(len(ps)):
        for j in range(i):
            assert exact.dot(ps[i], ps[j]) == 0


def test_exact_column_step_residual_equals_alg1():
    """With residual columns only, the general column step is Algorithm 1."""
    sysm = gen.tiny_integer(41, 7, 5, 3)
    A = sysm.A.dense()
    x1, _, ps1 = exact.plss_residual_exact(A, sysm.b)
    x2, _, ps2 = exact.plss_columns_exact(A, sysm.b, [("r",)] * 10)
    assert ps1 == ps2 and x1 == x2


# ---------------------------------------------------------------- brute force / Craig

@pytest.mark.parametrize("m,n", [(30, 12), (12, 30), (20, 20)])
def test_residual_updates_match_bruteforce_pklong(m, n):
    """eq. (pkLong) with S_k = [r_0 .. r_{k-1}] (eq. S) equals Algorithm 1's p_k."""
    sysm = gen.tiny(100 + m, m, n, 5)
    A = sysm.A.dense()
    res = O.plss_residual(A, sysm.b, tol=0.0, maxit=8, record=True)
    for k in range(1, len(res.ps) + 1):
        Sk = np.column_stack(res.rs[:k])
        pk = pins.pk_bruteforce(A, Sk, res.rs[k - 1])
        assert np.linalg.norm(pk - res.ps[k - 1]) <= 1e-12 * np.linalg.norm(pk)


def test_residual_sketch_weighted_matches_bruteforce():
    """eq. (pkShortW) / Section 4.1: the recursion with a diagonal W equals
    eq. (pkLong) with that W."""
    sysm = gen.tiny(7, 25, 10, 4)
    A = sysm.A.dense()
    wi = np.linalg.norm(A, axis=0)              # BᵀB = diag(||A_{:,j}||)
    res = O.plss_residual(A, sysm.b, tol=0.0, maxit=6, wi=wi, record=True)
    W = np.diag(1.0 / wi)
    for k in range(1, len(res.ps) + 1):
        Sk = np.column_stack(res.rs[:k])
        pk = pins.pk_bruteforce(A, Sk, res.rs[k - 1], W)
        assert np.linalg.norm(pk - res.ps[k - 1]) <= 1e-11 * np.linalg.norm(pk)


@pytest.mark.parametrize("m,n", [(40, 15), (15, 40)])
def test_residual_sketch_equals_craig(m, n):
    """Section 6: with W = I the iterates are Craig's iterates."""
    sysm = gen.tiny(200 + m, m, n, 6)
    A = sysm.A.dense()
    res = O.plss_residual(A, sysm.b, tol=0.0, maxit=10, record=True)
    cx = pins.craig(A, sysm.b, 10)
    for k in range(10):
        assert np.linalg.norm(cx[k] - res.xs[k + 1]) <= 1e-10 * np.linalg.norm(cx[k])


@pytest.mark.parametrize("sketch", ["identity", "mixed"])
def test_column_sketch_matches_bruteforce(sketch):
    """Identity and mixed sketches: every iterate equals the closed-form
    projection onto the sketch used so far (nested projections from
    eqs. itProb-cons): x_k = Aᵀ S (Sᵀ A Aᵀ S)^† Sᵀ b with x0 = 0."""
    sysm = gen.tiny(300, 14, 22, 5)
    A = sysm.A.dense()
    res = O.plss_columns(A, sysm.b, sketch, perm=sysm.perm, tol=0.0, maxit=10,
                         record=True)
    cols = []
    rk = 0
    for k, col in enumerate(res.columns):
        if col[0] == "r":
            cols.append(res.rs[k])
        else:
            e = np.zeros(A.shape[0]); e[col[1]] = 1.0
            cols.append(e)
        Sk = np.column_stack(cols)
        xb = pins.x_bruteforce(A, Sk, sysm.b)
        assert np.linalg.norm(xb - res.xs[k + 1]) <= 1e-10 * np.linalg.norm(xb)


def test_mixed_two_column_block_equals_two_single_steps():
    """Appending r and e_i in one block gives the same iterate as two single
    appends (the iterates are nested projections)."""
    sysm = gen.tiny(301, 16, 24, 5)
    A = sysm.A.dense()
    res = O.plss_columns(A, sysm.b, "mixed", perm=sysm.perm, tol=0.0, maxit=2,
                         record=True)
    e = np.zeros(16); e[res.columns[1][1]] = 1.0
    S2 = np.column_stack([sysm.b, e])          # r_0 = b, then e_{π0}
    x = pins.x_bruteforce(A, S2, sysm.b)
    np.testing.assert_allclose(res.xs[2], x, rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------- Kaczmarz

def test_identity_first_step_is_kaczmarz():
    sysm = gen.tiny(400, 30, 12, 5)
    A = sysm.A.dense()
    res = O.plss_columns(A, sysm.b, "identity", perm=sysm.perm, tol=0.0, maxit=1,
                         record=True)
    kz = pins.kaczmarz(A, sysm.b, [int(sysm.perm[0])])
    np.testing.assert_allclose(res.x, kz[0], rtol=1e-14, atol=1e-15)


def test_identity_orthogonal_rows_equals_kaczmarz():
    """Mutually orthogonal rows (disjoint supports): every PLSS KZ step equals
    the Kaczmarz step (Section 7, history term vanishes)."""
    m, n = 6, 18
    rng = np.random.default_rng(5)
    A = np.zeros((m, n))
    cols = rng.permutation(n)
    for i in range(m):
        A[i, cols[3 * i:3 * i + 3]] = rng.standard_normal(3)
    b = A @ rng.standard_normal(n)
    order = rng.permutation(m)
    res = O.plss_columns(A, b, "identity", perm=order, tol=0.0, maxit=m, record=True)
    kz = pins.kaczmarz(A, b, order)
    for k in range(m):
        np.testing.assert_allclose(res.xs[k + 1], kz[k], rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------- skipped columns

def _dependent_rows_system(eps=1e-3, seed=17):
    """6 x 9 system whose identity columns hit every branch of the skip rule
    (Section 7, eq. pkKacz; rank(S_k) = k of eq. seqS):
      row 1 = row 0 (a repeated row),
      row 3 = row 0 + row 2 (supports disjoint, so the float sum is exact),
      row 5 = row 2 + row 4 + eps e_8 (nearly dependent: delta = eps^2 in
      exact arithmetic, between 1e-14 and 1e-6 times ||a_5||^2).
    Values are not dyadic, so the float residual at a dependent row is a
    rounding remainder, not an exact zero."""
    rng = np.random.default_rng(seed)
    A = np.zeros((6, 9))
    A[0, [0, 1]] = rng.standard_normal(2)
    A[2, [2, 3, 4]] = rng.standard_normal(3)
    A[4, [5, 6, 7]] = rng.standard_normal(3)
    A[1] = A[0]
    A[3] = A[0] + A[2]
    A[5] = A[2] + A[4]
    A[5, 8] = eps
    xs = rng.standard_normal(9)
    return A, A @ xs


def test_identity_skip_rule_matches_exact_twin():
    """The float oracle leaves out exactly the columns the rational run leaves
    out: the repeated row and the exactly dependent row are skipped, the
    nearly dependent row (delta/||a||^2 ~ 1e-11) is an update.  Skipped
    columns are not counted, and one pass gives A†b (Corollary 2 on the
    independent rows, whose constraints imply the others)."""
    A, b = _dependent_rows_system()
    ratio = 1e-6 / (A[5] @ A[5])            # delta / ||a_5||^2 of the last row
    assert 1e-12 < ratio < 1e-6
    used = []
    xe, rs_e, ps_e = exact.plss_columns_exact(A, b, [("e", i) for i in range(6)], used=used)
    assert used == [("e", 0), ("e", 2), ("e", 4), ("e", 5)]
    res = O.plss_columns(A, b, "identity", perm=np.arange(6), tol=1e-300, maxit=6,
                         max_columns=6, record=True)
    assert [tuple(c) for c in res.columns] == used
    assert res.iters == 4 and len(res.ps) == 4
    # the float residual at rows 1 and 3 is not exactly zero when they are
    # examined, so their skip is the delta branch of the rule
    assert res.rs[1][1] != 0.0 or res.rs[2][3] != 0.0
    # delta of the last row is a difference of two numbers of size ||a_5||^2
    # that agree to ~6 digits, so ~1e-10 is what float64 leaves of it
    x_exact = np.array([float(v) for v in xe])
    assert np.linalg.norm(res.x - x_exact) <= 1e-8 * np.linalg.norm(x_exact)
    xm = pins.min_norm(A[[0, 2, 4, 5]], b[[0, 2, 4, 5]])
    assert np.linalg.norm(res.x - xm) <= 1e-8 * np.linalg.norm(xm)


def test_identity_skip_rule_hand_worked_exact():
    """Integer system with a repeated row and a dependent row, worked by hand:
    x* = (1,2,3,4,5), rows a0 = (1,1,0,0,0), a1 = a0, a2 = (0,0,1,2,0),
    a3 = a0 + a2, a4 = e_5; order 0,1,2,3,4.
      col 0: sigma = 3, delta = 2, p = (3/2)(1,1,0,0,0)
      col 1: r_1 = 0 -> skipped
      col 2: sigma = 11, w = 0, delta = 5, p = (11/5)(0,0,1,2,0)
      col 3: r_3 = 0 -> skipped
      col 4: sigma = 5, delta = 1, p = 5 e_5, then r = 0.
    Three updates, x = (3/2, 3/2, 11/5, 22/5, 5) = A†b."""
    A = np.array([[1, 1, 0, 0, 0], [1, 1, 0, 0, 0], [0, 0, 1, 2, 0], [1, 1, 1, 2, 0],
                  [0, 0, 0, 0, 1]], dtype=float)
    b = A @ np.array([1, 2, 3, 4, 5], dtype=float)
    used = []
    x, rs, ps = exact.plss_columns_exact(A, b, [("e", i) for i in range(5)], used=used)
    assert used == [("e", 0), ("e", 2), ("e", 4)]
    F = Fraction
    assert ps[0] == [F(3, 2), F(3, 2), 0, 0, 0]
    assert ps[1] == [0, 0, F(11, 5), F(22, 5), 0]
    assert ps[2] == [0, 0, 0, 0, F(5)]
    assert x == [F(3, 2), F(3, 2), F(11, 5), F(22, 5), F(5)]
    res = O.plss_columns(A, b, "identity", perm=np.arange(5), tol=1e-14, maxit=5, record=True)
    assert res.status == O.OK and res.iters == 3
    assert [tuple(c) for c in res.columns] == used
    np.testing.assert_allclose(res.x, [1.5, 1.5, 2.2, 4.4, 5.0], rtol=1e-14)


def test_mixed_skip_rule_matches_exact_twin():
    """Mixed sketch on the dependent-rows system: the identity columns it
    skips are those the rational run skips, and the update count agrees."""
    A, b = _dependent_rows_system(seed=23)
    cols = []
    for i in range(6):
        cols += [("r",), ("e", i)]
    used = []
    exact.plss_columns_exact(A, b, cols, used=used)
    res = O.plss_columns(A, b, "mixed", perm=np.arange(6), tol=1e-300, maxit=len(used),
                         max_columns=len(used) + 20, record=True)
    assert [tuple(c) for c in res.columns][:len(used)] == used
    assert res.iters == len(used)


# ---------------------------------------------------------------- limits

@pytest.mark.parametrize("m,n,L", [(20, 8, 4), (8, 20, 4), (64, 256, 30), (60, 60, 6)])
@pytest.mark.parametrize("sketch", ["residual", "identity", "mixed"])
def test_converges_to_min_norm(m, n, L, sketch):
    """x0 = 0: the limit is A†b (Theorem 1, Corollaries 1-2)."""
    sysm = gen.tiny(500 + m + n, m, n, L, "uniform")
    A = sysm.A.dense()
    res = O.plss(A, sysm.b, sketch, perm=sysm.perm, tol=1e-13, maxit=4000)
    assert res.status == O.OK, (res.status, res.iters)
    xm = pins.min_norm(A, sysm.b)
    assert np.linalg.norm(res.x - xm) <= 1e-9 * np.linalg.norm(xm)
    if m >= n and np.linalg.matrix_rank(A) == n:
        assert np.linalg.norm(res.x - sysm.xstar) <= 1e-9 * np.linalg.norm(sysm.xstar)


def test_small_workload_converges():
    sysm = gen.small()
    res = O.plss_residual(sysm.A, sysm.b, tol=1e-8, maxit=1000)
    assert res.status == O.OK and res.iters < 200
    assert res.relres_true <= 2e-8
    assert np.linalg.norm(res.x - sysm.xstar) <= 1e-6 * np.linalg.norm(sysm.xstar)


# ---------------------------------------------------------------- edge cases

def test_zero_rhs_returns_x0_without_updates():
    A = gen.tiny(1, 5, 4, 2).A.dense()
    res = O.plss_residual(A, np.zeros(5), tol=1e-8, maxit=10)
    assert res.iters == 0 and res.status == O.OK and not res.x.any()


def test_maxit_one_and_not_converged():
    sysm = gen.tiny(2, 30, 20, 5)
    res = O.plss_residual(sysm.A, sysm.b, tol=1e-14, maxit=1)
    assert res.iters == 1 and res.status == O.NOT_CONVERGED and len(res.hist) == 2


def test_inconsistent_rhs_breaks_down_or_stalls():
    sysm = gen.tiny(3, 30, 5, 3)
    b = sysm.b + np.random.default_rng(0).standard_normal(30)
    res = O.plss_residual(sysm.A, b, tol=1e-12, maxit=500)
    assert res.status in (O.BREAKDOWN, O.NOT_CONVERGED)


# ---------------------------------------------------------------- sparse helpers

def test_csc_transpose_definition():
    sysm = gen.tiny(9, 40, 25, 6)
    A = sysm.A
    cp, ri, cv = osp.csr_to_csc(A.m, A.n, A.row_ptr, A.col_idx, A.vals)
    D = A.dense()
    for j in range(A.n):
        rows = ri[cp[j]:cp[j + 1]]
        assert np.all(np.diff(rows) > 0)
        np.testing.assert_array_equal(rows, np.nonzero(D[:, j])[0])
        np.testing.assert_array_equal(cv[cp[j]:cp[j + 1]], D[rows, j])
    S = A.scipy().tocsc()
    S.sort_indices()
    np.testing.assert_array_equal(cp, S.indptr)
    np.testing.assert_array_equal(ri, S.indices)


def test_csc_transpose_with_empty_rows_and_columns():
    row_ptr = np.array([0, 0, 2, 2, 3], dtype=np.int64)
    col = np.array([1, 4, 1], dtype=np.int32)
    vals = np.array([1.0, 2.0, 3.0])
    cp, ri, cv = osp.csr_to_csc(4, 6, row_ptr, col, vals)
    np.testing.assert_array_equal(cp, [0, 0, 2, 2, 2, 3, 3])
    np.testing.assert_array_equal(ri, [1, 3, 1])
    np.testing.assert_array_equal(cv, [1.0, 3.0, 2.0])


@pytest.mark.parametrize("bad", ["ptr_dec", "col_range", "col_dup", "col_unsorted", "nan"])
def test_csr_validation(bad):
    row_ptr = np.array([0, 2, 4], dtype=np.int64)
    col = np.array([0, 2, 1, 3], dtype=np.int32)
    vals = np.ones(4)
    if bad == "ptr_dec":
        row_ptr = np.array([0, 3, 2], dtype=np.int64); col = col[:2]; vals = vals[:2]
    elif bad == "col_range":
        col = np.array([0, 2, 1, 4], dtype=np.int32)
    elif bad == "col_dup":
        col = np.array([0, 0, 1, 3], dtype=np.int32)
    elif bad == "col_unsorted":
        col = np.array([2, 0, 1, 3], dtype=np.int32)
    elif bad == "nan":
        vals = np.array([1.0, np.nan, 1.0, 1.0])
    with pytest.raises(osp.CSRError):
        osp.validate_csr(2, 4, row_ptr, col, vals)
    osp.validate_csr(2, 4, np.array([0, 2, 4]), np.array([0, 2, 1, 3]), np.ones(4))


# ---------------------------------------------------------------- generators

def test_generators_deterministic_and_well_formed():
    a = gen.small(seed=123, m=300, n=100)
    b = gen.small(seed=123, m=300, n=100)
    np.testing.assert_array_equal(a.A.col_idx, b.A.col_idx)
    np.testing.assert_array_equal(a.A.vals, b.A.vals)
    np.testing.assert_array_equal(a.b, b.b)
    osp.validate_csr(a.A.m, a.A.n, a.A.row_ptr, a.A.col_idx, a.A.vals)
    c = gen.large(seed=5, m=20000, n=5000)
    osp.validate_csr(c.A.m, c.A.n, c.A.row_ptr, c.A.col_idx, c.A.vals)
    L = np.diff(c.A.row_ptr)
    assert L.min() >= 2 and L.max() <= 2000
