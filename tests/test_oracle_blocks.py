"""Pins of the block-sketch oracle (``oracle.blocks``: the triangular update
of Section 2.4 taken a block of columns at a time) against what the paper
and the mathematics fix:

* brute-force eq. (pkLong) / the closed form of the iterate for the
  accumulated block sketch (nested projections), also across history clears;
* one column per block reduces to the one-column identity and mixed steps;
* exact rational termination (Theorem 1, Corollary 2) and orthogonal updates
  (Section 2.5) in the rational twin, which the float oracle follows;
* the column drop rule on repeated and dependent rows, against the rational
  twin;
* limits: A†b after a full pass on full-row-rank systems."""
import numpy as np
import pytest

import plss_inputs as gen
from oracle import blocks as B
from oracle import exact as E
from oracle import pins
from oracle import plss as O


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def sketch_matrix(m, cols_so_far, rs, step_of_col):
    """Explicit S (m x q) from the oracle's recorded columns: a residual
    column is the residual at the start of its step, e_i the unit vector."""
    S = np.zeros((m, len(cols_so_far)))
    for q, (c, k) in enumerate(zip(cols_so_far, step_of_col)):
        if c[0] == "r":
            S[:, q] = rs[k]
        else:
            S[c[1], q] = 1.0
    return S


@pytest.mark.parametrize("block,residual", [(3, False), (3, True), (5, True), (1, True)])
def test_block_iterates_equal_bruteforce(block, residual):
    """Every iterate before the first history clear is the closed form
    x_k = Aᵀ S_k (S_kᵀ A Aᵀ S_k)^† S_kᵀ b of the accumulated block sketch
    (eq. pkLong applied to nested projections from x0 = 0), and every update
    is brute-force eq. (pkLong) on r_{k-1} with that sketch."""
    sysm = gen.tiny(301 + block, 24, 40, 8)
    D = sysm.A.dense()
    w = block + (1 if residual else 0)
    steps = min(24 // block, 24 // w) - 1
    res = B.plss_blocks(sysm.A, sysm.b, block=block, residual=residual, perm=sysm.perm, tol=1e-300,
                        maxit=steps, record=True)
    assert res.iters == steps
    cols, owner = [], []
    for k in range(1, steps + 1):
        used = res.columns[k - 1]
        assert len(used) == w                       # random data: no column left out
        cols += used
        owner += [k - 1] * len(used)
        S = sketch_matrix(24, cols, res.rs, owner)
        assert rel(res.xs[k], pins.x_bruteforce(D, S, sysm.b)) <= 1e-10
        assert rel(res.ps[k - 1], pins.pk_bruteforce(D, S, res.rs[k - 1])) <= 1e-10


def test_block_iterates_after_history_clears():
    """With a history cap of two blocks, the history is cleared every second
    step; each stretch is the closed form started from the iterate at the
    clear: x = x_c + Aᵀ S (Sᵀ A Aᵀ S)^† Sᵀ (b - A x_c)."""
    sysm = gen.tiny(311, 30, 45, 8)
    D = sysm.A.dense()
    res = B.plss_blocks(sysm.A, sysm.b, block=3, residual=True, perm=sysm.perm, tol=1e-300, maxit=7,
                        hist_cap=8, record=True)
    assert res.iters == 7
    for k in range(1, 8):
        start = 2 * ((k - 1) // 2)                  # step index where this stretch began
        cols, owner = [], []
        for j in range(start + 1, k + 1):
            cols += res.columns[j - 1]
            owner += [j - 1] * len(res.columns[j - 1])
        S = sketch_matrix(30, cols, res.rs, owner)
        assert rel(res.xs[k], pins.x_bruteforce(D, S, sysm.b, x0=res.xs[start])) <= 1e-10


def test_block_history_cleared_at_pass_end():
    """Blocks of 3 rows plus r (4 columns) on 30 rows with room for 3 blocks:
    the history is cleared before steps 4, 7, 10 (the cap) and after step 10
    (the end of the pass), so the stretches start at steps 0, 3, 6, 9, 10,
    13; each stretch is the closed form from the iterate where it began."""
    sysm = gen.tiny(313, 30, 45, 8)
    D = sysm.A.dense()
    res = B.plss_blocks(sysm.A, sysm.b, block=3, residual=True, perm=sysm.perm, tol=1e-300, maxit=15,
                        hist_cap=12, record=True)
    assert res.iters == 15
    starts = [0, 3, 6, 9, 10, 13]
    for k in range(1, 16):
        start = max(s for s in starts if s <= k - 1)
        cols, owner = [], []
        for j in range(start + 1, k + 1):
            cols += res.columns[j - 1]
            owner += [j - 1] * len(res.columns[j - 1])
        S = sketch_matrix(30, cols, res.rs, owner)
        assert rel(res.xs[k], pins.x_bruteforce(D, S, sysm.b, x0=res.xs[start])) <= 1e-10


def test_block_keeps_a_nearly_dependent_row():
    """Rows w, z and w + z + 2^-10 e_c in one block: the third row's pivot is
    about 1e-7 of its squared norm, a new direction the rational twin keeps
    (pivot not zero); so does the float oracle, and it matches the twin to
    within the rounding that a pivot of 1e-7 amplifies (about 1e7 eps)."""
    rng = np.random.default_rng(372)
    D = np.zeros((6, 14))
    D[0, [0, 1, 2, 3]] = rng.integers(1, 4, 4)
    D[1, [4, 5, 6, 7]] = rng.integers(1, 4, 4)
    D[2] = D[0] + D[1]
    D[2, 8] = 2.0 ** -10
    for i in (3, 4, 5):
        D[i, rng.choice(14, 4, replace=False)] = rng.integers(1, 4, 4)
    b = D @ rng.integers(-2, 3, 14).astype(np.float64)
    used_e = []
    x, rs, ps = E.plss_blocks_exact(D, b, blocks_of(np.arange(6), 3, False, 2), used=used_e)
    assert used_e == [[("e", 0), ("e", 1), ("e", 2)], [("e", 3), ("e", 4), ("e", 5)]]
    f = B.plss_blocks(D, b, block=3, residual=False, perm=np.arange(6), tol=1e-300, maxit=2, record=True)
    assert [[tuple(c) for c in u] for u in f.columns] == used_e
    assert rel(f.x, [float(v) for v in x]) <= 1e-7


def test_block_of_one_identity_column_is_plss_kaczmarz():
    sysm = gen.tiny(321, 30, 60, 8)
    a = B.plss_blocks(sysm.A, sysm.b, block=1, residual=False, perm=sysm.perm, tol=1e-300, maxit=40,
                      record=True)
    c = O.plss_columns(sysm.A, sysm.b, "identity", perm=sysm.perm, tol=1e-300, maxit=40, record=True)
    assert a.iters == c.iters == 40
    for xa, xc in zip(a.xs, c.xs):
        assert rel(xa, xc) <= 1e-12


def test_mixed_block_of_one_row_is_two_mixed_columns():
    """A block [r_{k-1}, e_i] gives the iterate of the one-column mixed
    sketch after its residual column and its identity column (iterates
    depend only on the span of the sketch)."""
    sysm = gen.tiny(331, 40, 70, 8)
    a = B.plss_blocks(sysm.A, sysm.b, block=1, residual=True, perm=sysm.perm, tol=1e-300, maxit=15,
                      record=True)
    c = O.plss_columns(sysm.A, sysm.b, "mixed", perm=sysm.perm, tol=1e-300, maxit=30, record=True)
    assert [u[0] for u in c.columns] == ["r", "e"] * 15   # no column skipped
    for k in range(1, 16):
        assert rel(a.xs[k], c.xs[2 * k]) <= 1e-10


def test_block_steps_equal_single_steps_of_the_same_columns():
    """A block of 4 identity columns gives the iterate of 4 one-column
    identity steps (same span), step after step."""
    sysm = gen.tiny(341, 32, 50, 8)
    a = B.plss_blocks(sysm.A, sysm.b, block=4, residual=False, perm=sysm.perm, tol=1e-300, maxit=7,
                      record=True)
    c = O.plss_columns(sysm.A, sysm.b, "identity", perm=sysm.perm, tol=1e-300, maxit=28, record=True)
    for k in range(1, 8):
        assert rel(a.xs[k], c.xs[4 * k]) <= 1e-10


def integer_system(seed, m, n, L):
    s = gen.tiny_integer(seed, m, n, L)
    return s.A.dense(), s.b, s.perm


def blocks_of(perm, block, residual, nsteps):
    out = []
    m = len(perm)
    pos = 0
    for _ in range(nsteps):
        rows = [int(i) for i in perm[pos:min(pos + block, m)]]
        pos += len(rows)
        out.append(([("r",)] if residual else []) + [("e", i) for i in rows])
        if pos >= m:
            out.append(("clear",))
            pos = 0
    return out


@pytest.mark.parametrize("block", [2, 3])
def test_block_exact_termination_underdetermined(block):
    """Corollary 2 with block identity sketches: on a full-row-rank integer
    system (m < n), one pass of blocks gives A†b exactly in rationals; the
    float oracle follows the rational iterates and reaches A†b."""
    D, b, perm = integer_system(351, 6, 10, 4)
    assert np.linalg.matrix_rank(D) == 6
    nsteps = -(-6 // block)
    x, rs, ps = E.plss_blocks_exact(D, b, blocks_of(perm, block, False, nsteps))
    xm = E.min_norm_exact(D, b)
    assert x == xm
    assert all(v == 0 for v in rs[-1])
    for i in range(len(ps)):
        for j in range(i):
            assert E.dot(ps[i], ps[j]) == 0
    f = B.plss_blocks(D, b, block=block, residual=False, perm=perm, tol=1e-300, maxit=nsteps, record=True)
    for k, pk in enumerate(ps):
        assert rel(f.ps[k], [float(v) for v in pk]) <= 1e-12
    assert rel(f.x, [float(v) for v in xm]) <= 1e-12


def test_block_exact_termination_mixed_overdetermined():
    """Mixed blocks [r, e_i, e_j] on a full-column-rank consistent integer
    system (m > n): the residual vanishes exactly within n columns' worth of
    rank, and x = x*."""
    s = gen.tiny_integer(361, 9, 5, 3)
    D = s.A.dense()
    assert np.linalg.matrix_rank(D) == 5
    x, rs, ps = E.plss_blocks_exact(D, s.b, blocks_of(s.perm, 2, True, 5))
    assert all(v == 0 for v in rs[-1])
    assert [float(v) for v in x] == list(s.xstar)
    assert len(ps) <= 5
    for i in range(len(ps)):
        for j in range(i):
            assert E.dot(ps[i], ps[j]) == 0


def dependent_block_system():
    """Integer rows on 12 columns: row 2 repeats row 0, row 3 = row 0 + row 1,
    rows 4-7 generic, row 8 = row 4 - row 5 (dependent on a previous block)."""
    rng = np.random.default_rng(371)
    D = np.zeros((9, 12))
    for i in (0, 1, 4, 5, 6, 7):
        D[i, rng.choice(12, 4, replace=False)] = rng.integers(1, 4, 4) * rng.choice([-1, 1], 4)
    D[2] = D[0]
    D[3] = D[0] + D[1]
    D[8] = D[4] - D[5]
    xs = rng.integers(-2, 3, 12).astype(np.float64)
    return D, D @ xs


def test_block_drop_rule_against_rational_twin():
    """Rows that repeat or combine rows of the same block, or of an earlier
    block, are left out of the sketch: exactly the columns the rational twin
    leaves out (pivot exactly zero); the float oracle keeps the rest and
    reaches A†b after the pass."""
    D, b = dependent_block_system()
    perm = np.arange(9)
    blocks = blocks_of(perm, 4, False, 3)
    used_e = []
    x, rs, ps = E.plss_blocks_exact(D, b, blocks, used=used_e)
    assert used_e == [[("e", 0), ("e", 1)], [("e", 4), ("e", 5), ("e", 6), ("e", 7)]]
    f = B.plss_blocks(D, b, block=4, residual=False, perm=perm, tol=1e-300, maxit=10, max_steps=3,
                      record=True)
    assert f.iters == 2
    assert [[tuple(c) for c in u] for u in f.columns] == used_e
    assert rel(f.x, [float(v) for v in x]) <= 1e-12
    assert rel(f.x, pins.min_norm(D, b)) <= 1e-12


def test_block_limits_reach_min_norm():
    """The underdetermined recipe at 64 x 256: identity blocks of 8 reach
    A†b after one pass; mixed blocks reach it at the tolerance."""
    sysm = gen.tiny(77, 64, 256, 30, "uniform")
    xm = pins.min_norm(sysm.A.dense(), sysm.b)
    r1 = B.plss_blocks(sysm.A, sysm.b, block=8, residual=False, perm=sysm.perm, tol=1e-300, maxit=8)
    assert r1.iters == 8 and rel(r1.x, xm) <= 1e-10
    r2 = B.plss_blocks(sysm.A, sysm.b, block=8, residual=True, perm=sysm.perm, tol=1e-13, maxit=100)
    assert r2.status == O.OK and rel(r2.x, xm) <= 1e-10


def test_block_edge_cases():
    sysm = gen.tiny(381, 20, 30, 5)
    z = B.plss_blocks(sysm.A, np.zeros(20), block=4)
    assert z.status == O.OK and z.iters == 0 and not np.any(z.x)
    one = B.plss_blocks(sysm.A, sysm.b, block=4, residual=True, perm=sysm.perm, tol=1e-300, maxit=1)
    assert one.iters == 1 and one.status == O.NOT_CONVERGED
    # a block larger than m: one block of all rows (plus r) is the whole pass
    big = B.plss_blocks(sysm.A, sysm.b, block=50, residual=False, perm=sysm.perm, tol=1e-300, maxit=1)
    assert rel(big.x, pins.min_norm(sysm.A.dense(), sysm.b)) <= 1e-10
    with pytest.raises(ValueError):
        B.plss_blocks(sysm.A, sysm.b, block=0, residual=False)
