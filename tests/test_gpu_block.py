"""GPU parity of the block sketches (a block of identity rows, or the
residual and identity rows, appended per step; the block form of the
triangular update of Section 2.4) against the block oracle."""
import sys

import numpy as np
import pytest

import plss_inputs as gen
from oracle import blocks as OB
from oracle import pins

from gpu_common import (CONVERGED_TOL, chunk_dot, converged_check, fsum_dot, matrix, order_bound, rel,
                        rev_dot)

pytestmark = pytest.mark.gpu

SKETCH = {False: "block_identity", True: "block_mixed"}


@pytest.fixture(scope="module")
def h():
    import paper_2207_07615_amd as plss
    return plss.Handle(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def block_parity(h, sysm, block, residual, tol, maxit, cap, converged=True):
    """Equal update counts against the oracle (trajectory bound of
    order_bound), and converged solutions at the flat 1e-10."""
    import paper_2207_07615_amd as plss
    M = matrix(h, sysm.A)
    kw = dict(sketch=SKETCH[residual], block=block, row_perm=sysm.perm, hist_cap=cap)
    x, info, hist = plss.solve(h, M, sysm.b, tol=tol, maxit=maxit, **kw)
    k = info["iters"]
    okw = dict(block=block, residual=residual, perm=sysm.perm, hist_cap=cap)
    ref = OB.plss_blocks(sysm.A, sysm.b, tol=1e-300, maxit=k, **okw)
    spread = 0.0
    for dot in (fsum_dot, rev_dot, chunk_dot):
        alt = OB.plss_blocks(sysm.A, sysm.b, tol=1e-300, maxit=k, dot=dot, **okw)
        spread = max(spread, rel(alt.x, ref.x))
    err = rel(x, ref.x)
    case = f"{SKETCH[residual]}{block}_{sysm.A.m}x{sysm.A.n}_cap{cap}"
    say(f"  {case}: updates={k} blocks={info['outer_iters']} err={err:.3e} spread={spread:.3e}")
    assert ref.iters == k
    order_bound(err, spread, case)
    full = OB.plss_blocks(sysm.A, sysm.b, tol=tol, maxit=maxit, **okw)
    assert abs(full.iters - k) <= 1
    if converged:
        xc, ic, _ = plss.solve(h, M, sysm.b, tol=CONVERGED_TOL, maxit=20 * maxit, **kw)
        assert ic["status"] == 0, ic
        refc = OB.plss_blocks(sysm.A, sysm.b, tol=CONVERGED_TOL, maxit=20 * maxit, **okw)
        assert refc.status == 0
        converged_check(xc, refc.x, case)
    return x, info, hist, ref


@pytest.mark.parametrize("block,residual", [(1, False), (4, False), (16, False), (1, True), (3, True), (15, True)])
def test_tiny_block_matches_oracle(h, block, residual):
    say("tiny block", block, residual)
    sysm = gen.tiny(31, 60, 150, 8, "uniform")
    x, info, hist, ref = block_parity(h, sysm, block, residual, 1e-10, 4000, 60)
    assert info["status"] == 0
    np.testing.assert_allclose(hist[:4], ref.hist[:4], rtol=1e-9)


def test_first_block_steps_match_oracle_closely(h):
    """Before rounding differences are amplified, the first updates agree to
    1e-12 (overdetermined Zipf rows, mixed blocks of 7)."""
    import paper_2207_07615_amd as plss
    say("first block steps")
    sysm = gen.large(m=6000, n=1500)
    sysm.perm = np.random.default_rng(3).permutation(6000).astype(np.int32)
    M = matrix(h, sysm.A)
    for k in (1, 2, 5):
        x, info, _ = plss.solve(h, M, sysm.b, sketch="block_mixed", block=7, row_perm=sysm.perm,
                                hist_cap=128, tol=1e-300, maxit=k)
        ref = OB.plss_blocks(sysm.A, sysm.b, block=7, residual=True, perm=sysm.perm, hist_cap=128,
                             tol=1e-300, maxit=k)
        assert info["iters"] == k
        assert rel(x, ref.x) <= 1e-12


@pytest.mark.parametrize("block", [1, 8, 16])
def test_identity_blocks_reach_min_norm_in_one_pass(h, block):
    """Corollary 2 with block identity sketches: one pass of blocks over a
    full-row-rank 64 x 256 system gives A†b."""
    import paper_2207_07615_amd as plss
    say("block cor2", block)
    sysm = gen.tiny(77, 64, 256, 30, "uniform")
    M = matrix(h, sysm.A)
    steps = -(-64 // block)
    x, info, _ = plss.solve(h, M, sysm.b, sketch="block_identity", block=block, tol=1e-300, maxit=steps,
                            row_perm=sysm.perm, hist_cap=64)
    assert info["iters"] == steps
    assert rel(x, pins.min_norm(sysm.A.dense(), sysm.b)) <= 1e-10


def test_block_drop_rule_matches_oracle(h):
    """Repeated and dependent rows in a block and across blocks are left out
    of the sketch as by the oracle (whose rule is pinned against the
    rational twin): same update count, same iterate, A†b after the pass."""
    import paper_2207_07615_amd as plss
    from gpu_common import csr_from_dense
    say("block drop rule")
    rng = np.random.default_rng(371)
    D = np.zeros((9, 12))
    for i in (0, 1, 4, 5, 6, 7):
        D[i, rng.choice(12, 4, replace=False)] = rng.integers(1, 4, 4) * rng.choice([-1, 1], 4)
    D[2] = D[0]
    D[3] = D[0] + D[1]
    D[8] = D[4] - D[5]
    b = D @ rng.integers(-2, 3, 12).astype(np.float64)
    rp, ci, va = csr_from_dense(D)
    M = plss.Matrix(h, rp, ci, va, shape=(9, 12))
    perm = np.arange(9, dtype=np.int32)
    x, info, _ = plss.solve(h, M, b, sketch="block_identity", block=4, tol=1e-300, maxit=10, row_perm=perm,
                            hist_cap=12)
    ref = OB.plss_blocks(D, b, block=4, residual=False, perm=perm, tol=1e-300, maxit=10, hist_cap=12)
    assert info["iters"] == ref.iters
    assert rel(x, ref.x) <= 1e-12
    assert rel(x, pins.min_norm(D, b)) <= 1e-12


@pytest.mark.parametrize("cap", [8, 20])
def test_block_history_cap_matches_oracle(h, cap):
    """Small history capacities clear the stored blocks often, and the pass
    end clears them too, on both sides."""
    say("block cap", cap)
    sysm = gen.tiny(41, 80, 200, 10, "uniform")
    block_parity(h, sysm, 3, True, 1e-9, 3000, cap)


def test_mixed_blocks_underdetermined_medium(h):
    """The underdetermined recipe (30 entries per row, U(-1,1)) at 20,000 x
    100,000 with mixed blocks of 15 rows (16 columns, one MFMA tile)."""
    say("mixed blocks medium")
    sysm = gen.underdet(m=20000, n=100000)
    x, info, hist, ref = block_parity(h, sysm, 15, True, 1e-8, 2000, 256)
    assert info["status"] == 0 and info["relres_true"] <= 1.5e-8


def test_block_edge_cases(h):
    import paper_2207_07615_amd as plss
    say("block edges")
    sysm = gen.tiny(55, 40, 90, 6)
    M = matrix(h, sysm.A)
    x, info, _ = plss.solve(h, M, np.zeros(40), sketch="block_mixed", block=3, tol=1e-8, maxit=10)
    assert info["iters"] == 0 and info["status"] == 0 and not np.any(x)
    x, info, _ = plss.solve(h, M, sysm.b, sketch="block_identity", block=5, tol=1e-300, maxit=1,
                            row_perm=sysm.perm)
    ref = OB.plss_blocks(sysm.A, sysm.b, block=5, residual=False, perm=sysm.perm, tol=1e-300, maxit=1,
                         hist_cap=40)
    assert info["iters"] == 1 and info["status"] == 1
    assert rel(x, ref.x) <= 1e-13
    # a block wider than the rows left in the pass, m not a multiple of the block
    x, info, _ = plss.solve(h, M, sysm.b, sketch="block_identity", block=16, tol=1e-300, maxit=3,
                            row_perm=sysm.perm, hist_cap=40)
    ref = OB.plss_blocks(sysm.A, sysm.b, block=16, residual=False, perm=sysm.perm, tol=1e-300, maxit=3,
                         hist_cap=40)
    assert rel(x, ref.x) <= 1e-12
    for bad in (dict(sketch="block_identity", block=0), dict(sketch="block_identity", block=17),
                dict(sketch="block_mixed", block=16), dict(sketch="block_mixed", block=3, hist_cap=1025)):
        with pytest.raises(plss.PlssError):
            plss.solve(h, M, sysm.b, tol=1e-8, maxit=10, **bad)
    M32 = matrix(h, sysm.A, "f32")
    with pytest.raises(plss.PlssError):
        plss.solve(h, M32, sysm.b, sketch="block_mixed", block=3, tol=1e-8, maxit=10)
