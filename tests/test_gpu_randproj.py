"""GPU parity of the randomized projection (Section 8's comparison method:
eq. pkLong with a fresh standard normal sketch each iteration, drawn by
Philox4x32-10 and Box-Muller on both sides) against its oracle."""
import sys

import numpy as np
import pytest

import plss_inputs as gen
from oracle import pins
from oracle import randproj as RP

from gpu_common import CONVERGED_TOL, chunk_dot, converged_check, fsum_dot, matrix, order_bound, rel, rev_dot

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2207_07615_amd as plss
    return plss.Handle(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("r", [1, 5, 10, 16])
def test_first_iterates_match_oracle(h, r):
    """The device draws the oracle's sketches (same counters, same key), so
    the first iterates agree to rounding."""
    import paper_2207_07615_amd as plss
    say("randproj first iterates", r)
    sysm = gen.small(m=3000, n=1500)
    M = matrix(h, sysm.A)
    for k in (1, 3, 10):
        x, info, hist = plss.solve(h, M, sysm.b, sketch="randproj", block=r, seed=761508, tol=1e-300, maxit=k)
        ref = RP.randproj(sysm.A, sysm.b, r=r, seed=761508, tol=1e-300, maxit=k)
        assert info["iters"] == k
        assert rel(x, ref.x) <= 1e-12
        np.testing.assert_allclose(hist[:k + 1], ref.hist[:k + 1], rtol=1e-11)


def test_randproj_solve_matches_oracle(h):
    """A full solve (tol 1e-8): equal update counts (trajectory bound), and
    both sides solved to 1e-13 at the flat 1e-10 (an overdetermined system
    with full column rank: both reach x*)."""
    import paper_2207_07615_amd as plss
    say("randproj solve")
    sysm = gen.small(m=1200, n=200)
    M = matrix(h, sysm.A)
    kw = dict(sketch="randproj", block=10, seed=5)
    x, info, _ = plss.solve(h, M, sysm.b, tol=1e-8, maxit=20000, **kw)
    assert info["status"] == 0 and info["relres_true"] <= 1.5e-8
    k = info["iters"]
    ref = RP.randproj(sysm.A, sysm.b, r=10, seed=5, tol=1e-300, maxit=k)
    spread = 0.0
    for dot in (fsum_dot, rev_dot, chunk_dot):
        alt = RP.randproj(sysm.A, sysm.b, r=10, seed=5, tol=1e-300, maxit=k, dot=dot)
        spread = max(spread, rel(alt.x, ref.x))
    say(f"  iters={k} err={rel(x, ref.x):.3e} spread={spread:.3e}")
    order_bound(rel(x, ref.x), spread, "randproj10_1200x200")
    full = RP.randproj(sysm.A, sysm.b, r=10, seed=5, tol=1e-8, maxit=20000)
    assert abs(full.iters - k) <= 1
    xc, ic, _ = plss.solve(h, M, sysm.b, tol=CONVERGED_TOL, maxit=100000, **kw)
    refc = RP.randproj(sysm.A, sysm.b, r=10, seed=5, tol=CONVERGED_TOL, maxit=100000)
    assert ic["status"] == 0 and refc.status == 0
    converged_check(xc, refc.x, "randproj10_1200x200")
    assert rel(xc, sysm.xstar) <= 1e-10


def test_randproj_underdetermined_square_sketch(h):
    """r = m on a full-row-rank 12 x 30 system: one step gives A†b."""
    import paper_2207_07615_amd as plss
    say("randproj square sketch")
    sysm = gen.tiny(403, 12, 30, 6)
    M = matrix(h, sysm.A)
    x, info, _ = plss.solve(h, M, sysm.b, sketch="randproj", block=12, seed=5, tol=1e-300, maxit=1)
    assert rel(x, pins.min_norm(sysm.A.dense(), sysm.b)) <= 1e-10


def test_randproj_edge_cases(h):
    import paper_2207_07615_amd as plss
    say("randproj edges")
    sysm = gen.small(m=400, n=200)
    M = matrix(h, sysm.A)
    x, info, _ = plss.solve(h, M, np.zeros(400), sketch="randproj", block=5, tol=1e-8, maxit=10)
    assert info["iters"] == 0 and info["status"] == 0 and not np.any(x)
    x, info, _ = plss.solve(h, M, sysm.b, sketch="randproj", block=5, tol=1e-300, maxit=7)
    assert info["status"] == 1 and info["iters"] == 7
    for bad in (0, 17):
        with pytest.raises(plss.PlssError):
            plss.solve(h, M, sysm.b, sketch="randproj", block=bad, tol=1e-8, maxit=10)
    with pytest.raises(plss.PlssError):
        plss.solve(h, matrix(h, sysm.A, "f32"), sysm.b, sketch="randproj", block=5, tol=1e-8, maxit=10)


def test_randproj_on_striped_products(h):
    """With a striped store of A (the layout of the large workload) the
    product r -= A p and the initial and final residuals run on the stripes;
    the iterates are the oracle's."""
    import paper_2207_07615_amd as plss
    say("randproj striped")
    sysm = gen.large(m=60000, n=15000)
    M = matrix(h, sysm.A)
    lay = M.layout(a_stripes=True, t_stripes=True, unit_rows=512)
    assert lay["a_stripes"]
    for k in (1, 4):
        x, info, hist = plss.solve(h, M, sysm.b, sketch="randproj", block=5, seed=9, tol=1e-300, maxit=k)
        ref = RP.randproj(sysm.A, sysm.b, r=5, seed=9, tol=1e-300, maxit=k)
        assert info["iters"] == k
        assert rel(x, ref.x) <= 1e-12
        assert abs(info["relres_true"] - ref.relres_true) <= 1e-12 * max(1.0, ref.relres_true)
