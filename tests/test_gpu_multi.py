"""GPU parity of the many-right-hand-side path (block products over A and
Aᵀ, one Algorithm-1 recurrence per column) against the oracle per column."""
import sys

import numpy as np
import pytest

import plss_inputs as gen
from oracle import plss as O

from gpu_common import CONVERGED_TOL, converged_check, matrix, order_bound, order_spread, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2207_07615_amd as plss
    return plss.Handle(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("nrhs", [1, 5, 32, 70])
def test_multi_fp64_matches_oracle_per_column(h, nrhs):
    import paper_2207_07615_amd as plss
    say("multi fp64", nrhs)
    A, B, X = gen.shared_multi_rhs(m=3000, n=1500, L=8, nrhs=nrhs)
    M = matrix(h, A)
    Xg, infos = plss.solve_multi(h, M, B.T, tol=1e-8, maxit=2000)
    assert Xg.shape == (1500, nrhs)
    for c in range(0, nrhs, max(1, nrhs // 6)):
        inf = infos[c]
        assert inf["status"] == 0, (c, inf)
        assert inf["relres_true"] <= 1.5e-8
        ref, spread = order_spread(A, B[c], inf["iters"])
        err = rel(Xg[:, c], ref.x)
        say(f"  col {c}: iters={inf['iters']} err={err:.3e} spread={spread:.3e}")
        order_bound(err, spread, f"multi{nrhs}_col{c}")
    # converged (relres 1e-13) against the oracle per column at the flat 1e-10
    Xc, infc = plss.solve_multi(h, M, B.T, tol=CONVERGED_TOL, maxit=20000)
    for c in range(0, nrhs, max(1, nrhs // 6)):
        assert infc[c]["status"] == 0, (c, infc[c])
        ref = O.plss_residual(A, B[c], tol=CONVERGED_TOL, maxit=20000)
        converged_check(Xc[:, c], ref.x, f"multi{nrhs}_col{c}")


def test_multi_column_equals_single_solve(h):
    """A column of the block solve and the same right-hand side solved alone
    reach the same iterate (different summation orders: within the order
    spread)."""
    import paper_2207_07615_amd as plss
    say("multi vs single")
    A, B, X = gen.shared_multi_rhs(m=4000, n=2000, L=10, nrhs=8)
    M = matrix(h, A)
    Xg, infos = plss.solve_multi(h, M, B.T, tol=1e-9, maxit=2000)
    for c in (0, 7):
        x1, i1, _ = plss.solve(h, M, B[c], tol=1e-9, maxit=2000)
        assert abs(i1["iters"] - infos[c]["iters"]) <= 1
        assert rel(Xg[:, c], X[c]) <= 1e-7 and rel(x1, X[c]) <= 1e-7


def test_multi_fp32_refinement(h):
    import paper_2207_07615_amd as plss
    say("multi fp32")
    A, B, X = gen.shared_multi_rhs(m=3000, n=1500, L=8, nrhs=8, storage=np.float32)
    M = matrix(h, A, "f32")
    Xg, infos = plss.solve_multi(h, M, B.T, tol=1e-11, maxit=5000, refine=True, inner_tol=1e-4)
    for c in range(8):
        assert infos[c]["status"] == 0, infos[c]
        assert infos[c]["relres_true"] <= 1e-11
        assert infos[c]["outer_iters"] >= 2
        assert rel(Xg[:, c], X[c]) <= 1e-9


def test_multi_edge_cases(h):
    import paper_2207_07615_amd as plss
    say("multi edges")
    A, B, X = gen.shared_multi_rhs(m=500, n=300, L=6, nrhs=3)
    B[1] = 0.0
    M = matrix(h, A)
    Xg, infos = plss.solve_multi(h, M, B.T, tol=1e-8, maxit=500)
    assert infos[1]["iters"] == 0 and not np.any(Xg[:, 1])
    assert infos[0]["status"] == 0 and infos[2]["status"] == 0
    Xg, infos = plss.solve_multi(h, M, B.T, tol=1e-14, maxit=1)
    ref = O.plss_residual(A, B[0], tol=1e-14, maxit=1)
    assert infos[0]["iters"] == 1 and infos[0]["status"] == 1
    assert rel(Xg[:, 0], ref.x) <= 1e-13
