"""The benchmark's other workloads at their full sizes, in the configuration
bench.py times them: sampled outputs against the oracle (first iterates), and
properties that hold at any size, checked on the host in float64 (the true
relative residual of every converged system, results in a batch equal to
results alone).  The large and small workloads have their own full-size tests
(test_gpu_stripes.py, test_gpu_core.py)."""
import sys

import numpy as np
import pytest

import plss_inputs as gen
from oracle import plss as O

from gpu_common import matrix, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2207_07615_amd as plss
    return plss.Handle(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host_relres(A, x, b):
    """||b - A x|| / ||b|| with the stored values (float32 storage: Â) in
    float64 arithmetic."""
    S = A.scipy().astype(np.float64)
    return float(np.linalg.norm(b - S @ x) / np.linalg.norm(b))


def test_underdet_workload(h):
    """200,000 x 1,000,000, 30 nnz per row, mixed sketch with a history of
    128 columns (Section 7 columns alternating with residual columns): the
    first 8 updates match the oracle's, and the solve to 1e-8 converges with
    its true residual below the tolerance."""
    import paper_2207_07615_amd as plss
    say("underdet workload: generating")
    sysm = gen.underdet()
    M = matrix(h, sysm.A)
    kw = dict(sketch="mixed", row_perm=sysm.perm, hist_cap=128)
    say("underdet workload: 8 updates")
    x, info, _ = plss.solve(h, M, sysm.b, tol=1e-300, maxit=8, **kw)
    ref = O.plss_columns(sysm.A, sysm.b, "mixed", perm=sysm.perm, tol=1e-300, maxit=8, hist_cap=128)
    assert info["iters"] == ref.iters
    assert rel(x, ref.x) <= 1e-12
    say("underdet workload: full solve")
    x, info, _ = plss.solve(h, M, sysm.b, tol=1e-8, maxit=2000, **kw)
    assert info["status"] == 0, info
    assert host_relres(sysm.A, x, sysm.b) <= 1.5e-8


def test_multi_workload(h):
    """Shared 500,000 x 250,000 (20 nnz per row), 32 right-hand sides, float32
    storage: before refinement the first 8 block iterates of sampled columns
    follow Algorithm 1 on Â within 1e-5 (float32 vectors against the float64
    oracle); with float64 refinement every column converges with its true
    residual below 1e-8."""
    import paper_2207_07615_amd as plss
    say("multi workload: generating")
    A, B, X = gen.shared_multi_rhs(storage=np.float32)
    M = matrix(h, A, "f32")
    say("multi workload: 8 iterations, no refinement")
    X8, infos = plss.solve_multi(h, M, B.T, tol=1e-300, maxit=8, refine=False)
    for c in (0, 13, 31):
        assert infos[c]["iters"] == 8
        ref = O.plss_residual(A, B[c], tol=1e-300, maxit=8)
        assert rel(X8[:, c], ref.x) <= 1e-5
    say("multi workload: refined solve")
    Xg, infos = plss.solve_multi(h, M, B.T, tol=1e-8, maxit=5000, refine=True, inner_tol=1e-4)
    for c in range(B.shape[0]):
        assert infos[c]["status"] == 0, (c, infos[c])
        assert host_relres(A, Xg[:, c], B[c]) <= 1.5e-8


def test_batch_workload(h):
    """256 uneven systems (m log-uniform in [1e3, 2e5], 5-50 nnz per row),
    float32 storage + float64 refinement, iteration cap 4000, all in one
    batch: every converged system's true residual is below 1e-8 and the
    others return a finite iterate with a warning status; two sampled systems
    give bit-identical results solved alone."""
    import paper_2207_07615_amd as plss
    say("batch workload: generating")
    data = []
    for s in gen.batch_systems(256):
        A32 = s.A.astype(np.float32)
        data.append((A32, gen.rhs(A32, s.xstar)))
    mats = [matrix(h, A, "f32") for A, _ in data]
    kw = dict(tol=1e-8, maxit=4000, refine=True, inner_tol=1e-4)
    say("batch workload: solve")
    xs, infos = plss.solve_batch(h, mats, [b for _, b in data], **kw)
    ok = 0
    for (A, b), x, inf in zip(data, xs, infos):
        assert np.all(np.isfinite(x))
        if inf["status"] == 0:
            ok += 1
            assert host_relres(A, x, b) <= 1.5e-8
        else:
            # stopped by the cap, by the bound on outer steps, or by an
            # outer step that no longer reduced the residual
            assert inf["status"] in (1, 2), inf
    say("batch workload: converged", ok)
    assert ok >= 240
    sizes = np.argsort([A.m for A, _ in data])
    for i in (int(sizes[0]), int(sizes[len(sizes) // 2])):
        xa, ia, _ = plss.solve(h, mats[i], data[i][1], **kw)
        assert ia["iters"] == infos[i]["iters"]
        np.testing.assert_array_equal(xa, xs[i])


def test_serve_workload(h):
    """100 systems of the served stream (m log-uniform in [1e3, 1e6], n/m in
    U(0.3, 1), Zipf rows, tolerance 1e-6 or 1e-10 each), float32 storage +
    float64 refinement, all submitted at once as in the saturated run: every
    request finishes; each converged one meets its own tolerance on the host;
    two sampled results are bit-identical to the same system solved alone on
    the per-phase engine the server runs."""
    import time
    import paper_2207_07615_amd as plss
    say("serve workload: generating")
    data = []
    for s in gen.stream_systems(100):
        A32 = s.A.astype(np.float32)
        data.append((s, A32, gen.rhs(A32, s.xstar)))
    srv = plss.Server(h, hbm_budget_bytes=200 << 30, max_slots=256)
    kws = [dict(tol=s.tol, maxit=min(s.A.n + 1000, 4000), refine=True, inner_tol=1e-4) for s, _, _ in data]
    say("serve workload: submitting")
    reqs = [srv.submit(A32, b, storage="f32", **kw) for (_, A32, b), kw in zip(data, kws)]
    out = {}
    t0 = time.time()
    while len(out) < len(reqs):
        for i, r in enumerate(reqs):
            if i not in out:
                got = srv.poll(r)
                if got is not None:
                    out[i] = got
        assert time.time() - t0 < 200, f"{len(out)} of {len(reqs)} finished"
        time.sleep(0.002)
    st = srv.stats()
    srv.close()
    assert st["submitted"] == st["finished"] == len(reqs)
    ok = 0
    for i, ((s, A32, b), kw) in enumerate(zip(data, kws)):
        x, info = out[i]
        assert np.all(np.isfinite(x))
        if info["status"] == 0:
            ok += 1
            assert host_relres(A32, x, b) <= 1.5 * kw["tol"], (i, info)
        else:
            assert info["status"] in (1, 2), (i, info)
    say("serve workload: converged", ok)
    assert ok >= 60
    sizes = np.argsort([s.A.m for s, _, _ in data])
    for i in (int(sizes[0]), int(sizes[len(sizes) // 2])):
        s, A32, b = data[i]
        M = matrix(h, A32, "f32")
        xa, ia, _ = plss.solve(h, M, b, engine="multi", **kws[i])
        x, info = out[i]
        assert ia["iters"] == info["iters"]
        np.testing.assert_array_equal(xa, x)
