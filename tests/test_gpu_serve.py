"""Request loop (continuous batching): results identical alone and in the
mix, admission by memory budget, cancellation, input errors."""
import sys
import time

import numpy as np
import pytest

import plss_inputs as gen

from gpu_common import matrix, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2207_07615_amd as plss
    return plss.Handle(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def wait(srv, req, timeout=120.0):
    t0 = time.time()
    while True:
        r = srv.poll(req)
        if r is not None:
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError(req)
        time.sleep(0.002)


def single_fits(A, kind):
    """The single-workgroup engine holds x, r, p, y and the row pointers in LDS."""
    vb = 4 if kind == "f32" else 8
    return 8 * A.n + vb * (A.m + 2 * A.n) + 4 * (A.m + A.n + 40) <= 156 * 1024 - 1024


def test_served_results_equal_alone(h):
    """Requests arriving while others run join the running batch; each
    result is bit-identical to the same system solved alone on the same
    engine (the per-phase engine, or the single-workgroup engine for the
    requests that ask for it)."""
    import paper_2207_07615_amd as plss
    say("serve mix")
    systems = gen.stream_systems(10, m_lo=1e3, m_hi=3e4)
    kinds = ["f64" if i % 2 == 0 else "f32" for i in range(len(systems))]
    srv = plss.Server(h, hbm_budget_bytes=8 << 30, max_slots=16)
    reqs = []
    n_single = 0
    for i, (s, kind) in enumerate(zip(systems, kinds)):
        engine = "single" if i % 4 != 2 and single_fits(s.A, kind) else "multi"
        n_single += engine == "single"
        kw = dict(tol=s.tol, maxit=s.A.n + 1000, engine=engine)
        if kind == "f32":
            A32 = s.A.astype(np.float32)
            b = gen.rhs(A32, s.xstar)
            reqs.append((srv.submit(A32, b, storage="f32", refine=True, inner_tol=1e-4, **kw), A32, b, kw, kind))
        else:
            reqs.append((srv.submit(s.A, s.b, **kw), s.A, s.b, kw, kind))
        time.sleep(0.003 * (i % 3))
    out = [wait(srv, r[0]) for r in reqs]
    st = srv.stats()
    assert st["submitted"] == st["finished"] == len(systems)
    srv.close()
    for (req, A, b, kw, kind), (x, info) in zip(reqs, out):
        M = matrix(h, A, kind)
        extra = dict(refine=True, inner_tol=1e-4) if kind == "f32" else {}
        xa, ia, _ = plss.solve(h, M, b, **kw, **extra)
        say(f"  {kind} {kw['engine']} m={A.m} iters={info['iters']} status={info['status_name']} "
            f"latency_ms={info['ms']:.1f}")
        assert info["status"] == ia["status"]
        assert info["iters"] == ia["iters"]
        np.testing.assert_array_equal(x, xa)
    assert n_single >= 1


def test_small_budget_queues_requests(h):
    import paper_2207_07615_amd as plss
    say("serve budget")
    systems = gen.stream_systems(4, m_lo=2e4, m_hi=3e4, first=20)
    # room for roughly one system at a time
    nnz = max(s.A.nnz for s in systems)
    m = max(s.A.m for s in systems)
    budget = int(24 * nnz + 80 * m + (8 << 20))
    srv = plss.Server(h, hbm_budget_bytes=budget, max_slots=8)
    reqs = [srv.submit(s.A, s.b, tol=1e-8, maxit=s.A.n + 1000) for s in systems]
    res = [wait(srv, r) for r in reqs]
    st = srv.stats()
    srv.close()
    assert st["peak_bytes"] <= budget
    for s, (x, info) in zip(systems, res):
        assert info["status"] == 0
        assert info["relres_true"] <= 1.5e-8


def test_errors_and_cancel(h):
    import paper_2207_07615_amd as plss
    say("serve errors")
    s = gen.stream_systems(1, m_lo=5e4, m_hi=6e4, first=40)[0]
    srv = plss.Server(h, hbm_budget_bytes=1 << 20, max_slots=4)
    with pytest.raises(plss.PlssError) as e:
        srv.submit(s.A, s.b, tol=1e-8, maxit=100)
    assert e.value.code == -2  # ENOMEM: larger than the budget
    srv.close()
    srv = plss.Server(h, hbm_budget_bytes=8 << 30, max_slots=1)
    bad = s.b.copy()
    bad[0] = np.nan
    with pytest.raises(plss.PlssError) as e:
        srv.submit(s.A, bad, tol=1e-8, maxit=100)
    assert e.value.code == -1
    # a long solve (unreachable tolerance) and one queued behind it (1 slot)
    r1 = srv.submit(s.A, s.b, tol=1e-300, maxit=10**7)
    r2 = srv.submit(s.A, s.b, tol=1e-8, maxit=s.A.n + 1000)
    time.sleep(0.05)
    srv.cancel(r2)
    srv.cancel(r1)
    for r in (r1, r2):
        with pytest.raises(plss.PlssError) as e:
            wait(srv, r)
        assert e.value.code == -4  # ECANCELLED
    r3 = srv.submit(s.A, s.b, tol=1e-8, maxit=s.A.n + 1000)
    x, info = wait(srv, r3)
    assert info["status"] == 0
    srv.close()
