"""The fused residual pair (plss_residual_pair: r <- r - A p, then y = Aᵀ r
with the updated r, in one pass over the CSR) against the oracle's
residual_pair, entry by entry.

Tolerances: float64 accumulation in a different order than the oracle's, so
each entry of r is within 1e-14 (|r| + |A| |p|) of the oracle's, and each
entry of y within 1e-14 |A|ᵀ (|r| + |A| |p| + |r_new|) (the first term
carries the difference in r, the second the rounding of y's own sum); the
squared norms within the bound these entry-wise bounds imply.  Results are
bit-reproducible (fixed summation order), and the host-array and device-
tensor paths run the same kernels, so they agree bit for bit."""
import sys
import time

import numpy as np
import pytest

import plss_inputs as gen
from oracle import sparse as osp

from gpu_common import matrix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2207_07615_amd as plss
    return plss.Handle(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ragged(seed, m, n):
    """Empty rows, short rows, and rows of 4500 and 2048 entries."""
    rng = gen.rng_for(seed)
    L = rng.integers(0, 12, size=m)
    L[rng.random(m) < 0.1] = 0
    L[:: max(1, m // 3)] = min(n, 4500)
    L[5] = min(n, 2048)
    return gen.make_csr(rng, m, n, np.minimum(L, n), "normal")


CASES = {
    "small": lambda: gen.small(m=3000, n=1500).A,
    "ragged": lambda: ragged(11, 9000, 13000),
    # most columns empty (y_j = 0 exactly)
    "wide": lambda: gen.tiny(4, 300, 20000, 30).A,
    # one row of 8000 entries
    "dense_row": lambda: gen.make_csr(gen.rng_for(9), 1, 9000, np.array([8000]), "normal"),
    # one column of 5000 entries
    "one_col": lambda: gen.make_csr(gen.rng_for(12), 5000, 1, np.ones(5000, dtype=np.int64), "normal"),
    # the large workload's Zipf row lengths, at a size the oracle runs in seconds
    "zipf": lambda: gen.large(m=60000, n=15000).A,
    # 8000 rows of 1200 entries: every row is summed by a whole workgroup
    # (four waves), and each row's contributions need the residual entry as
    # it was before the row's update, in every wave
    "long_rows": lambda: gen.make_csr(gen.rng_for(14), 8000, 20000, np.full(8000, 1200, dtype=np.int64), "normal"),
}


def bounds(S, p, r, r_o):
    absS = abs(S)
    tol_r = 1e-14 * (np.abs(r) + absS @ np.abs(p)) + 1e-300
    tol_y = 1e-14 * (absS.T @ (np.abs(r) + absS @ np.abs(p) + np.abs(r_o))) + 1e-300
    return tol_r, tol_y


def check_against_oracle(S, p, r, got, case):
    r1, y1, rho, phi = got
    r_o, y_o, rho_o, phi_o = osp.residual_pair(S, p, r)
    tol_r, tol_y = bounds(S, p, r, r_o)
    err_r = np.abs(r1 - r_o)
    err_y = np.abs(y1 - y_o)
    say(case, "max err/bound r", float(np.max(err_r / tol_r)), "y", float(np.max(err_y / tol_y)))
    assert np.all(err_r <= tol_r)
    assert np.all(err_y <= tol_y)
    # ||r||² and ||y||²: |a² - b²| <= (2|b| + |a - b|) |a - b| per entry
    assert abs(rho - rho_o) <= float(np.sum((2 * np.abs(r_o) + tol_r) * tol_r)) + 1e-13 * rho_o
    assert abs(phi - phi_o) <= float(np.sum((2 * np.abs(y_o) + tol_y) * tol_y)) + 1e-13 * phi_o


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_residual_pair_matches_oracle(h, case, storage):
    import paper_2207_07615_amd as plss
    say("residual pair", case, storage)
    A = CASES[case]()
    M = matrix(h, A, storage)
    S = A.astype(np.float32).scipy() if storage == "f32" else A.scipy()
    rng = np.random.default_rng(3)
    p = rng.standard_normal(A.n)
    r = rng.standard_normal(A.m)
    r_keep = r.copy()
    got = plss.residual_pair(h, M, p, r)
    np.testing.assert_array_equal(r, r_keep)  # the caller's r is left alone
    check_against_oracle(S, p, r, got, case)
    # empty columns sum to exactly zero
    empty = np.diff(S.tocsc().indptr) == 0
    assert np.all(got[1][empty] == 0.0)
    # a second call: the same bits
    again = plss.residual_pair(h, M, p, r)
    np.testing.assert_array_equal(again[0], got[0])
    np.testing.assert_array_equal(again[1], got[1])
    assert again[2] == got[2] and again[3] == got[3]


def test_residual_pair_device_tensors(h):
    """Device tensors are used in place; the results equal the host path's."""
    import torch
    import paper_2207_07615_amd as plss
    say("residual pair: device tensors")
    A = CASES["zipf"]()
    M = matrix(h, A)
    rng = np.random.default_rng(8)
    p = rng.standard_normal(A.n)
    r = rng.standard_normal(A.m)
    host = plss.residual_pair(h, M, p, r)
    dev = torch.device("cuda:0")
    pd, rd = torch.from_numpy(p).to(dev), torch.from_numpy(r).to(dev)
    r1, y1, rho, phi = plss.residual_pair(h, M, pd, rd)
    assert r1.is_cuda and y1.is_cuda
    np.testing.assert_array_equal(rd.cpu().numpy(), r)  # input tensor unchanged
    np.testing.assert_array_equal(r1.cpu().numpy(), host[0])
    np.testing.assert_array_equal(y1.cpu().numpy(), host[1])
    assert rho == host[2] and phi == host[3]


def test_residual_pair_errors(h):
    """Null arguments return EINVAL through the C ABI; wrong lengths are
    refused by the binding before any call."""
    import paper_2207_07615_amd as plss
    from paper_2207_07615_amd import _lib
    say("residual pair: errors")
    A = CASES["small"]()
    M = matrix(h, A)
    r = np.zeros(A.m)
    y = np.zeros(A.n)
    lib = _lib.load()
    PLSS_EINVAL = -1
    assert lib.plss_residual_pair(h.h, M.A, None, r.ctypes.data, y.ctypes.data, None) == PLSS_EINVAL
    assert lib.plss_residual_pair(None, M.A, y.ctypes.data, r.ctypes.data, y.ctypes.data, None) == PLSS_EINVAL
    assert lib.plss_residual_pair(h.h, None, y.ctypes.data, r.ctypes.data, y.ctypes.data, None) == PLSS_EINVAL
    with pytest.raises(ValueError):
        plss.residual_pair(h, M, np.zeros(A.n + 1), np.zeros(A.m))
    with pytest.raises(ValueError):
        plss.residual_pair(h, M, np.zeros(A.n), np.zeros(A.m - 1))


def test_residual_pair_no_entries(h):
    """A matrix without stored entries: r is unchanged, y and ||y||² are zero."""
    import paper_2207_07615_amd as plss
    say("residual pair: no entries")
    A = gen.make_csr(gen.rng_for(15), 6, 4, np.zeros(6, dtype=np.int64), "normal")
    M = matrix(h, A)
    r = np.arange(6.0) - 2.5
    r1, y1, rho, phi = plss.residual_pair(h, M, np.ones(4), r)
    np.testing.assert_array_equal(r1, r)
    np.testing.assert_array_equal(y1, np.zeros(4))
    assert rho == float(np.dot(r, r)) and phi == 0.0


def test_residual_pair_chained_iterations(h):
    """Three pairs in a row, each from the last one's r, against the oracle
    chained the same way (the position map and the contribution buffer are
    reused across calls)."""
    import paper_2207_07615_amd as plss
    say("residual pair: chained")
    A = CASES["ragged"]()
    M = matrix(h, A)
    S = A.scipy()
    rng = np.random.default_rng(21)
    r = rng.standard_normal(A.m)
    for k in range(3):
        p = rng.standard_normal(A.n)
        got = plss.residual_pair(h, M, p, r)
        check_against_oracle(S, p, r, got, f"chained {k}")
        r = got[0]


@pytest.mark.slow
def test_residual_pair_large_workload(h):
    """The 2,000,000 x 500,000 Zipf workload at full size, in the layout the
    benchmark runs: sampled rows of r match the row products computed one by
    one, and y equals the oracle's Aᵀ applied to the returned r, entry by
    entry (a property that holds at any size)."""
    import torch
    import paper_2207_07615_amd as plss
    say("residual pair, large workload: generating")
    A = gen.large().A
    M = matrix(h, A)
    rng = np.random.default_rng(6)
    p = rng.standard_normal(A.n)
    r = rng.standard_normal(A.m)
    dev = torch.device("cuda:0")
    pd, rd = torch.from_numpy(p).to(dev), torch.from_numpy(r).to(dev)
    plss.residual_pair(h, M, pd, rd)  # builds the position map
    t0 = time.perf_counter()
    r1, y1, rho, phi = plss.residual_pair(h, M, pd, rd)
    say("residual pair, large workload: %.3f ms per call" % (1e3 * (time.perf_counter() - t0)))
    r1, y1 = r1.cpu().numpy(), y1.cpu().numpy()
    for i in np.random.default_rng(5).choice(A.m, 200, replace=False):
        lo, hi = A.row_ptr[i], A.row_ptr[i + 1]
        want = r[i] - float(np.dot(A.vals[lo:hi], p[A.col_idx[lo:hi]]))
        bound = 1e-14 * (abs(r[i]) + float(np.abs(A.vals[lo:hi]) @ np.abs(p[A.col_idx[lo:hi]]))) + 1e-300
        assert abs(r1[i] - want) <= bound
    S = A.scipy()
    y_o = osp.rmatvec(S, r1)
    tol_y = 1e-14 * (abs(S).T @ np.abs(r1)) + 1e-300
    assert np.all(np.abs(y1 - y_o) <= tol_y)
    rr = float(np.dot(r1, r1))
    yy = float(np.dot(y1, y1))
    assert abs(rho - rr) <= 1e-12 * rr
    assert abs(phi - yy) <= 1e-12 * yy
