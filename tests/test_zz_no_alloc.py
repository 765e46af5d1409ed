"""plss_spmv_noalloc (the product with every scratch buffer in a fixed
per-device array) against plss_spmv, through the C ABI: bit-identical
products on two calls in a row (the second smaller), the oracle's
entry-wise bound, and the error paths."""
import sys

import numpy as np
import pytest

import plss_inputs as gen

from gpu_common import matrix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2207_07615_amd as plss
    return plss.Handle(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def products(h, M, A, seed):
    """Both directions through plss_spmv_noalloc and plss_spmv; checks the
    two agree bit for bit and meet |y - S x| <= 1e-14 (|S| |x|)."""
    import torch
    import paper_2207_07615_amd as plss
    dev = torch.device("cuda:0")
    S = A.scipy()
    rng = np.random.default_rng(seed)
    for tr in (False, True):
        nin, nout = (A.m, A.n) if tr else (A.n, A.m)
        xh = rng.standard_normal(nin)
        x = torch.from_numpy(xh).to(dev)
        y = torch.full((nout,), float("nan"), dtype=torch.float64, device=dev)
        plss.spmv_noalloc(h, M, x, y, transpose=tr)
        got = y.cpu().numpy()
        want = plss.spmv(h, M, xh, transpose=tr)
        np.testing.assert_array_equal(got, want)
        St = S.T if tr else S
        assert np.all(abs(got - St @ xh) <= 1e-14 * (abs(St) @ abs(xh)) + 1e-300)


@pytest.mark.parametrize("layout", ["stripes", "tiles"])
def test_noalloc_matches_spmv_two_calls(h, layout):
    import paper_2207_07615_amd as plss
    say("noalloc product", layout)
    big = gen.large(m=500_000, n=125_000).A        # row-blocked transpose (8 XCD blocks)
    small = gen.small(m=3000, n=1500).A
    Mb = matrix(h, big)
    Ms = matrix(h, small)
    on = layout == "stripes"
    Mb.layout(a_stripes=on, t_stripes=on)
    Ms.layout(a_stripes=on, t_stripes=on, unit_rows=64 if on else 0)
    products(h, Mb, big, 1)      # first call: the larger product
    products(h, Ms, small, 2)    # second call: smaller, on the array the first one left
    products(h, Mb, big, 3)


def test_noalloc_edge_cases(h):
    import torch
    import paper_2207_07615_amd as plss
    say("noalloc edges")
    dev = torch.device("cuda:0")
    # rows and columns without entries, a 1-column matrix
    A = gen.make_csr(gen.rng_for(14), 700, 1, np.r_[np.zeros(300, np.int64), np.ones(400, np.int64)], "normal")
    M = matrix(h, A)
    products(h, M, A, 4)
    A2 = gen.make_csr(gen.rng_for(15), 50, 400, np.r_[np.zeros(49, np.int64), [3]], "normal")
    products(h, matrix(h, A2), A2, 5)
    s = gen.small(m=400, n=200).A
    Ms = matrix(h, s)
    x = torch.zeros(200, dtype=torch.float64, device=dev)
    y = torch.zeros(400, dtype=torch.float64, device=dev)
    # host memory is refused (the entry point stages nothing)
    from paper_2207_07615_amd import _lib as L
    xh = np.zeros(200)
    yh = np.zeros(400)
    code = plss._clib().plss_spmv_noalloc(h.h, Ms.A, 0, xh.ctypes.data, yh.ctypes.data)
    assert code == L.PLSS_EINVAL
    # overlapping x and y are refused
    buf = torch.zeros(600, dtype=torch.float64, device=dev)
    code = plss._clib().plss_spmv_noalloc(h.h, Ms.A, 0, buf.data_ptr(), buf.data_ptr() + 8 * 100)
    assert code == L.PLSS_EINVAL
    assert b"overlap" in plss._clib().plss_last_error()
    plss.spmv_noalloc(h, Ms, x, y)
    assert not torch.any(y)


def test_noalloc_refuses_beyond_the_array(h):
    """A striped transposed product whose per-row-block partial vectors
    (8 blocks x 1,100,000 columns x 8 bytes = 70.4 MB) exceed the 64 MiB
    array is refused with the sizes in the message; plss_spmv still runs it."""
    import torch
    import paper_2207_07615_amd as plss
    from paper_2207_07615_amd import _lib as L
    say("noalloc limit")
    A = gen.make_csr(gen.rng_for(16), 400_000, 1_100_000, np.full(400_000, 2, dtype=np.int64), "normal")
    M = matrix(h, A)
    lay = M.layout(t_stripes=True)
    assert lay["t_stripes"]
    dev = torch.device("cuda:0")
    x = torch.zeros(A.m, dtype=torch.float64, device=dev)
    y = torch.zeros(A.n, dtype=torch.float64, device=dev)
    code = plss._clib().plss_spmv_noalloc(h.h, M.A, 1, x.data_ptr(), y.data_ptr())
    assert code == L.PLSS_EINVAL
    msg = plss._clib().plss_last_error().decode()
    say("  ", msg)
    assert "scratch" in msg and str(64 << 20) in msg
    # the direction that fits still runs
    xa = torch.from_numpy(np.random.default_rng(6).standard_normal(A.n)).to(dev)
    ya = torch.empty(A.m, dtype=torch.float64, device=dev)
    plss.spmv_noalloc(h, M, xa, ya)
    np.testing.assert_array_equal(ya.cpu().numpy(), plss.spmv(h, M, xa.cpu().numpy()))
