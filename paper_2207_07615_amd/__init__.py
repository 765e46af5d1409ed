"""PLSS on AMD MI355X: Python binding of libplss.so (include/plss.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  Arrays may be NumPy arrays (host) or torch CUDA tensors (device);
results come back in the kind of the right-hand side.

    import paper_2207_07615_amd as plss
    h = plss.Handle(0)
    A = plss.Matrix(h, row_ptr, col_idx, values)           # CSR, uploads + builds the CSC copy
    x, info, hist = plss.solve(h, A, b, sketch="residual", tol=1e-8, maxit=1000)
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib as L

__all__ = ["Handle", "Matrix", "PlssError", "solve", "solve_batch", "solve_multi", "spmv",
           "Server", "kernel_times", "status_name"]


class PlssError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{status_name(code)} ({code}): {msg}")
        self.code = code


def _clib():
    return L.load()


def status_name(code: int) -> str:
    return _clib().plss_status_string(int(code)).decode()


def _check(code: int) -> int:
    if code < 0:
        raise PlssError(code, _clib().plss_last_error().decode())
    return code


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


class _Arr:
    """Pointer to a contiguous array of the wanted dtype (host or device)."""

    def __init__(self, a, dtype):
        self.keep = None
        if a is None:
            self.ptr = None
            self.torch = False
            return
        if _is_torch(a):
            import torch
            tdt = {np.float64: torch.float64, np.int64: torch.int64, np.int32: torch.int32,
                   np.float32: torch.float32}[dtype]
            t = a.detach().to(tdt).contiguous()
            if t.is_cuda:
                torch.cuda.current_stream(t.device).synchronize()
            self.keep = t
            self.ptr = t.data_ptr()
            self.torch = True
            self.device = t.device
        else:
            arr = np.ascontiguousarray(a, dtype=dtype)
            self.keep = arr
            self.ptr = arr.ctypes.data
            self.torch = False


def _out_like(ref: _Arr, shape, dtype=np.float64):
    if ref.torch:
        import torch
        t = torch.empty(shape, dtype=torch.float64, device=ref.device)
        return t, t.data_ptr()
    a = np.empty(shape, dtype=dtype)
    return a, a.ctypes.data


class Handle:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(_clib().plss_create(C.byref(h), int(device)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            _clib().plss_destroy(self.h)
            self.h = None

    def release_workspace(self):
        """Free the handle's grown scratch (plss_release_workspace)."""
        _check(_clib().plss_release_workspace(self.h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _csr_struct(m, n, row_ptr, col_idx, values):
    rp = _Arr(row_ptr, np.int64)
    ci = _Arr(col_idx, np.int32)
    va = _Arr(values, np.float64)
    nnz = int(row_ptr[-1]) if not _is_torch(row_ptr) else int(row_ptr[-1].item())
    s = L.plss_csr(int(m), int(n), nnz, rp.ptr, ci.ptr, va.ptr)
    return s, (rp, ci, va)


class Matrix:
    """Device store of A: CSR + CSC copy, in float64 or float32 storage."""

    def __init__(self, handle: Handle, row_ptr, col_idx, values, shape=None, storage="f64",
                 m: Optional[int] = None, n: Optional[int] = None):
        if shape is not None:
            m, n = shape
        if m is None:
            m = len(row_ptr) - 1
        if n is None:
            raise ValueError("n (or shape) is required")
        s, keep = _csr_struct(m, n, row_ptr, col_idx, values)
        out = C.c_void_p()
        _check(_clib().plss_matrix_create(handle.h, C.byref(s), L.DTYPE[storage], C.byref(out)))
        self.A = out
        self.handle = handle
        self.m, self.n, self.nnz = int(m), int(n), int(s.nnz)
        self.storage = storage

    @classmethod
    def from_csr(cls, handle, csr, storage="f64"):
        """From an object with m, n, row_ptr, col_idx, vals attributes."""
        return cls(handle, csr.row_ptr, csr.col_idx, csr.vals, shape=(csr.m, csr.n), storage=storage)

    def info(self):
        v = [C.c_int64() for _ in range(4)]
        _check(_clib().plss_matrix_info(self.A, *[C.byref(x) for x in v]))
        return {"m": v[0].value, "n": v[1].value, "nnz": v[2].value, "device_bytes": v[3].value}

    def csc(self):
        """(col_ptr int64[n+1], row_idx int32[nnz], values float64[nnz]) of the device CSC copy."""
        cp = np.empty(self.n + 1, np.int64)
        ri = np.empty(self.nnz, np.int32)
        va = np.empty(self.nnz, np.float64)
        _check(_clib().plss_matrix_csc(self.A, cp.ctypes.data, ri.ctypes.data, va.ctypes.data))
        return cp, ri, va

    def autotune(self):
        a, t = C.c_int32(), C.c_int32()
        _check(_clib().plss_matrix_autotune(self.handle.h, self.A, C.byref(a), C.byref(t)))
        return a.value, t.value

    def layout(self, a_stripes=None, t_stripes=None, unit_rows=0):
        """Read the product layout, or change it when a_stripes / t_stripes is
        given: {"a_stripes": bool, "t_stripes": bool, "unit_rows": int}."""
        got = L.plss_layout()
        if a_stripes is None and t_stripes is None:
            _check(_clib().plss_matrix_layout(self.handle.h, self.A, None, C.byref(got)))
        else:
            cur = self.layout()
            want = L.plss_layout(int(cur["a_stripes"] if a_stripes is None else bool(a_stripes)),
                                 int(cur["t_stripes"] if t_stripes is None else bool(t_stripes)),
                                 int(unit_rows))
            _check(_clib().plss_matrix_layout(self.handle.h, self.A, C.byref(want), C.byref(got)))
        return {"a_stripes": bool(got.a_stripes), "t_stripes": bool(got.t_stripes), "unit_rows": got.unit_rows}

    def close(self):
        if self.A:
            _clib().plss_matrix_destroy(self.A)
            self.A = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_opts(sketch="residual", tol=1e-8, maxit=1000, tol_absolute=False, refine=True,
              inner_tol=1e-4, max_outer=20, x0=None, wi=None, row_perm=None, hist_cap=0,
              chunk=0, timing=False, engine="auto", block=0, seed=0, keep=None):
    o = L.plss_opts()
    _clib().plss_opts_default(C.byref(o))
    o.sketch = L.SKETCH[sketch]
    o.tol = float(tol)
    o.maxit = int(maxit)
    o.tol_absolute = int(bool(tol_absolute))
    o.refine = int(bool(refine))
    o.inner_tol = float(inner_tol)
    o.max_outer = int(max_outer)
    keep = keep if keep is not None else []
    for name, arr, dt in (("x0", x0, np.float64), ("wi_diag", wi, np.float64),
                          ("row_perm", row_perm, np.int32)):
        if arr is not None:
            a = _Arr(arr, dt)
            keep.append(a)
            setattr(o, name, a.ptr)
    o.hist_cap = int(hist_cap)
    o.chunk = int(chunk)
    o.timing = int(bool(timing))
    o.engine = L.ENGINE[engine]
    o.block = int(block)
    o.seed = int(seed)
    return o, keep


def _info_dict(inf: L.plss_info):
    return {"iters": inf.iters, "outer_iters": inf.outer_iters, "relres": inf.relres,
            "relres_true": inf.relres_true, "status": inf.status,
            "status_name": status_name(inf.status), "ms": inf.ms}


def solve(handle: Handle, A: Matrix, b, hist_len: int = 0, **kw):
    """Solve A x = b.  Returns (x, info dict, residual history array of at
    most hist_len entries; default maxit + 2).  Keyword options are those of
    plss_opts (sketch, tol, maxit, refine, inner_tol, x0, wi, row_perm,
    hist_cap = identity/mixed history capacity, ...)."""
    bb = _Arr(b, np.float64)
    o, keep = make_opts(**kw)
    x, xp = _out_like(bb, (A.n,))
    hc = int(hist_len) if hist_len else int(min(kw.get("maxit", 1000) + 2, 1 << 20))
    hist = np.empty(hc, np.float64)
    inf = L.plss_info()
    _check(_clib().plss_solve(handle.h, A.A, bb.ptr, C.byref(o), xp, hist.ctypes.data, hc, C.byref(inf)))
    info = _info_dict(inf)
    nh = min(hc, info["iters"] + 1)
    return x, info, hist[:nh]


def solve_batch(handle: Handle, mats: Sequence[Matrix], bs: Sequence, **kw):
    """Solve many independent systems together.  Returns (list of x, list of info)."""
    ns = len(mats)
    keep = []
    barr = [_Arr(b, np.float64) for b in bs]
    opts = (L.plss_opts * ns)()
    for i in range(ns):
        o, keep = make_opts(keep=keep, **kw)
        opts[i] = o
    xs, xps = [], (C.c_void_p * ns)()
    for i in range(ns):
        x, xp = _out_like(barr[i], (mats[i].n,))
        xs.append(x)
        xps[i] = xp
    Aps = (C.c_void_p * ns)(*[m.A.value for m in mats])
    bps = (C.c_void_p * ns)(*[b.ptr for b in barr])
    infos = (L.plss_info * ns)()
    _check(_clib().plss_solve_batch(handle.h, ns, Aps, bps, opts, xps, infos))
    return xs, [_info_dict(infos[i]) for i in range(ns)]


def solve_multi(handle: Handle, A: Matrix, B, **kw):
    """Solve A X = B for the columns of B (m x nrhs).  Returns (X n x nrhs, infos)."""
    if _is_torch(B):
        nrhs = B.shape[1]
        Bc = B.t().contiguous()            # column-major m x nrhs
    else:
        B = np.asarray(B, dtype=np.float64)
        nrhs = B.shape[1]
        Bc = np.ascontiguousarray(B.T)
    bb = _Arr(Bc, np.float64)
    o, keep = make_opts(**kw)
    Xc, xp = _out_like(bb, (nrhs, A.n))
    infos = (L.plss_info * nrhs)()
    _check(_clib().plss_solve_multi(handle.h, A.A, nrhs, bb.ptr, C.byref(o), xp, infos))
    return Xc.T, [_info_dict(infos[i]) for i in range(nrhs)]


def spmv(handle: Handle, A: Matrix, x, transpose=False):
    xx = _Arr(x, np.float64)
    y, yp = _out_like(xx, (A.n if transpose else A.m,))
    _check(_clib().plss_spmv(handle.h, A.A, int(bool(transpose)), xx.ptr, yp))
    return y


def residual_pair(handle: Handle, A: Matrix, p, r):
    """r <- r - A p, then y = Aᵀ r with the updated r, in one pass over A
    (plss_residual_pair).  p and r: host arrays or device tensors (the
    caller's r is not modified).  Returns (r_new, y, rho, phi) with
    rho = ||r_new||² and phi = ||y||²; vectors are of r's kind."""
    pp = _Arr(p, np.float64)
    rr = _Arr(r, np.float64)
    if pp.keep.shape != (A.n,) or rr.keep.shape != (A.m,):
        raise ValueError(f"p must hold {A.n} and r {A.m} entries (one-dimensional)")
    if rr.torch:
        r_new = rr.keep.clone()
        rp = r_new.data_ptr()
    else:
        r_new = np.array(rr.keep, dtype=np.float64, copy=True)
        rp = r_new.ctypes.data
    y, yp = _out_like(rr, (A.n,))
    out = (C.c_double * 2)()
    _check(_clib().plss_residual_pair(handle.h, A.A, pp.ptr, rp, yp, out))
    return r_new, y, out[0], out[1]


def spmv_noalloc(handle: Handle, A: Matrix, x, y, transpose=False):
    """y <- A x (or Aᵀ x) through plss_spmv_noalloc: x and y are float64
    device tensors of the handle's GPU, y preallocated by the caller; the
    library allocates nothing.  Returns y."""
    if not (_is_torch(x) and _is_torch(y) and x.is_cuda and y.is_cuda):
        raise TypeError("spmv_noalloc takes device tensors (x, y)")
    import torch
    if x.dtype != torch.float64 or y.dtype != torch.float64 or not x.is_contiguous() or not y.is_contiguous():
        raise TypeError("x and y must be contiguous float64 tensors")
    nin, nout = (A.m, A.n) if transpose else (A.n, A.m)
    if x.numel() != nin or y.numel() != nout:
        raise ValueError(f"x must hold {nin} and y {nout} entries")
    torch.cuda.current_stream(x.device).synchronize()
    _check(_clib().plss_spmv_noalloc(handle.h, A.A, int(bool(transpose)), x.data_ptr(), y.data_ptr()))
    return y


def kernel_times(handle: Handle):
    """Accumulated per-kernel device ms and launch counts since the last call:
    [product with A, product with Aᵀ, step scalars, vector update]."""
    ms = (C.c_double * 4)()
    n = (C.c_int64 * 4)()
    _check(_clib().plss_kernel_times(handle.h, ms, n))
    return list(ms), list(n)


class Server:
    """Request loop with continuous batching (plss_server_*)."""

    def __init__(self, handle: Handle, hbm_budget_bytes: int, max_slots: int = 256):
        out = C.c_void_p()
        _check(_clib().plss_server_create(handle.h, int(hbm_budget_bytes), int(max_slots), C.byref(out)))
        self.s = out
        self._n = {}

    def submit(self, A_csr, b, storage="f64", **kw) -> int:
        s, keep = _csr_struct(A_csr.m, A_csr.n, A_csr.row_ptr, A_csr.col_idx, A_csr.vals)
        bb = _Arr(b, np.float64)
        o, keep2 = make_opts(**kw)
        req = C.c_uint64()
        _check(_clib().plss_server_submit(self.s, C.byref(s), L.DTYPE[storage], bb.ptr, C.byref(o),
                                         C.byref(req)))
        self._n[req.value] = A_csr.n
        return req.value

    def poll(self, req: int):
        """None while pending, else (x, info)."""
        x = np.empty(self._n[req], np.float64)
        inf = L.plss_info()
        code = _clib().plss_server_poll(self.s, C.c_uint64(req), x.ctypes.data, C.byref(inf))
        if code == L.PLSS_PENDING:
            return None
        _check(code)
        del self._n[req]
        return x, _info_dict(inf)

    def cancel(self, req: int):
        _check(_clib().plss_server_cancel(self.s, C.c_uint64(req)))

    def drain(self):
        _check(_clib().plss_server_drain(self.s))

    def stats(self):
        v = [C.c_int64() for _ in range(4)]
        _check(_clib().plss_server_stats(self.s, *[C.byref(x) for x in v]))
        return {"submitted": v[0].value, "finished": v[1].value, "active": v[2].value,
                "peak_bytes": v[3].value}

    def close(self):
        if self.s:
            _check(_clib().plss_server_destroy(self.s))
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
