"""The C-ABI library loads and exports every function include/plss.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "plss.h")
LIB = os.path.join(ROOT, "paper_2207_07615_amd", "libplss.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(plss_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("plss_create", "plss_matrix_create", "plss_solve", "plss_solve_batch",
              "plss_solve_multi", "plss_server_submit", "plss_server_poll"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libplss.so is not built (python -m paper_2207_07615_amd.build)")
    from paper_2207_07615_amd import _lib as L
    lib = L.load()
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_the_same_symbols():
    from paper_2207_07615_amd import _lib as L
    assert sorted(L.EXPORTS) == declared()


def test_status_strings_without_device():
    from paper_2207_07615_amd import _lib as L
    lib = L.load()
    assert lib.plss_status_string(0) == b"ok"
    assert lib.plss_status_string(-1) == b"invalid argument"
    o = L.plss_opts()
    lib.plss_opts_default(ctypes.byref(o))
    assert o.tol == 1e-8 and o.maxit == 1000 and o.sketch == 0
