"""The C-ABI library loads on the CPU and exports every symbol that
include/pintoc.h declares; host-side validation works without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pintoc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pintoc_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_2405_18964_amd as P
    try:
        return P.library()
    except P.LibraryMissing:
        from paper_2405_18964_amd.build import build
        build()
        P._lib._lib = None
        return P.library()


def test_every_declared_symbol_exported(lib):
    names = _declared()
    assert "pintoc_solve" in names and "pintoc_precond_apply" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_2405_18964_amd._lib import SIGNATURES
    assert set(_declared()) <= set(SIGNATURES)


def test_host_validation(lib):
    from paper_2405_18964_amd._lib import Desc, default_options
    o = default_options()
    h = ctypes.c_void_p()
    for bad in [Desc(3, 8, 1.0, 1.0, 1e-2, 0, None), Desc(4, 3, 1.0, 1.0, 1e-2, 0, None),
                Desc(4, 8, 0.0, 1.0, 1e-2, 0, None), Desc(4, 8, 1.0, 1.0, 0.0, 0, None)]:
        assert lib.pintoc_problem_create(ctypes.byref(bad), ctypes.byref(o), ctypes.byref(h)) == -1
        assert lib.pintoc_last_error()
    good = Desc(8, 16, 1.0, 1.0, 1e-2, 0, None)
    assert lib.pintoc_problem_create(ctypes.byref(good), ctypes.byref(o), ctypes.byref(h)) == 0
    assert lib.pintoc_vector_length(h) == 2 * 16 * (2 * 17 ** 2 + 9 ** 2)
    assert lib.pintoc_workspace_bytes(h) > 0
    assert lib.pintoc_bind_workspace(h, None, 0, None) == -1
    assert lib.pintoc_kkt_apply(h, None, None, None) < 0          # unbound: refused before any GPU call
    lib.pintoc_problem_destroy(h)
