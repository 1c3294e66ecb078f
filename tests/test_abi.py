"""The C-ABI library loads and exports every function include/amg.h
declares; host-only calls validate their arguments (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2506_02663_amd", "libamg.so")


def declared():
    text = open(os.path.join(ROOT, "include", "amg.h")).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(amg_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for must in ("amg_create", "amg_finalize", "amg_solve", "amg_apply_operator", "amg_vcycle", "amg_destroy"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_argument_checks(lib):
    from paper_2506_02663_amd import amg as A
    h = ctypes.c_void_p()
    base = (ctypes.c_int32 * 2)(16, 16)
    L = A.lib()
    assert L.amg_create(4, base, 1.0 / 16, 2, 1, ctypes.byref(h)) == A.EINVAL   # bad dim
    assert L.amg_create(2, base, 1.0 / 16, 3, 1, ctypes.byref(h)) == A.EINVAL   # ratio
    assert L.amg_create(2, base, -1.0, 2, 1, ctypes.byref(h)) == A.EINVAL      # h0
    assert L.amg_create(2, base, 1.0 / 16, 2, 1, ctypes.byref(h)) == A.OK
    assert L.amg_set_operator(h, A.HELMHOLTZ, -1.0) == A.EINVAL
    assert b"c > 0" in L.amg_last_error(h)
    assert L.amg_set_physical_bc(h, 2, 0, A.DIRICHLET) == A.EINVAL          # d >= dim
    assert L.amg_set_cf_mode(h, 0, A.CF_NEUMANN) == A.EINVAL                 # level 0 has no interface
    assert L.amg_set_bottom_cells(h, -1) == A.EINVAL
    assert L.amg_set_bottom_cells(h, 1025) == A.EINVAL                      # host inverse O(n^3)
    assert L.amg_set_bottom_cells(h, 512) == A.OK
    assert L.amg_solve(h, 0, 0, None, None, None, None, None, None) == A.EINVAL  # not finalized
    assert b"finalize" in L.amg_last_error(h)
    assert L.amg_destroy(h) == A.OK
